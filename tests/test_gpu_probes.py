"""GPU checks of the bandwidth probes (libeik_probe.so): the copy copies, and the LDS read and
write streams return the checksums their access patterns define."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _xor4(words):
    out = np.zeros(words.shape[:-1], dtype=np.uint32)
    for c in range(4):
        out ^= words[..., c]
    return out


def test_copy_probe_copies():
    import torch
    from paper_1306_4743_amd import probes
    dev = torch.device("cuda:0")
    a = torch.arange(3 * 1024 * 1024 + 6, dtype=torch.float64, device=dev)  # ragged tail
    b = torch.zeros_like(a)
    ms = probes.copy(a, b, reps=2)
    assert ms > 0 and torch.equal(a, b)


@pytest.mark.parametrize("blocks,iters", [(1, 8), (3, 37), (512, 1000)])
def test_lds_probe_checksums(blocks, iters):
    import torch
    from paper_1306_4743_amd import probes
    dev = torch.device("cuda:0")
    out = torch.zeros(blocks * 256, dtype=torch.int32, device=dev)
    t = np.arange(256, dtype=np.uint32)
    # read: thread t reads word (t + 256 k) mod 2048 holding (j, 3j+1, 5j+2, 7j+3)
    ms, nb = probes.lds(out, blocks, iters, write=False, reps=2)
    assert ms > 0 and nb == blocks * 256 * iters * 16
    want = np.zeros(256, dtype=np.uint32)
    for k in range(iters):
        j = (t + 256 * k) % 2048
        want ^= _xor4(np.stack([j, 3 * j + 1, 5 * j + 2, 7 * j + 3], axis=-1).astype(np.uint32))
    got = out.cpu().numpy().view(np.uint32).reshape(blocks, 256)
    assert np.array_equal(got, np.broadcast_to(want, got.shape))
    # write: word t + 256 m ends with the last iteration k = m (mod 8): (t + k, k, t, 1)
    probes.lds(out, blocks, iters, write=True, reps=2)
    want = np.zeros(256, dtype=np.uint32)
    for m in range(8):
        k = m + 8 * ((iters - 1 - m) // 8)
        want ^= _xor4(np.stack([t + k, np.full(256, k), t, np.ones(256)], axis=-1)
                      .astype(np.uint32))
    got = out.cpu().numpy().view(np.uint32).reshape(blocks, 256)
    assert np.array_equal(got, np.broadcast_to(want, got.shape))
