"""eik_solve_noalloc -- the entry point that allocates nothing (its workspace is the library's
static device scratch) -- against eik_solve_ex, the entry point whose kernels it shares, on the
same inputs through the C ABI: identical +inf masks, exits equal to q, and values within the
FP64 bar (1e-10 relative) of eik_solve_ex's and of the oracle's.  Two calls in a row, the
second on a smaller grid, whose result must not depend on what the first left in the scratch."""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1306_4743_amd import eik
    eik.load()
    return torch.device("cuda:0")


def compare(got, want, p):
    assert np.array_equal(np.isinf(got), np.isinf(want)), "+inf masks differ"
    assert not np.any(np.isnan(got))
    s = p.src
    assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], p.q)
    fin = np.isfinite(want) & (want > 0)
    rel = float(np.max(np.abs(got[fin] - want[fin]) / want[fin]))
    assert rel <= REL_TOL, rel
    return rel


@pytest.mark.parametrize("cell", [8, 4, 16])
def test_two_calls_match_solve_ex(orc, dev, cell):
    import torch
    from paper_1306_4743_amd import eik
    ps = [W.maze(129, seed=3), W.oscillatory(49, periods=3)]   # the second is smaller
    Fs = [torch.from_numpy(np.ascontiguousarray(p.F)).to(dev) for p in ps]
    refs = []
    for p, F in zip(ps, Fs):
        u = eik.solve(F, p.h, p.src, p.q, cell=cell)             # eik_solve_ex
        assert eik.status()[0] == 0
        refs.append(u.cpu().numpy())
    outs = [torch.full(F.shape, -1.0, dtype=torch.float64, device=dev) for F in Fs]
    for p, F, u in zip(ps, Fs, outs):                            # two calls in a row
        assert eik.solve_noalloc(F, p.h, p.src, p.q, cell=cell, u_out=u) == eik.EIK_OK
        rc, st = eik.status()
        assert rc == 0 and st["visits"] > 0
    for p, u, ref in zip(ps, outs, refs):
        got = u.cpu().numpy()
        e1 = compare(got, ref, p)
        e2 = compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
        print(f"noalloc {p.name} r {cell}: vs eik_solve_ex {e1:.2e}, vs oracle {e2:.2e}",
              flush=True)


def test_mixed_mode_device_exits_and_release(orc, dev):
    """EIK_MODE_MIXED (FP32 twins in the scratch, the polish and its check), exits given in
    device memory, and a call after eik_release (which makes the next call set up again)."""
    import torch
    from paper_1306_4743_amd import eik
    p = W.maze(97, seed=5, n_sources=3)
    F = torch.from_numpy(p.F).to(dev)
    want = orc.fmm(p.F, p.h, p.src, p.q)
    ref = eik.solve(F, p.h, p.src, p.q, cell=8, mode=eik.EIK_MODE_MIXED)
    assert eik.status()[0] == 0
    u = torch.empty_like(ref)
    assert eik.solve_noalloc(F, p.h, torch.from_numpy(p.src).to(dev),
                             torch.from_numpy(p.q).to(dev), cell=8, u_out=u,
                             mode=eik.EIK_MODE_MIXED) == eik.EIK_OK
    rc, st = eik.status()
    assert rc == 0 and st["polish_redone"] == 0
    compare(u.cpu().numpy(), ref.cpu().numpy(), p)
    compare(u.cpu().numpy(), want, p)
    torch.cuda.synchronize()
    eik.release()
    u2 = torch.empty_like(ref)
    assert eik.solve_noalloc(F, p.h, p.src, p.q, cell=8, u_out=u2) == eik.EIK_OK
    assert eik.status()[0] == 0
    compare(u2.cpu().numpy(), want, p)


def test_limits_refused_before_any_work(dev):
    import torch
    from paper_1306_4743_amd import eik
    big = torch.ones((300, 300, 300), dtype=torch.float32, device=dev)
    u = torch.empty(big.shape, dtype=torch.float64, device=dev)
    src = np.array([[1, 2, 3]])
    assert eik.solve_noalloc(big, 1 / 299, src, np.zeros(1), cell=8, u_out=u,
                             check=False) == eik.EIK_ETOOBIG
    del big, u
    F = torch.ones((33, 33, 33), dtype=torch.float32, device=dev)
    u = torch.empty(F.shape, dtype=torch.float64, device=dev)
    many = np.array([[i, i, i] for i in range(33)])
    assert eik.solve_noalloc(F, 1 / 32, many, np.zeros(33), cell=8, u_out=u,
                             check=False) == eik.EIK_EINVAL
    assert eik.solve_noalloc(F, 1 / 32, many[:32], np.zeros(32), cell=8, u_out=u,
                             timing=True, check=False) == eik.EIK_EINVAL
    assert eik.solve_noalloc(F, 1 / 32, many[:32], np.zeros(32), cell=8, u_out=u) == eik.EIK_OK
    assert eik.status()[0] == 0
    got = u.cpu().numpy()
    assert np.all(got[np.arange(32), np.arange(32), np.arange(32)] == 0.0)
    assert np.all(np.isfinite(got))
