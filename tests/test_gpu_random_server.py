"""A seeded random stream through the continuous-batching server: random grid extents, speeds,
exits and arrival order, some requests solved from scratch and some polished from an FP32
result (``u_approx``), a pool that holds only a few grids at a time and random rounds per step.
Every result must be the oracle's (same +inf mask, exits exact, relative error <= 1e-10): a
grid's solution does not depend on the grids it shares the device with (Section 4)."""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu


def draw_problem(rng, k):
    nx, ny, nz = (int(v) for v in rng.integers(2, 33, size=3))
    F = rng.uniform(0.2, 2.0, size=(nz, ny, nx)).astype(np.float32)
    ns = int(rng.integers(1, 5))
    src = {(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(ns)}
    src = np.array(sorted(src), dtype=np.int64)
    q = rng.uniform(0.0, 0.1, size=len(src))
    return W.Problem(f"server{k}", F, float(rng.choice([1 / 16, 0.1])), src, q, 8, 0.0, {})


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_stream_through_server(orc, seed):
    import torch
    from paper_1306_4743_amd import eik
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(90_000 + seed)
    ps = [draw_problem(rng, k) for k in range(24)]
    polish = rng.integers(0, 2, size=len(ps)).astype(bool)
    Fs = [torch.from_numpy(p.F).to(dev) for p in ps]
    approx = {}
    for k, p in enumerate(ps):
        if polish[k]:
            approx[k] = eik.solve(Fs[k], p.h, p.src, p.q, cell=8, mode=eik.EIK_MODE_FP32)
            assert eik.status()[0] == 0
    big = max(eik.problem_bytes(p.F.shape[::-1], 8, eik.EIK_F32) for p in ps)
    srv = eik.Server(pool_bytes=3 * big, max_cells=1 << 14, max_problems=4, cell=8)
    pending = list(rng.permutation(len(ps)))
    tickets, done, steps = {}, {}, 0
    while pending or len(done) < len(ps):
        while pending:
            k = int(pending[0])
            t = srv.submit(Fs[k], ps[k].h, ps[k].src, ps[k].q, 0.0, approx.get(k),
                           u_approx=approx.get(k))
            if t is None:
                break
            tickets[t] = k
            pending.pop(0)
        for t, (status, u) in srv.step(int(rng.integers(1, 20))).items():
            assert status == 0
            done[tickets[t]] = u
        steps += 1
        assert steps < 10_000, "server did not drain"
    srv.close()
    for k, p in enumerate(ps):
        got = done[k].cpu().numpy()
        want = orc.fmm(p.F, p.h, p.src, p.q)
        assert np.array_equal(np.isinf(got), np.isinf(want)), k
        s = p.src
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], want[s[:, 2], s[:, 1], s[:, 0]]), k
        fin = np.isfinite(want) & (want > 0)
        if fin.any():
            assert float(np.max(np.abs(got[fin] - want[fin]) / want[fin])) <= 1e-10, k
