"""The check after every FP64 polish (EIK_MODE_MIXED, eik_problem.u_approx): a start that lies
below the solution somewhere cannot be raised by the method's updates (values only decrease),
so the polished result would be wrong there; the eq. (2) check finds the grid and it is solved
again from +inf.  Every result below is compared with the oracle at the FP64 bar, and the
re-solve counters must say exactly which grids were redone (Section 6, "single precision":
the precision of the data; Section 4: the discrete solution is unique, so a grid whose every
node satisfies eq. (2) holds it)."""
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
    s = p.src
    assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], p.q)
    fin = np.isfinite(want) & (want > 0)
    rel = float(np.max(np.abs(got[fin] - want[fin]) / want[fin]))
    assert rel <= REL_TOL, rel
    return rel


def low_block(want):
    """The solution with one block of nodes 10% below it (everything else exact)."""
    start = want.copy()
    start[20:40, 10:30, 30:50] *= 0.9
    return start


@pytest.mark.parametrize("cell", [8, 4])
def test_start_below_solution_is_solved_again(orc, dev, cell):
    import torch
    from paper_1306_4743_amd import eik
    p = W.maze(65, seed=8, n_sources=2)
    want = orc.fmm(p.F, p.h, p.src, p.q)
    F = torch.from_numpy(p.F).to(dev)
    for name, start in (("block 10% low", low_block(want)), ("zeros", np.zeros_like(want)),
                        ("0.999 U", 0.999 * want)):
        ua = torch.from_numpy(np.ascontiguousarray(start)).to(dev)
        u = eik.solve(F, p.h, p.src, p.q, cell=cell, u_approx=ua)
        rc, st = eik.status()
        assert rc == 0
        err = compare(u.cpu().numpy(), want, p)
        print(f"{name}: redone {st['polish_redone']}, max rel err {err:.2e}", flush=True)
        assert st["polish_redone"] == 1


def test_good_polishes_are_not_redone(orc, dev):
    """An FP32 result (the normal input) and an upper bound pass the check."""
    import torch
    from paper_1306_4743_amd import eik
    p = W.maze(97, seed=3)
    want = orc.fmm(p.F, p.h, p.src, p.q)
    F = torch.from_numpy(p.F).to(dev)
    u = eik.solve(F, p.h, p.src, p.q, cell=8, mode=eik.EIK_MODE_MIXED)
    rc, st = eik.status()
    assert rc == 0 and st["polish_redone"] == 0
    compare(u.cpu().numpy(), want, p)
    u32 = eik.solve(F, p.h, p.src, p.q, cell=8, mode=eik.EIK_MODE_FP32)
    assert eik.status()[0] == 0
    u = eik.solve(F, p.h, p.src, p.q, cell=8, u_approx=u32)
    rc, st = eik.status()
    assert rc == 0 and st["polish_redone"] == 0
    compare(u.cpu().numpy(), want, p)
    ub = torch.from_numpy(np.where(np.isfinite(want), 1.2 * want + 0.01, np.inf)).to(dev)
    u = eik.solve(F, p.h, p.src, p.q, cell=8, u_approx=ub)
    rc, st = eik.status()
    assert rc == 0 and st["polish_redone"] == 0
    compare(u.cpu().numpy(), want, p)


def test_batch_redoes_only_the_bad_grid(orc, dev):
    import torch
    from paper_1306_4743_amd import eik
    ps = [W.maze(65, seed=8, n_sources=2), W.oscillatory(49, periods=3, dtype=np.float32),
          W.random_small(23, 4, n_sources=3, nx=31, ny=17)]
    for p in ps:
        p.F = p.F.astype(np.float32)
    wants = [orc.fmm(p.F, p.h, p.src, p.q) for p in ps]
    starts = [low_block(wants[0]), np.where(np.isfinite(wants[1]), 1.1 * wants[1], np.inf), None]
    probs = []
    for p, s0 in zip(ps, starts):
        d = dict(F=torch.from_numpy(p.F).to(dev), h=p.h, src=p.src, q=p.q)
        if s0 is not None:
            d["u_approx"] = torch.from_numpy(np.ascontiguousarray(s0)).to(dev)
        probs.append(d)
    outs = eik.solve_batch(probs, cell=8)
    assert list(eik.batch_status(len(ps))) == [0, 0, 0]
    rc, st = eik.status()
    assert rc == 0 and st["polish_redone"] == 1
    for p, u, want in zip(ps, outs, wants):
        compare(u.cpu().numpy(), want, p)


def test_server_restarts_a_bad_polish(orc, dev):
    """Through a server: the polish with a too-low start is restarted at the step that would
    have retired it and finishes later with the oracle's values; the good one is not."""
    import torch
    from paper_1306_4743_amd import eik
    pa, pb = W.maze(65, seed=8, n_sources=2), W.maze(49, seed=4, n_sources=3)
    wa, wb = orc.fmm(pa.F, pa.h, pa.src, pa.q), orc.fmm(pb.F, pb.h, pb.src, pb.q)
    srv = eik.Server(1 << 28, 20000, 4, cell=8)
    try:
        Fa, Fb = torch.from_numpy(pa.F).to(dev), torch.from_numpy(pb.F).to(dev)
        ta = srv.submit(Fa, pa.h, pa.src, pa.q,
                        u_approx=torch.from_numpy(low_block(wa)).to(dev))
        tb = srv.submit(Fb, pb.h, pb.src, pb.q,
                        u_approx=torch.from_numpy(np.where(np.isfinite(wb), 1.3 * wb, np.inf)).to(dev))
        got = {}
        for _ in range(2000):
            for t, (stt, u) in srv.step(8).items():
                assert stt == 0
                got[t] = u.cpu().numpy()
            if len(got) == 2:
                break
        assert srv.polish_redone() == 1
        compare(got[ta], wa, pa)
        compare(got[tb], wb, pb)
    finally:
        srv.close()
