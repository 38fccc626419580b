"""GPU parity at cells of 16 nodes per side against the serial FP64 oracle.

At r = 16 a diagonal plane of the cell holds up to 192 nodes, so a sweep takes each plane in up
to three 64-node wave steps (88 steps instead of 46 planes), a lane stages four nodes of each
face, and a CU holds two FP64 (four FP32) cell workers.  The discrete solution does not depend
on the cell size (Section 4), so every case must give the oracle's values: same +inf mask,
exits exact, max relative error <= 1e-10 in FP64.
"""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-10
INNERS = [1, 2]  # EIK_INNER_SWEEP, EIK_INNER_LIST (two sweep streams stop at r = 8)


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1306_4743_amd import eik
    eik.load()
    return torch.device("cuda:0")


def solve16(dev, p, **kw):
    import torch
    from paper_1306_4743_amd import eik
    F = torch.from_numpy(np.ascontiguousarray(p.F)).to(dev)
    u = eik.solve(F, p.h, p.src, p.q, cell=16, tol=kw.pop("tol", 0.0), **kw)
    rc, stats = eik.status()
    return u.cpu().numpy(), rc, stats


def compare(got, want, p, tol=REL_TOL, exact_exits=True):
    assert np.array_equal(np.isinf(got), np.isinf(want)), "+inf masks differ"
    assert not np.any(np.isnan(got))
    s = p.src
    if len(s) and exact_exits:
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], want[s[:, 2], s[:, 1], s[:, 0]])
    fin = np.isfinite(want) & (want > 0)
    if not fin.any():
        return 0.0
    rel = np.abs(got[fin] - want[fin]) / want[fin]
    worst = float(rel.max())
    assert worst <= tol, f"max rel err {worst:.3e}"
    return worst


def check(orc, dev, p, **kw):
    got, rc, stats = solve16(dev, p, **kw)
    assert rc == 0, stats
    err = compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
    print(f"r=16 {p.name} {kw}: max rel err {err:.2e}, stats {stats}", flush=True)
    return got, stats


@pytest.mark.parametrize("inner", INNERS)
def test_constant_small(orc, dev, inner):
    """65^3, F = 1, centre source: 5 cells per axis, the last one node thick; axis values
    k h exactly."""
    p = W.constant(65, cell=16, tol=1e-14)
    got, stats = check(orc, dev, p, inner=inner, tol=1e-14)
    c = 32
    assert np.array_equal(got[c, c, :], np.abs(np.arange(-c, c + 1)) * p.h)
    assert stats["cells"] == 125 and stats["visits"] >= 100


@pytest.mark.parametrize("inner", INNERS)
@pytest.mark.parametrize("seed", range(6))
def test_random_small(orc, dev, seed, inner):
    """Random speeds, several sources, sizes from 2 to 40 per axis: single partial cells and
    ragged last cells."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(9, 40))
    p = W.random_small(n, seed, n_sources=int(rng.integers(1, 5)), nx=int(rng.integers(2, 40)),
                       ny=int(rng.integers(2, 25)))
    check(orc, dev, p, inner=inner)


@pytest.mark.parametrize("inner", INNERS)
def test_oscillatory(orc, dev, inner):
    check(orc, dev, W.oscillatory(97, periods=4), inner=inner)


@pytest.mark.parametrize("inner", INNERS)
@pytest.mark.parametrize("case", ["corner", "faces", "tiny", "thin", "plane"])
def test_edge_cases(orc, dev, case, inner):
    rng = np.random.default_rng(7)
    if case == "corner":
        n = 33
        p = W.Problem("corner", rng.uniform(0.5, 2, (n, n, n)), 1 / (n - 1),
                      np.array([[0, 0, 0], [n - 1, n - 1, n - 1]]), np.array([0.0, 0.3]))
    elif case == "faces":      # exits on r = 16 cell faces, edges and corners
        n = 41
        src = np.array([[16, 20, 20], [15, 16, 3], [16, 16, 16], [31, 32, 31], [39, 23, 24]])
        p = W.Problem("faces", rng.uniform(0.5, 2, (n, n, n)), 1 / (n - 1), src,
                      rng.uniform(0, 0.05, 5))
    elif case == "tiny":
        p = W.Problem("tiny", np.ones((2, 2, 2)), 0.5, np.array([[0, 0, 0]]), np.array([0.0]))
    elif case == "thin":
        p = W.Problem("thin", rng.uniform(0.2, 2, (3, 70, 2)), 1 / 69, np.array([[1, 0, 2]]),
                      np.array([0.0]))
    else:                      # a plane of exits: the 1D reduction, exact
        n = 40
        src = np.array([[0, j, k] for k in range(n) for j in range(n)])
        fx = 2.0 ** rng.integers(-2, 3, size=n)
        F = np.broadcast_to(fx[None, None, :], (n, n, n)).copy()
        p = W.Problem("plane", F, 1 / 32, src, np.zeros(len(src)))
    got, _ = check(orc, dev, p, inner=inner)
    if case == "plane":
        want = np.concatenate([[0.0], np.cumsum(p.h / fx[1:])])
        assert np.array_equal(got[3, 7, :], want)


@pytest.mark.parametrize("inner", INNERS)
@pytest.mark.parametrize("delta", [0.0, 0.02, 0.5])
def test_maze_priority_bands(orc, dev, delta, inner):
    check(orc, dev, W.maze(97, seed=3), delta=delta, inner=inner)


@pytest.mark.parametrize("shuffle", [1, 2])
def test_processing_order_invariance(orc, dev, shuffle):
    check(orc, dev, W.oscillatory(65, periods=4), shuffle=shuffle)


@pytest.mark.parametrize("cap", [1, 3])
def test_sweep_cap_requeues(orc, dev, cap):
    _, stats = check(orc, dev, W.oscillatory(49, periods=3), max_sweeps=cap)
    assert stats["requeued"] > 0


@pytest.mark.parametrize("inner", INNERS)
def test_fp32_and_mixed_modes(orc, dev, inner):
    """FP32 values within the single-precision bound (4 n 2^-24); the FP32 bulk with FP64
    polish at the FP64 bar; an FP32 result polished through u_approx at the FP64 bar."""
    import torch
    from paper_1306_4743_amd import eik
    for p in (W.maze(97, seed=3), W.oscillatory(65, periods=3)):
        want = orc.fmm(p.F, p.h, p.src, p.q)
        got, rc, _ = solve16(dev, p, inner=inner, mode=eik.EIK_MODE_FP32)
        assert rc == 0
        compare(got, want, p, tol=4.0 * max(p.dims) * 2.0 ** -24, exact_exits=False)
        got, rc, _ = solve16(dev, p, inner=inner, mode=eik.EIK_MODE_MIXED)
        assert rc == 0
        compare(got, want, p)
        F = torch.from_numpy(np.ascontiguousarray(p.F)).to(dev)
        u = eik.solve(F, p.h, p.src, p.q, cell=16, inner=inner, mode=eik.EIK_MODE_FP32)
        assert eik.status()[0] == 0
        u = eik.solve(F, p.h, p.src, p.q, cell=16, inner=inner, u_out=u, u_approx=u)
        assert eik.status()[0] == 0
        compare(u.cpu().numpy(), want, p)


def test_eq9_cell_values(orc, dev):
    from paper_1306_4743_amd import eik
    for p in (W.shell_maze(65), W.maze(97, seed=3)):
        check(orc, dev, p, delta=4.0 * 16 * p.h, cell_value=eik.EIK_CELL_VALUE_OLD)


def test_batch_and_server_match_alone(orc, dev):
    """Uneven grids in one batch launch and through a server with room for two at a time: each
    result equals the oracle's."""
    import torch
    from paper_1306_4743_amd import eik
    ps = [W.maze(49, seed=21, n_sources=2), W.random_small(19, 7, n_sources=3, nx=37, ny=11),
          W.oscillatory(33, periods=2)]
    for p in ps:
        p.F = p.F.astype(np.float32)
    wants = [orc.fmm(p.F, p.h, p.src, p.q) for p in ps]
    Fs = [torch.from_numpy(np.ascontiguousarray(p.F)).to(dev) for p in ps]
    outs = eik.solve_batch([dict(F=F, h=p.h, src=p.src, q=p.q) for F, p in zip(Fs, ps)], cell=16,
                           delta=0.05)
    assert list(eik.batch_status(len(ps))) == [0, 0, 0]
    for p, u, w in zip(ps, outs, wants):
        compare(u.cpu().numpy(), w, p)
    srv = eik.Server(pool_bytes=1 << 28, max_cells=4096, max_problems=2, cell=16,
                     f_dtype=eik.EIK_F32)
    try:
        pending = list(range(len(ps)))
        done = {}
        for _ in range(2000):
            while pending:
                i = pending[0]
                if srv.submit(Fs[i], ps[i].h, ps[i].src, ps[i].q) is None:
                    break
                pending.pop(0)
            done.update(srv.step(8))
            if len(done) == len(ps):
                break
        assert sorted(done) == [0, 1, 2]
        for t, (st, u) in done.items():
            assert st == 0
            compare(u.cpu().numpy(), wants[t], ps[t])
    finally:
        srv.close()


def test_oscillatory_257_full(orc, dev):
    """The oscillatory workload at its full size (257^3, 4 periods) with cells of 16."""
    p = W.oscillatory(257, periods=4)
    want = orc.fmm(p.F, p.h, p.src, p.q)
    for inner in INNERS:
        got, rc, stats = solve16(dev, p, inner=inner)
        assert rc == 0
        err = compare(got, want, p)
        print(f"257^3 cell 16 inner {inner}: max rel err {err:.2e} {stats}", flush=True)
