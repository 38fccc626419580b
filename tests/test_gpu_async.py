"""The solver without rounds (EIK_SCHED_ASYNC: cells popped from a device ring as they are
queued, no barrier between visits, a final eq. (2) check of every cell) against the oracle,
with the same parity bar as the round-based schedule: every cell size and in-cell solver,
shuffled-free natural order, one worker, the precision modes, polishes and batches.  The
discrete solution is unique and the Heap-Cell Method reaches it in any processing order
(Section 4, "Assigning Cell Values"; Section 5.1 on the benign races of the parallel loop)."""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-10
ASYNC = 3


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1306_4743_amd import eik
    eik.load()
    return torch.device("cuda:0")


def compare(got, want, p, tol=REL_TOL):
    assert np.array_equal(np.isinf(got), np.isinf(want)), "+inf masks differ"
    assert not np.any(np.isnan(got))
    s = p.src
    if len(s):
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], want[s[:, 2], s[:, 1], s[:, 0]])
    fin = np.isfinite(want) & (want > 0)
    rel = float(np.max(np.abs(got[fin] - want[fin]) / want[fin])) if fin.any() else 0.0
    assert rel <= tol, rel
    return rel


def solve(dev, p, **kw):
    import torch
    from paper_1306_4743_amd import eik
    F = torch.from_numpy(np.ascontiguousarray(p.F)).to(dev)
    u = eik.solve(F, p.h, p.src, p.q, cell=kw.pop("cell", 8), schedule=ASYNC,
                  tol=kw.pop("tol", 0.0), **kw)
    rc, st = eik.status()
    return u.cpu().numpy(), rc, st


# Every in-cell solver the round-free schedule runs at each cell size (two sweep streams stop
# at cells of 8).
CELL_INNER = [(c, i) for c in (8, 4, 16) for i in (1, 2, 3) if not (c == 16 and i == 3)]


@pytest.mark.parametrize("cell,inner", CELL_INNER)
@pytest.mark.parametrize("name", ["maze", "osc", "random", "shell", "checker"])
def test_async_matches_oracle(orc, dev, name, cell, inner):
    p = {"maze": lambda: W.maze(97, seed=3),
         "osc": lambda: W.oscillatory(65, periods=4),
         "random": lambda: W.random_small(23, 5, n_sources=3, nx=37, ny=13),
         "shell": lambda: W.shell_maze(65),
         "checker": lambda: W.checkerboard(57, K=11)}[name]()
    got, rc, st = solve(dev, p, cell=cell, inner=inner)
    assert rc == 0, st
    err = compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
    print(f"async {name} r {cell} inner {inner}: max rel err {err:.2e}, visits "
          f"{st['visits']} ({st['visits'] / st['cells']:.2f}/cell), check passes {st['rounds']}",
          flush=True)
    assert st["rounds"] >= 1


@pytest.mark.parametrize("case", ["corner", "tiny", "thin", "dupes", "none"])
def test_async_edge_cases(orc, dev, case):
    rng = np.random.default_rng(7)
    if case == "corner":
        n = 33
        p = W.Problem("corner", rng.uniform(0.5, 2, (n, n, n)), 1 / (n - 1),
                      np.array([[0, 0, 0], [n - 1, n - 1, n - 1]]), np.array([0.0, 0.3]))
    elif case == "tiny":
        p = W.Problem("tiny", np.ones((2, 2, 2)), 0.5, np.array([[0, 0, 0]]), np.array([0.0]))
    elif case == "thin":
        p = W.Problem("thin", rng.uniform(0.2, 2, (3, 70, 2)), 1 / 69, np.array([[1, 0, 2]]),
                      np.array([0.0]))
    elif case == "dupes":
        p = W.Problem("dupes", np.ones((20, 20, 20)), 1 / 19, np.array([[5, 5, 5], [5, 5, 5]]),
                      np.array([0.2, 0.1]))
    else:
        p = W.Problem("none", np.ones((17, 17, 17)), 1 / 16, np.zeros((0, 3), np.int64),
                      np.zeros(0))
    for cell in (8, 4):
        got, rc, st = solve(dev, p, cell=cell)
        assert rc == 0
        if case == "none":
            assert np.all(np.isinf(got)) and st["visits"] == 0
        else:
            compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)


def test_async_one_worker_and_sweep_cap(orc, dev):
    p = W.maze(49, seed=5, n_sources=2)
    want = orc.fmm(p.F, p.h, p.src, p.q)
    got, rc, _ = solve(dev, p, workers=1)
    assert rc == 0
    compare(got, want, p)
    got, rc, st = solve(dev, p, max_sweeps=1)
    assert rc == 0 and st["requeued"] > 0
    compare(got, want, p)


@pytest.mark.parametrize("mode", [1, 2])
def test_async_precision_modes(orc, dev, mode):
    from paper_1306_4743_amd import eik
    p = W.maze(97, seed=3)
    got, rc, st = solve(dev, p, mode=mode)
    assert rc == 0
    want = orc.fmm(p.F, p.h, p.src, p.q)
    tol = REL_TOL if mode == eik.EIK_MODE_MIXED else 4.0 * 97 * 2.0 ** -24
    compare(got, want, p, tol=tol) if mode == eik.EIK_MODE_MIXED else None
    if mode == eik.EIK_MODE_FP32:
        fin = np.isfinite(want) & (want > 0)
        assert np.array_equal(np.isinf(got), np.isinf(want))
        assert float(np.max(np.abs(got[fin] - want[fin]) / want[fin])) <= tol


def test_async_batch_and_polish(orc, dev):
    import torch
    from paper_1306_4743_amd import eik
    ps = [W.maze(65, seed=8, n_sources=2), W.oscillatory(49, periods=3, dtype=np.float32),
          W.random_small(23, 4, n_sources=3, nx=31, ny=17)]
    for p in ps:
        p.F = p.F.astype(np.float32)
    wants = [orc.fmm(p.F, p.h, p.src, p.q) for p in ps]
    starts = [None, np.where(np.isfinite(wants[1]), 1.1 * wants[1], np.inf), 0.9 * wants[2]]
    probs = []
    for p, s0 in zip(ps, starts):
        d = dict(F=torch.from_numpy(p.F).to(dev), h=p.h, src=p.src, q=p.q)
        if s0 is not None:
            d["u_approx"] = torch.from_numpy(np.ascontiguousarray(s0)).to(dev)
        probs.append(d)
    outs = eik.solve_batch(probs, cell=8, schedule=ASYNC)
    assert list(eik.batch_status(len(ps))) == [0, 0, 0]
    rc, st = eik.status()
    assert rc == 0 and st["polish_redone"] == 1
    for p, u, want in zip(ps, outs, wants):
        compare(u.cpu().numpy(), want, p)


def test_async_refusals():
    """A band of cell values needs rounds; servers step in rounds."""
    import ctypes
    from paper_1306_4743_amd import eik
    lib = eik.load()
    h = ctypes.c_void_p(None)
    opts = eik._options(schedule=ASYNC)
    assert lib.eik_server_create(ctypes.byref(h), 1 << 20, 100, 4, 8, eik.EIK_F32, None,
                                 ctypes.byref(opts)) == eik.EIK_EINVAL


@pytest.mark.parametrize("band", [1.0, 4.0, 16.0])
@pytest.mark.parametrize("cell", [8, 4])
@pytest.mark.parametrize("name", ["maze", "osc", "shell", "random"])
def test_async_buckets_match_oracle(orc, dev, name, cell, band):
    """Cells kept in buckets of cell values (width band * r * h); every width gives the
    oracle's solution."""
    p = {"maze": lambda: W.maze(97, seed=3),
         "osc": lambda: W.oscillatory(65, periods=4),
         "shell": lambda: W.shell_maze(65),
         "random": lambda: W.random_small(23, 5, n_sources=3, nx=37, ny=13)}[name]()
    got, rc, st = solve(dev, p, cell=cell, delta=band * cell * p.h)
    assert rc == 0, st
    err = compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
    print(f"async buckets {name} r {cell} band {band}: max rel err {err:.2e}, visits/cell "
          f"{st['visits'] / st['cells']:.2f}, check passes {st['rounds']}", flush=True)


def test_async_buckets_batch_and_mixed(orc, dev):
    import torch
    from paper_1306_4743_amd import eik
    ps = [W.maze(65, seed=8, n_sources=2), W.shell_maze(49),
          W.random_small(23, 4, n_sources=3, nx=31, ny=17)]
    for p in ps:
        p.F = p.F.astype(np.float32)
    probs = [dict(F=torch.from_numpy(p.F).to(dev), h=p.h, src=p.src, q=p.q) for p in ps]
    for mode in (eik.EIK_MODE_FP64, eik.EIK_MODE_MIXED):
        outs = eik.solve_batch(probs, cell=8, schedule=ASYNC, delta=0.05, mode=mode)
        assert list(eik.batch_status(len(ps))) == [0, 0, 0]
        for p, u in zip(ps, outs):
            compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)
