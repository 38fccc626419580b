"""GPU parity of batched solves and of the continuous-batching server (through the C ABI).

Every grid of a batch or of a server is an independent instance of eq. (2); its discrete
solution does not depend on which other grids share the launch, nor on the processing order
(Section 4).  So each grid is compared with the oracle's FMM node by node (identical +inf masks,
exact exits, max relative error <= 1e-10) and with the same grid solved alone.
"""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1306_4743_amd import eik
    eik.load()
    return torch.device("cuda:0")


def compare(got, want, p, tol=REL_TOL):
    assert got.shape == want.shape
    assert np.array_equal(np.isinf(got), np.isinf(want)), "+inf masks differ"
    assert not np.any(np.isnan(got))
    s = p.src
    if len(s):
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], want[s[:, 2], s[:, 1], s[:, 0]])
    fin = np.isfinite(want) & (want > 0)
    if not fin.any():
        return 0.0
    worst = float((np.abs(got[fin] - want[fin]) / want[fin]).max())
    assert worst <= tol, f"{p.name}: max rel err {worst:.3e}"
    return worst


def mixed_problems(f32=True):
    """Grids of different sizes, shapes, speeds and source counts (ragged cells included)."""
    ps = [
        W.maze(33, seed=21, n_sources=2),
        W.oscillatory(41, periods=3),
        W.random_small(19, 7, n_sources=3, nx=27, ny=11),
        W.constant(17, tol=0.0),
        W.maze(49, seed=22, n_sources=1),
        W.random_small(9, 8, n_sources=1, nx=5, ny=30),
        W.checkerboard(25, K=5),
    ]
    for p in ps:
        p.F = np.ascontiguousarray(p.F.astype(np.float32 if f32 else np.float64))
    return ps


def as_dicts(ps, dev):
    import torch
    return [dict(F=torch.from_numpy(p.F).to(dev), h=p.h, src=p.src, q=p.q, tol=0.0) for p in ps]


@pytest.mark.parametrize("inner", [1, 2, 3])
@pytest.mark.parametrize("cell", [8, 4])
def test_batch_matches_oracle_and_alone(orc, torch_dev, cell, inner):
    from paper_1306_4743_amd import eik
    ps = mixed_problems()
    outs = eik.solve_batch(as_dicts(ps, torch_dev), cell=cell, inner=inner)
    st = eik.batch_status(len(ps))
    assert list(st) == [0] * len(ps)
    rc, stats = eik.status()
    assert rc == 0
    assert stats["cells"] == sum(-(-p.dims[0] // cell) * -(-p.dims[1] // cell) *
                                 -(-p.dims[2] // cell) for p in ps)
    worst_alone = 0.0
    for p, u in zip(ps, outs):
        got = u.cpu().numpy()
        want = orc.fmm(p.F, p.h, p.src, p.q)
        compare(got, want, p)
        import torch
        alone = eik.solve(torch.from_numpy(p.F).to(torch_dev), p.h, p.src, p.q, cell=cell,
                          tol=0.0, inner=inner).cpu().numpy()
        assert eik.status()[0] == 0
        worst_alone = max(worst_alone, compare(got, alone, p))
    print(f"cell {cell} inner {inner}: batch vs alone max rel diff {worst_alone:.2e}, {stats}",
          flush=True)


def test_batch_fp64_speeds_and_empty_sources(orc, torch_dev):
    """FP64 speeds; a grid without sources stays +inf everywhere next to solved grids."""
    from paper_1306_4743_amd import eik
    ps = mixed_problems(f32=False)[:3]
    empty = W.constant(21)
    empty.src = np.zeros((0, 3), dtype=np.int64)
    empty.q = np.zeros(0)
    ps.append(empty)
    outs = eik.solve_batch(as_dicts(ps, torch_dev), cell=8)
    assert list(eik.batch_status(len(ps))) == [0] * len(ps)
    for p, u in zip(ps[:3], outs[:3]):
        compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)
    assert np.all(np.isinf(outs[3].cpu().numpy()))


def test_batch_status_is_per_problem(orc, torch_dev):
    """An invalid speed in one grid is reported for that grid only; the others are solved."""
    from paper_1306_4743_amd import eik
    ps = mixed_problems()[:4]
    ps[2].F[3, 4, 5] = 0.0
    outs = eik.solve_batch(as_dicts(ps, torch_dev), cell=8)
    st = eik.batch_status(len(ps))
    assert list(st) == [0, 0, eik.EIK_EINVAL, 0]
    for i in (0, 1, 3):
        p = ps[i]
        compare(outs[i].cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)


def test_batch_of_many_small_grids(orc, torch_dev):
    """64 grids of 9..24 nodes per side in one launch (the many-small-requests regime)."""
    from paper_1306_4743_amd import eik
    rng = np.random.default_rng(5)
    ps = []
    for i in range(64):
        n = int(rng.integers(9, 25))
        p = W.random_small(n, 100 + i, n_sources=int(rng.integers(1, 4)))
        p.F = p.F.astype(np.float32)
        ps.append(p)
    outs = eik.solve_batch(as_dicts(ps, torch_dev), cell=4)
    assert list(eik.batch_status(len(ps))) == [0] * len(ps)
    for p, u in zip(ps, outs):
        compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)


def run_server(eik, srv, queue, rounds, max_steps=5000):
    """Submit in order (retrying after EIK_EBUSY), step until everything is retired."""
    done, tickets = {}, {}
    pending = list(queue)
    steps = 0
    while pending or len(done) < len(queue):
        while pending:
            key, kw = pending[0]
            t = srv.submit(**kw)
            if t is None:
                break
            tickets[t] = key
            pending.pop(0)
        for t, (status, u) in srv.step(rounds).items():
            done[tickets[t]] = (status, u)
        steps += 1
        assert steps < max_steps, "server did not drain"
    return done, steps


@pytest.mark.parametrize("rounds", [1, 6, 1000])
def test_server_matches_oracle(orc, torch_dev, rounds):
    """A pool that holds about two grids at a time: admission waits (EIK_EBUSY), grids retire
    independently, each result equals the oracle's and the grid solved alone."""
    import torch
    from paper_1306_4743_amd import eik
    ps = mixed_problems()
    big = max(eik.problem_bytes(p.dims, 8, eik.EIK_F32) for p in ps)
    srv = eik.Server(pool_bytes=2 * big + 4096, max_cells=4096, max_problems=3, cell=8)
    queue = [(i, dict(F=torch.from_numpy(p.F).to(torch_dev), h=p.h, idx3=p.src, q=p.q, tol=0.0))
             for i, p in enumerate(ps)]
    done, steps = run_server(eik, srv, queue, rounds)
    assert sorted(done) == list(range(len(ps)))
    assert srv.load() == {"problems": 0, "cells": 0, "pool_bytes": 0}
    for i, p in enumerate(ps):
        status, u = done[i]
        assert status == 0
        got = u.cpu().numpy()
        compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
        alone = eik.solve(torch.from_numpy(p.F).to(torch_dev), p.h, p.src, p.q, cell=8,
                          tol=0.0).cpu().numpy()
        compare(got, alone, p)
    srv.close()
    print(f"rounds/step {rounds}: {steps} steps", flush=True)


def test_server_late_arrivals_and_invalid_grid(orc, torch_dev):
    """Grids arriving while others are mid-solve, one with an invalid speed (reported for it
    alone), cell side 4, and the server reused after it drained."""
    import torch
    from paper_1306_4743_amd import eik
    ps = mixed_problems()
    ps[1].F[2, 2, 2] = np.nan
    srv = eik.Server(pool_bytes=256 << 20, max_cells=1 << 16, max_problems=8, cell=4)
    tick = {}
    results = {}
    t = srv.submit(torch.from_numpy(ps[0].F).to(torch_dev), ps[0].h, ps[0].src, ps[0].q)
    tick[t] = 0
    nxt = 1
    for step in range(4000):
        if nxt < len(ps) and step % 2 == 1:
            p = ps[nxt]
            t = srv.submit(torch.from_numpy(p.F).to(torch_dev), p.h, p.src, p.q)
            assert t is not None
            tick[t] = nxt
            nxt += 1
        for t, r in srv.step(2).items():
            results[tick[t]] = r
        if len(results) == len(ps):
            break
    assert len(results) == len(ps)
    assert sorted(tick) == list(range(len(ps)))  # tickets 0, 1, 2, ... in submission order
    for i, p in enumerate(ps):
        status, u = results[i]
        if i == 1:
            assert status == eik.EIK_EINVAL
            continue
        assert status == 0
        compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)
    # reuse after draining
    p = ps[4]
    t = srv.submit(torch.from_numpy(p.F).to(torch_dev), p.h, p.src, p.q)
    again = {}
    for _ in range(4000):
        again.update(srv.step(50))
        if t in again:
            break
    assert again[t][0] == 0
    compare(again[t][1].cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)
    srv.close()


def test_server_rejects_grid_that_never_fits(torch_dev):
    import torch
    from paper_1306_4743_amd import eik
    p = W.constant(65)
    p.F = p.F.astype(np.float32)
    srv = eik.Server(pool_bytes=1 << 20, max_cells=64, max_problems=2, cell=8)
    with pytest.raises(eik.EikError):
        srv.submit(torch.from_numpy(p.F).to(torch_dev), p.h, p.src, p.q)
    srv.close()


def test_autotune_picks_a_valid_configuration(orc, torch_dev):
    """The autotuner tries every configuration, each one reaches EIK_OK, the fastest is
    returned, and the problem's result is the oracle's."""
    import torch
    from paper_1306_4743_amd import eik
    p = W.maze(65, seed=4, n_sources=2)
    F = torch.from_numpy(p.F).to(torch_dev)
    best, table = eik.autotune(F, p.h, p.src, p.q, reps=1)
    # r in {8, 4} x four in-cell solvers, r = 16 x two (no dual or paired sweeps), x two
    # worker counts, then three bands
    assert len(table) == 23
    assert {(t["cell"], t["inner"]) for t in table} == (
        {(c, i) for c in (8, 4) for i in (1, 2, 3, 4)} | {(16, 1), (16, 2)})
    assert all(t["status"] == 0 and 0 < t["ms"] < 1e4 for t in table)
    assert best["ms"] == min(t["ms"] for t in table)
    u = eik.solve(F, p.h, p.src, p.q, cell=best["cell"], inner=best["inner"],
                  workers=best["workers"], delta=best["delta"])
    assert eik.status()[0] == 0
    compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)
    print("autotune best", best, flush=True)


def test_fp32_mode_batch_and_server(orc, torch_dev):
    """FP32 mode through a batch and a server: each grid within the single-precision bound of
    the oracle (4 n 2^-24), same +inf mask."""
    import torch
    from paper_1306_4743_amd import eik
    ps = mixed_problems()[:5]
    bound = lambda p: 4.0 * max(p.dims) * 2.0 ** -24
    outs = eik.solve_batch(as_dicts(ps, torch_dev), cell=8, mode=eik.EIK_MODE_FP32)
    assert list(eik.batch_status(len(ps))) == [0] * len(ps)
    for p, u in zip(ps, outs):
        want = orc.fmm(p.F, p.h, p.src, p.q)
        got = u.cpu().numpy()
        assert np.array_equal(np.isinf(got), np.isinf(want))
        fin = np.isfinite(want) & (want > 0)
        assert float(np.max(np.abs(got[fin] - want[fin]) / want[fin])) <= bound(p)
    srv = eik.Server(pool_bytes=64 << 20, max_cells=1 << 14, max_problems=3, cell=8,
                     mode=eik.EIK_MODE_FP32)
    queue = [(i, dict(F=torch.from_numpy(p.F).to(torch_dev), h=p.h, idx3=p.src, q=p.q))
             for i, p in enumerate(ps)]
    done, _ = run_server(eik, srv, queue, 4)
    srv.close()
    for i, p in enumerate(ps):
        status, u = done[i]
        assert status == 0
        want = orc.fmm(p.F, p.h, p.src, p.q)
        got = u.cpu().numpy()
        fin = np.isfinite(want) & (want > 0)
        assert float(np.max(np.abs(got[fin] - want[fin]) / want[fin])) <= bound(p)


@pytest.mark.parametrize("delta", [0.02, 0.3])
def test_batch_with_band_per_grid(orc, torch_dev, delta):
    """With a band, each grid of a batch takes its band from its own smallest queued value
    (grids of different sizes and value ranges side by side); results are the oracle's."""
    import torch
    from paper_1306_4743_amd import eik
    ps = mixed_problems()
    outs = eik.solve_batch(as_dicts(ps, torch_dev), cell=8, delta=delta)
    assert list(eik.batch_status(len(ps))) == [0] * len(ps)
    for p, u in zip(ps, outs):
        compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)


def test_batch_polish_and_scratch_together(orc, torch_dev):
    """A batch where some grids start from an FP32 result (u_approx) and the others from
    scratch: every result is the oracle's."""
    import torch
    from paper_1306_4743_amd import eik
    ps = mixed_problems()
    ds = as_dicts(ps, torch_dev)
    approx = eik.solve_batch(ds, cell=8, mode=eik.EIK_MODE_FP32)
    assert list(eik.batch_status(len(ps))) == [0] * len(ps)
    for i, d in enumerate(ds):
        if i % 2 == 0:
            d["u_approx"] = approx[i]
    outs = eik.solve_batch(ds, cell=8)
    assert list(eik.batch_status(len(ps))) == [0] * len(ps)
    for p, u in zip(ps, outs):
        compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)


@pytest.mark.parametrize("banded", [False, True])
@pytest.mark.parametrize("rounds", [2, 50])
def test_server_chain_fp32_then_polish(orc, torch_dev, rounds, banded):
    """Mixed-precision serving: an FP32 server's results go to an FP64 server as u_approx (the
    same buffer); the polished results are the oracle's to 1e-10 and equal the grid solved
    alone.  Few problem slots, so admissions happen while others are mid-polish."""
    import torch
    from paper_1306_4743_amd import eik
    ps = mixed_problems()
    dev_F = [torch.from_numpy(p.F).to(torch_dev) for p in ps]
    s32 = eik.Server(pool_bytes=64 << 20, max_cells=1 << 14, max_problems=3, cell=8,
                     mode=eik.EIK_MODE_FP32)
    done32, _ = run_server(eik, s32, [(i, dict(F=dev_F[i], h=p.h, idx3=p.src, q=p.q))
                                      for i, p in enumerate(ps)], rounds)
    s32.close()
    assert all(done32[i][0] == 0 for i in range(len(ps)))
    band = 8.0 * 8 * min(p.h for p in ps) if banded else 0.0
    s64 = eik.Server(pool_bytes=64 << 20, max_cells=1 << 14, max_problems=3, cell=8, delta=band)
    queue = [(i, dict(F=dev_F[i], h=p.h, idx3=p.src, q=p.q, u_out=done32[i][1],
                      u_approx=done32[i][1])) for i, p in enumerate(ps)]
    done, steps = run_server(eik, s64, queue, rounds)
    s64.close()
    for i, p in enumerate(ps):
        status, u = done[i]
        assert status == 0
        got = u.cpu().numpy()
        compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
        alone = eik.solve(dev_F[i], p.h, p.src, p.q, cell=8, tol=0.0).cpu().numpy()
        compare(got, alone, p)
    print(f"polish server, rounds/step {rounds}: {steps} steps", flush=True)
