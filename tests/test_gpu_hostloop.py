"""The host-driven round loop (EIK_SCHED_HOST_LOOP: one ordinary launch per round, no grid
barrier) against the oracle: the same parity bar as the cooperative launch, on single solves,
bands, the single-precision and mixed modes, batches, a server, and the round cap."""
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


def compare(got, want, p, tol=REL_TOL):
    assert np.array_equal(np.isinf(got), np.isinf(want)), "+inf masks differ"
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
    u = eik.solve(F, p.h, p.src, p.q, cell=kw.pop("cell", 8), schedule=eik.EIK_SCHED_HOST_LOOP,
                  **kw)
    rc, st = eik.status()
    return u.cpu().numpy(), rc, st


@pytest.mark.parametrize("cell", [8, 4, 16])
@pytest.mark.parametrize("name", ["maze", "osc", "random"])
def test_host_loop_matches_oracle(orc, dev, name, cell):
    p = {"maze": lambda: W.maze(97, seed=3),
         "osc": lambda: W.oscillatory(65, periods=4),
         "random": lambda: W.random_small(21, 5, n_sources=3, nx=37, ny=13)}[name]()
    got, rc, st = solve(dev, p, cell=cell)
    assert rc == 0, st
    err = compare(got, orc.fmm(p.F, p.h, p.src, p.q), p)
    print(f"host loop {name} r {cell}: max rel err {err:.2e}, rounds {st['rounds']}, "
          f"visits {st['visits']}, workers {st['workers']}", flush=True)
    assert st["rounds"] >= 1 and st["workers"] > 0


def test_host_loop_same_as_cooperative(dev):
    """Both schedules run the same rounds on the same lists: identical values."""
    import torch
    from paper_1306_4743_amd import eik
    p = W.maze(65, seed=7, n_sources=2)
    F = torch.from_numpy(p.F).to(dev)
    a = eik.solve(F, p.h, p.src, p.q, cell=8, schedule=eik.EIK_SCHED_COOPERATIVE)
    rc_a, st_a = eik.status()
    b = eik.solve(F, p.h, p.src, p.q, cell=8, schedule=eik.EIK_SCHED_HOST_LOOP)
    rc_b, st_b = eik.status()
    assert rc_a == 0 and rc_b == 0
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    fin = np.isfinite(ga) & (ga > 0)
    assert np.array_equal(np.isinf(ga), np.isinf(gb))
    assert float(np.max(np.abs(ga[fin] - gb[fin]) / ga[fin])) <= 1e-13
    print(f"rounds cooperative {st_a['rounds']} host loop {st_b['rounds']}", flush=True)


@pytest.mark.parametrize("mode", [1, 2])
def test_host_loop_precision_modes(orc, dev, mode):
    from paper_1306_4743_amd import eik
    p = W.maze(65, seed=3)
    got, rc, _ = solve(dev, p, mode=mode)
    assert rc == 0
    tol = REL_TOL if mode == eik.EIK_MODE_MIXED else 4.0 * 65 * 2.0 ** -24
    want = orc.fmm(p.F, p.h, p.src, p.q)
    fin = np.isfinite(want) & (want > 0)
    assert np.array_equal(np.isinf(got), np.isinf(want))
    assert float(np.max(np.abs(got[fin] - want[fin]) / want[fin])) <= tol


def test_host_loop_band_and_round_cap(orc, dev):
    from paper_1306_4743_amd import eik
    p = W.maze(97, seed=3)
    got, rc, _ = solve(dev, p, delta=0.05)
    assert rc == 0
    want = orc.fmm(p.F, p.h, p.src, p.q)
    compare(got, want, p)
    got, rc, st = solve(dev, p, max_rounds=5)
    assert rc == eik.EIK_ENOCONV and st["rounds"] == 5
    assert np.all(got >= want * (1 - 1e-12))


def test_host_loop_batch_and_server(orc, dev):
    import torch
    from paper_1306_4743_amd import eik
    ps = [W.maze(33, seed=21, n_sources=2), W.random_small(19, 7, n_sources=3, nx=27, ny=11),
          W.oscillatory(41, periods=2, dtype=np.float32)]
    for p in ps:
        p.F = p.F.astype(np.float32)
    Fs = [torch.from_numpy(p.F).to(dev) for p in ps]
    outs = eik.solve_batch([dict(F=F, h=p.h, src=p.src, q=p.q) for p, F in zip(ps, Fs)], cell=8,
                           schedule=eik.EIK_SCHED_HOST_LOOP)
    assert list(eik.batch_status(len(ps))) == [0, 0, 0]
    for p, u in zip(ps, outs):
        compare(u.cpu().numpy(), orc.fmm(p.F, p.h, p.src, p.q), p)
    srv = eik.Server(1 << 28, 20000, 2, cell=8, schedule=eik.EIK_SCHED_HOST_LOOP)
    try:
        pending, done = list(range(len(ps))), {}
        tickets = {}
        while len(done) < len(ps):
            while pending:
                i = pending[0]
                t = srv.submit(Fs[i], ps[i].h, ps[i].src, ps[i].q)
                if t is None:
                    break
                tickets[t] = i
                pending.pop(0)
            for t, (st, u) in srv.step(3).items():
                assert st == 0
                done[tickets[t]] = u.cpu().numpy()
        for i, p in enumerate(ps):
            compare(done[i], orc.fmm(p.F, p.h, p.src, p.q), p)
    finally:
        srv.close()
