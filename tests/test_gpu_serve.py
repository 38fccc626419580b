"""GPU parity of the serving harness: a small Poisson stream of mixed-size maze requests
through the continuous-batching server.  Every served result equals the oracle's FMM (same
+inf masks, exact exits, rel err <= 1e-10) and the same request solved alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

REL_TOL = 1e-10


def _rel(a, b):
    assert np.array_equal(np.isinf(a), np.isinf(b))
    fin = np.isfinite(b) & (b > 0)
    return float(np.max(np.abs(a[fin] - b[fin]) / b[fin])) if fin.any() else 0.0


@pytest.mark.parametrize("cell,rounds", [(8, 4), (4, 16)])
def test_served_stream_matches_oracle(orc, cell, rounds):
    import torch
    from paper_1306_4743_amd import eik, serve
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    reqs = serve.make_requests(24, dev, seed=7, sizes=(17, 33, 49))
    arrivals = serve.poisson_arrivals(len(reqs), rate=3000.0, seed=3)
    res = serve.run_server(reqs, arrivals, cell=cell, rounds=rounds, pool_bytes=24 << 20,
                           max_problems=6)
    assert res["requests"] == len(reqs) and res["p99_ms"] >= res["p50_ms"] > 0
    for r in reqs:
        got = r.u.cpu().numpy()
        F = r.F.cpu().numpy()
        want = orc.fmm(F, r.h, r.src, r.q)
        s = r.src
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], r.q)
        assert _rel(got, want) <= REL_TOL, r
        alone = eik.solve(r.F, r.h, r.src, r.q, cell=cell, tol=0.0).cpu().numpy()
        assert eik.status()[0] == 0
        assert _rel(got, alone) <= REL_TOL
    seq = serve.run_sequential(reqs, arrivals, cell=cell)
    assert seq["requests"] == len(reqs)
    print(f"cell {cell}: served p50 {res['p50_ms']:.2f} ms p99 {res['p99_ms']:.2f} ms, "
          f"one-at-a-time p50 {seq['p50_ms']:.2f} p99 {seq['p99_ms']:.2f}", flush=True)


def test_mixed_precision_stream_matches_oracle(orc):
    """The serving harness's FP32 + FP64-polish chain on a small Poisson stream: every result
    equals the oracle's FMM to 1e-10 with exact exits."""
    import torch
    from paper_1306_4743_amd import serve
    dev = torch.device("cuda:0")
    reqs = serve.make_requests(16, dev, seed=11, sizes=(17, 33, 49))
    arrivals = serve.poisson_arrivals(len(reqs), rate=3000.0, seed=4)
    res = serve.run_server_mixed(reqs, arrivals, cell=8, rounds=4, pool_bytes=24 << 20,
                                 max_problems=5)
    assert res["requests"] == len(reqs) and res["p99_ms"] >= res["p50_ms"] > 0
    for r in reqs:
        got = r.u.cpu().numpy()
        want = orc.fmm(r.F.cpu().numpy(), r.h, r.src, r.q)
        s = r.src
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], r.q)
        assert _rel(got, want) <= REL_TOL, r


def test_mode_mix_stream_matches_oracle(orc):
    """The coin-mixed stream (FP64 requests to an FP64 server, FP32 + polish requests through an
    FP32 server into a polishing server): every result is the oracle's to 1e-10."""
    import torch
    from paper_1306_4743_amd import serve
    dev = torch.device("cuda:0")
    reqs = serve.make_requests(20, dev, seed=13, sizes=(17, 33, 49))
    assert 0 < sum(r.polish for r in reqs) < len(reqs)
    arrivals = serve.poisson_arrivals(len(reqs), rate=2000.0, seed=5)
    res = serve.run_stream(reqs, arrivals, cell=8, rounds=3, pool_bytes=24 << 20, max_problems=4)
    assert res["requests"] == len(reqs) and res["polish_requests"] == sum(r.polish for r in reqs)
    for r in reqs:
        got = r.u.cpu().numpy()
        want = orc.fmm(r.F.cpu().numpy(), r.h, r.src, r.q)
        s = r.src
        assert np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], r.q)
        assert _rel(got, want) <= REL_TOL, r
    seq = serve.run_sequential(reqs, arrivals, cell=8, by_mode=True)
    assert seq["requests"] == len(reqs)
    for r in reqs:
        assert _rel(r.u.cpu().numpy(), orc.fmm(r.F.cpu().numpy(), r.h, r.src, r.q)) <= REL_TOL
