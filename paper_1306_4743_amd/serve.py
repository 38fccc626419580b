"""Serving harness: a Poisson stream of Eikonal requests through the continuous-batching server
(``eik_server_*``), measured against one-at-a-time solves of the same stream.

The request mix is the mixed-size serving workload: request i has n nodes per side drawn
uniformly from {33, 65, 129, 193, 257}, the barrier-maze speeds of ``workloads.maze_layout``
drawn with seed 5000 + i (wall thickness and opening size scaled with (n-1)/512, floors 1 and
2), 1-4 exit nodes drawn uniformly, q = 0, FP32 speeds, FP64 values, tol 0.  Speeds and result
buffers of every request are resident in device memory before the clock starts (a serving
process keeps its inputs in HBM); a request's latency runs from its arrival time to the end of
the server step (or solve) after which its result is in its output buffer.

Runs:
  * saturated: every request arrives at time 0; gives the server's throughput (requests/s).
  * Poisson arrivals at fractions (0.5, 0.8, 1.0) of that throughput: p50 / p99 latency.
  * saturated in FP32 mode (for context: values about 1e-5 relative, not the FP64 bar).
  * the mode mix, saturated and at Poisson arrivals: a fair coin (``request_modes``) gives each
    request FP64 or FP32 + FP64 polish; FP64 requests go to the FP64 server, the others to an
    FP32 server and then to the same FP64 server, which polishes the FP32 result
    (``eik_problem.u_approx``) to the FP64 solution (``run_stream``); every request at 1e-10.
  * every request in FP32 + polish, saturated.
  * one-at-a-time: the same stream, FIFO, each request solved alone with ``eik_solve`` (in FP64,
    and in its own mode: FP32 + polish = one EIK_MODE_MIXED solve).

Usage: python -m paper_1306_4743_amd.serve [--requests N] [--rounds R] [--json]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

SIZES = (33, 65, 129, 193, 257)


@dataclasses.dataclass
class Request:
    i: int
    n: int
    seed: int
    n_sources: int
    F: object       # torch float32 [n, n, n] on the device
    h: float
    src: np.ndarray
    q: np.ndarray
    u: object       # torch float64 [n, n, n] on the device (the result buffer)
    polish: bool = False  # mode: FP32 solve + FP64 polish (True) or FP64 (False)

    @property
    def nodes(self) -> int:
        return self.n ** 3


def request_shapes(count: int, seed: int = 1234, sizes=SIZES):
    """(n, number of exits) of the first `count` requests of the stream."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(sizes[int(rng.integers(len(sizes)))])
        out.append((n, int(rng.integers(1, 5))))
    return out


def request_shape(i: int, seed: int = 1234, sizes=SIZES):
    """(n, number of exits) of request i of the stream."""
    return request_shapes(i + 1, seed, sizes)[i]


def request_modes(count: int, seed: int = 4321) -> np.ndarray:
    """Mode of each request of the stream: a fair coin, True = FP32 solve + FP64 polish."""
    return np.random.default_rng(seed).integers(0, 2, size=count).astype(bool)


def make_requests(count: int, device, seed: int = 1234, sizes=SIZES):
    """The request stream: sizes and exit counts from ``seed``, maze i from seed 5000 + i, modes
    from ``request_modes``."""
    import torch
    from . import workloads as W
    reqs = []
    modes = request_modes(count)
    for i, (n, ns) in enumerate(request_shapes(count, seed, sizes)):
        F, h, src, q = W.maze_torch(n, 5000 + i, ns, device)
        u = torch.empty(F.shape, dtype=torch.float64, device=device)
        reqs.append(Request(i, n, 5000 + i, ns, F, h, src, q, u, bool(modes[i])))
    torch.cuda.synchronize(device)
    return reqs


def poisson_arrivals(count: int, rate: float, seed: int = 99) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate, the first at 0."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
    return np.concatenate([[0.0], np.cumsum(gaps[:-1])])


def _summary(reqs, arrivals, finish, t_first, t_last):
    lat = (finish - arrivals) * 1000.0
    nodes = sum(r.nodes for r in reqs)
    span = t_last - t_first
    by = {}
    for n in sorted({r.n for r in reqs}):
        sel = np.array([r.n == n for r in reqs])
        by[str(n)] = {"count": int(sel.sum()), "p50_ms": float(np.percentile(lat[sel], 50)),
                      "p99_ms": float(np.percentile(lat[sel], 99))}
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "makespan_s": span,
            "requests_per_s": len(reqs) / span, "solved_nodes_per_s": nodes / span,
            "by_size": by}


def pool_config(reqs, cell: int, pool_bytes: int, mode: int = 0):
    from . import eik
    per_cell = eik.problem_bytes((cell, cell, cell), cell, eik.EIK_F32, mode)
    biggest = max(eik.problem_bytes((r.n,) * 3, cell, eik.EIK_F32, mode) for r in reqs)
    pool_bytes = max(pool_bytes, biggest)
    return pool_bytes, pool_bytes // per_cell + 1


def run_server(reqs, arrivals, cell: int = 8, rounds: int = 8, pool_bytes: int = 32 << 30,
               max_problems: int = 512, **opt):
    """Feed ``reqs`` (arriving at ``arrivals`` seconds) to one server; returns the summary."""
    import torch
    from . import eik
    pool_bytes, max_cells = pool_config(reqs, cell, pool_bytes, opt.get("mode", 0))
    srv = eik.Server(pool_bytes, max_cells, max_problems, cell=cell, f_dtype=eik.EIK_F32, **opt)
    count = len(reqs)
    finish = np.full(count, np.nan)
    owner = {}
    nxt, done, on_dev, steps = 0, 0, 0, 0
    statuses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < count:
        now = time.perf_counter() - t0
        while nxt < count and arrivals[nxt] <= now:
            r = reqs[nxt]
            t = srv.submit(r.F, r.h, r.src, r.q, 0.0, r.u)
            if t is None:
                break  # no room now: the head of the queue waits for a retirement
            owner[t] = nxt
            nxt += 1
            on_dev += 1
        if on_dev == 0:
            while time.perf_counter() - t0 < arrivals[nxt]:
                pass
            continue
        out = srv.step(rounds)
        steps += 1
        tnow = time.perf_counter() - t0
        for t, (status, _) in out.items():
            finish[owner[t]] = tnow
            statuses.append(status)
            done += 1
            on_dev -= 1
    srv.close()
    if any(s != 0 for s in statuses):
        raise RuntimeError(f"server returned statuses {sorted(set(statuses))}")
    res = _summary(reqs, arrivals, finish, 0.0, float(np.nanmax(finish)))
    res["steps"] = steps
    return res


def run_stream(reqs, arrivals, cell: int = 8, rounds: int = 8, pool_bytes: int = 32 << 30,
               max_problems: int = 512, polish=None):
    """Feed ``reqs`` to servers by mode: an FP64 request goes to the FP64 server; an FP32 +
    polish request goes to an FP32 server and, when it retires there, to the same FP64 server
    with ``u_approx`` = its FP32 result (in the request's own output buffer), which polishes it.
    polish: None = each request's own mode, True / False = every request in that mode.
    Arrivals are admitted in order; the two servers step in turn on one stream.  A request
    finishes when the FP64 server retires it."""
    import torch
    from . import eik
    want = [r.polish if polish is None else bool(polish) for r in reqs]
    count = len(reqs)

    def server(subset, mode):
        if not subset:
            return None
        pb, mc = pool_config(subset, cell, pool_bytes, mode)
        return eik.Server(pb, mc, max_problems, cell=cell, f_dtype=eik.EIK_F32, mode=mode)

    pol = [r for r, w in zip(reqs, want) if w]
    s64 = server(reqs, eik.EIK_MODE_FP64)  # FP64 requests and the polish of the others
    s32 = server(pol, eik.EIK_MODE_FP32)
    owner = {id(x): {} for x in (s64, s32) if x is not None}
    on = {id(x): 0 for x in (s64, s32) if x is not None}
    finish = np.full(count, np.nan)
    polish_queue = []
    nxt, done, steps = 0, 0, 0

    def submit(srv, k, **kw):
        r = reqs[k]
        t = srv.submit(r.F, r.h, r.src, r.q, 0.0, r.u, **kw)
        if t is None:
            return False
        owner[id(srv)][t] = k
        on[id(srv)] += 1
        return True

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < count:
        now = time.perf_counter() - t0
        while nxt < count and arrivals[nxt] <= now:
            if not submit(s32 if want[nxt] else s64, nxt):
                break  # no room now: the head of the queue waits for a retirement
            nxt += 1
        while polish_queue and submit(s64, polish_queue[0], u_approx=reqs[polish_queue[0]].u):
            polish_queue.pop(0)
        if sum(on.values()) == 0:
            while time.perf_counter() - t0 < arrivals[nxt]:
                pass
            continue
        for srv in (s32, s64):
            if srv is None or on[id(srv)] == 0:
                continue
            out = srv.step(rounds)
            steps += 1
            tnow = time.perf_counter() - t0
            for t, (status, _) in out.items():
                k = owner[id(srv)].pop(t)
                on[id(srv)] -= 1
                if status != 0:
                    raise RuntimeError(f"request {k}: {eik.strerror(status)}")
                if srv is s32:
                    polish_queue.append(k)
                else:
                    finish[k] = tnow
                    done += 1
    for srv in (s64, s32):
        if srv is not None:
            srv.close()
    res = _summary(reqs, arrivals, finish, 0.0, float(np.nanmax(finish)))
    res["steps"] = steps
    res["polish_requests"] = int(sum(want))
    return res


def run_server_mixed(reqs, arrivals, cell: int = 8, rounds: int = 8,
                     pool_bytes: int = 32 << 30, max_problems: int = 512):
    """Every request in FP32 + polish mode (``run_stream`` with polish=True)."""
    return run_stream(reqs, arrivals, cell, rounds, pool_bytes, max_problems, True)


def run_sequential(reqs, arrivals, cell: int = 8, by_mode: bool = False, **opt):
    """The same stream, FIFO, one ``eik_solve`` at a time (each waits for the previous); with
    by_mode, each request in its own mode (FP32 + polish = one EIK_MODE_MIXED solve)."""
    import torch
    from . import eik
    count = len(reqs)
    finish = np.full(count, np.nan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        while time.perf_counter() - t0 < arrivals[k]:
            pass
        kw = dict(opt)
        if by_mode and r.polish:
            kw["mode"] = eik.EIK_MODE_MIXED
        eik.solve(r.F, r.h, r.src, r.q, cell=cell, tol=0.0, u_out=r.u, **kw)
        rc, _ = eik.status()
        if rc != 0:
            raise RuntimeError(f"request {r.i}: {eik.strerror(rc)}")
        finish[k] = time.perf_counter() - t0
    return _summary(reqs, arrivals, finish, 0.0, float(finish.max()))


def check_against_alone(reqs, sample: int = 10, cell: int = 8):
    """Max relative difference between served results and the same requests solved alone."""
    import torch
    from . import eik
    idx = np.linspace(0, len(reqs) - 1, min(sample, len(reqs))).astype(int)
    worst = 0.0
    for k in idx:
        r = reqs[int(k)]
        alone = eik.solve(r.F, r.h, r.src, r.q, cell=cell, tol=0.0)
        rc, _ = eik.status()
        if rc != 0:
            raise RuntimeError(eik.strerror(rc))
        a, b = alone.cpu().numpy(), r.u.cpu().numpy()
        if not np.array_equal(np.isinf(a), np.isinf(b)):
            return float("inf")
        fin = np.isfinite(a) & (a > 0)
        worst = max(worst, float(np.max(np.abs(a[fin] - b[fin]) / a[fin])))
        del alone
    torch.cuda.synchronize()
    return worst


def serve_benchmark(count: int = 2000, rounds: int = 8, cell: int = 8,
                    fractions=(0.5, 0.8, 1.0), seq_fraction: float = 0.8,
                    pool_bytes: int = 32 << 30, log=None, tune: bool = False,
                    tune_cache: str | None = None):
    """The whole serving measurement; returns a JSON-able dict.  With ``tune`` the servers'
    cell size and rounds per step come from the tuning cache (``tuning.tuned_server_config``,
    measured on a sample of this stream when the cache has no entry for it) instead of
    ``cell`` and ``rounds``."""
    import torch
    from . import eik
    eik.load()
    dev = torch.device("cuda:0")

    def say(msg):
        if log:
            print(msg, file=log, flush=True)

    def poisson_runs(runner, sat_rate):
        out = {}
        for f in fractions:
            rate = f * sat_rate
            res = runner(poisson_arrivals(count, rate))
            res["arrival_rate_per_s"] = rate
            out[str(f)] = res
            say(f"serve: {f:.1f}x rate: p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms")
        return out

    t = time.perf_counter()
    reqs = make_requests(count, dev)
    say(f"serve: {count} requests generated in {time.perf_counter() - t:.1f} s")
    tuned = None
    if tune:
        from . import tuning
        cache = tuning.TuneCache(tune_cache) if tune_cache else tuning.TuneCache()
        cfg, key, table = tuning.tuned_server_config(reqs, SIZES, eik.EIK_MODE_FP64, cache,
                                                     log=log, pool_bytes=pool_bytes)
        cell, rounds = cfg["cell"], cfg["rounds_per_step"]
        tuned = {"key": key, "cell": cell, "rounds_per_step": rounds,
                 "measured_now": table is not None, "table": table}
        say(f"serve: tuned server configuration {key}: cell {cell}, {rounds} rounds per step")
    # warm-up: a few requests through each kind of server and alone
    run_server(reqs[:8], np.zeros(8), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    run_stream(reqs[:8], np.zeros(8), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    run_sequential(reqs[:4], np.zeros(4), cell=cell, by_mode=True)
    out = {"requests": count, "sizes": list(SIZES), "cell": cell, "rounds_per_step": rounds,
           "pool_bytes": pool_bytes, "tuned": tuned}
    # Every request in FP64.
    sat = run_server(reqs, np.zeros(count), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    say(f"serve: FP64 saturated {sat['requests_per_s']:.1f} req/s, {sat['steps']} steps")
    out["saturated"] = sat
    out["max_rel_diff_served_vs_alone"] = check_against_alone(reqs, cell=cell)
    out["poisson"] = poisson_runs(
        lambda arr: run_server(reqs, arr, cell=cell, rounds=rounds, pool_bytes=pool_bytes),
        sat["requests_per_s"])
    # The same stream in single precision (values ~1e-5 relative, not the FP64 bar).
    sat32 = run_server(reqs, np.zeros(count), cell=cell, rounds=rounds, pool_bytes=pool_bytes,
                       mode=eik.EIK_MODE_FP32)
    out["saturated_fp32_mode"] = sat32
    say(f"serve: saturated, FP32 mode {sat32['requests_per_s']:.1f} req/s")
    # The mode mix: a fair coin picks FP64 or FP32 + FP64 polish per request (both at 1e-10).
    for r in reqs:
        r.u.fill_(float("nan"))  # the checks below must see these results, not earlier ones
    coin = run_stream(reqs, np.zeros(count), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    coin["max_rel_diff_served_vs_alone"] = check_against_alone(reqs, cell=cell)
    say(f"serve: coin-mix saturated {coin['requests_per_s']:.1f} req/s "
        f"({coin['polish_requests']} FP32 + polish), max rel diff "
        f"{coin['max_rel_diff_served_vs_alone']:.1e}")
    out["mode_mix"] = {"saturated": coin, "poisson": poisson_runs(
        lambda arr: run_stream(reqs, arr, cell=cell, rounds=rounds, pool_bytes=pool_bytes),
        coin["requests_per_s"])}
    # Every request in FP32 + polish.
    for r in reqs:
        r.u.fill_(float("nan"))
    mixed = run_server_mixed(reqs, np.zeros(count), cell=cell, rounds=rounds,
                             pool_bytes=pool_bytes)
    mixed["max_rel_diff_served_vs_alone"] = check_against_alone(reqs, cell=cell)
    out["mixed_fp32_polish_saturated"] = mixed
    say(f"serve: saturated, all FP32 + FP64 polish {mixed['requests_per_s']:.1f} req/s")
    # One at a time.
    seq_sat = run_sequential(reqs, np.zeros(count), cell=cell)
    out["one_at_a_time_saturated"] = seq_sat
    say(f"serve: one-at-a-time FP64 {seq_sat['requests_per_s']:.1f} req/s")
    rate = seq_fraction * sat["requests_per_s"]
    seq = run_sequential(reqs, poisson_arrivals(count, rate), cell=cell)
    seq["arrival_rate_per_s"] = rate
    out["one_at_a_time_poisson"] = {str(seq_fraction): seq}
    say(f"serve: one-at-a-time at {seq_fraction}x: p50 {seq['p50_ms']:.1f} p99 {seq['p99_ms']:.1f}")
    seq_mix = run_sequential(reqs, np.zeros(count), cell=cell, by_mode=True)
    out["mode_mix"]["one_at_a_time_saturated"] = seq_mix
    say(f"serve: one-at-a-time, coin mix {seq_mix['requests_per_s']:.1f} req/s")
    del reqs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rounds", type=int, default=8, help="worklist rounds per server step")
    ap.add_argument("--cell", type=int, default=8)
    ap.add_argument("--pool-gib", type=float, default=32.0)
    ap.add_argument("--tune", action="store_true",
                    help="cell size and rounds per step from the tuning cache (measured if absent)")
    ap.add_argument("--tune-cache", default=None, help="tuning cache file (JSON)")
    a = ap.parse_args()
    res = serve_benchmark(a.requests, a.rounds, a.cell, pool_bytes=int(a.pool_gib * (1 << 30)),
                          log=sys.stderr, tune=a.tune, tune_cache=a.tune_cache)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
