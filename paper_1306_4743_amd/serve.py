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
  * mixed precision, saturated and at Poisson arrivals: an FP32 server solves each request, a
    second (FP64) server polishes that result (``eik_problem.u_approx``) to the FP64 solution;
    a request moves from the first server to the second when it retires there.
  * one-at-a-time: the same stream, FIFO, each request solved alone with ``eik_solve``.

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


def make_requests(count: int, device, seed: int = 1234, sizes=SIZES):
    """The request stream: sizes and exit counts from ``seed``, maze i from seed 5000 + i."""
    import torch
    from . import workloads as W
    reqs = []
    for i, (n, ns) in enumerate(request_shapes(count, seed, sizes)):
        F, h, src, q = W.maze_torch(n, 5000 + i, ns, device)
        u = torch.empty(F.shape, dtype=torch.float64, device=device)
        reqs.append(Request(i, n, 5000 + i, ns, F, h, src, q, u))
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


def run_server(reqs, arrivals, cell: int = 8, rounds: int = 8, pool_bytes: int = 16 << 30,
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


def polish_band(reqs, cell: int) -> float:
    """Priority band of the polishing server: 32 cell crossings at the finest grid step (on the
    mixed-size maze stream the fastest of 8, 32, 128 and 512 crossings or no band)."""
    return 32.0 * cell * min(r.h for r in reqs)


def run_server_mixed(reqs, arrivals, cell: int = 8, rounds: int = 8,
                     pool_bytes: int = 16 << 30, max_problems: int = 512, band=None):
    """Feed ``reqs`` through an FP32 server and then an FP64 polishing server (u_approx = the
    FP32 result, in the request's own output buffer); both step in turn on one stream.  A
    request finishes when the polishing server retires it."""
    import torch
    from . import eik
    p32, c32 = pool_config(reqs, cell, pool_bytes, eik.EIK_MODE_FP32)
    p64, c64 = pool_config(reqs, cell, pool_bytes, eik.EIK_MODE_FP64)
    s32 = eik.Server(p32, c32, max_problems, cell=cell, f_dtype=eik.EIK_F32,
                     mode=eik.EIK_MODE_FP32)
    s64 = eik.Server(p64, c64, max_problems, cell=cell, f_dtype=eik.EIK_F32,
                     delta=polish_band(reqs, cell) if band is None else band)
    count = len(reqs)
    finish = np.full(count, np.nan)
    own32, own64 = {}, {}
    polish_queue = []  # requests whose FP32 result waits for the polishing server
    nxt, done, on32, on64, steps = 0, 0, 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < count:
        now = time.perf_counter() - t0
        while nxt < count and arrivals[nxt] <= now:
            r = reqs[nxt]
            t = s32.submit(r.F, r.h, r.src, r.q, 0.0, r.u)
            if t is None:
                break
            own32[t] = nxt
            nxt += 1
            on32 += 1
        while polish_queue:
            r = reqs[polish_queue[0]]
            t = s64.submit(r.F, r.h, r.src, r.q, 0.0, r.u, u_approx=r.u)
            if t is None:
                break
            own64[t] = polish_queue.pop(0)
            on64 += 1
        if on32 == 0 and on64 == 0:
            while time.perf_counter() - t0 < arrivals[nxt]:
                pass
            continue
        if on32:
            for t, (status, _) in s32.step(rounds).items():
                if status != 0:
                    raise RuntimeError(f"FP32 server: request {own32[t]}: {eik.strerror(status)}")
                polish_queue.append(own32.pop(t))
                on32 -= 1
            steps += 1
        if on64:
            out = s64.step(rounds)
            tnow = time.perf_counter() - t0
            for t, (status, _) in out.items():
                if status != 0:
                    raise RuntimeError(f"polish server: request {own64[t]}: {eik.strerror(status)}")
                finish[own64.pop(t)] = tnow
                done += 1
                on64 -= 1
            steps += 1
    s32.close()
    s64.close()
    res = _summary(reqs, arrivals, finish, 0.0, float(np.nanmax(finish)))
    res["steps"] = steps
    return res


def run_sequential(reqs, arrivals, cell: int = 8, **opt):
    """The same stream, FIFO, one ``eik_solve`` at a time (each waits for the previous)."""
    import torch
    from . import eik
    count = len(reqs)
    finish = np.full(count, np.nan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        while time.perf_counter() - t0 < arrivals[k]:
            pass
        eik.solve(r.F, r.h, r.src, r.q, cell=cell, tol=0.0, u_out=r.u, **opt)
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
                    pool_bytes: int = 16 << 30, log=None):
    """The whole serving measurement; returns a JSON-able dict."""
    import torch
    from . import eik
    eik.load()
    dev = torch.device("cuda:0")

    def say(msg):
        if log:
            print(msg, file=log, flush=True)

    t = time.perf_counter()
    reqs = make_requests(count, dev)
    say(f"serve: {count} requests generated in {time.perf_counter() - t:.1f} s")
    # warm-up: a few requests through a server and alone
    run_server(reqs[:8], np.zeros(8), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    run_sequential(reqs[:4], np.zeros(4), cell=cell)
    run_server_mixed(reqs[:8], np.zeros(8), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    sat = run_server(reqs, np.zeros(count), cell=cell, rounds=rounds, pool_bytes=pool_bytes)
    say(f"serve: saturated {sat['requests_per_s']:.1f} req/s, {sat['steps']} steps")
    alone_diff = check_against_alone(reqs, cell=cell)
    out = {"requests": count, "sizes": list(SIZES), "cell": cell, "rounds_per_step": rounds,
           "pool_bytes": pool_bytes, "saturated": sat, "max_rel_diff_served_vs_alone": alone_diff,
           "poisson": {}}
    for f in fractions:
        rate = f * sat["requests_per_s"]
        res = run_server(reqs, poisson_arrivals(count, rate), cell=cell, rounds=rounds,
                         pool_bytes=pool_bytes)
        res["arrival_rate_per_s"] = rate
        out["poisson"][str(f)] = res
        say(f"serve: {f:.1f}x rate: p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms")
    # The same stream served in single precision (values ~1e-5 relative, not the FP64 bar).
    sat32 = run_server(reqs, np.zeros(count), cell=cell, rounds=rounds, pool_bytes=pool_bytes,
                       mode=eik.EIK_MODE_FP32)
    out["saturated_fp32_mode"] = sat32
    say(f"serve: saturated, FP32 mode {sat32['requests_per_s']:.1f} req/s")
    # FP32 bulk + FP64 polish: the FP64 bar at FP32's cost plus the polish.
    for r in reqs:
        r.u.fill_(float("nan"))  # the check below must see the mixed results, not old ones
    mixed = run_server_mixed(reqs, np.zeros(count), cell=cell, rounds=rounds,
                             pool_bytes=pool_bytes)
    mixed["max_rel_diff_served_vs_alone"] = check_against_alone(reqs, cell=cell)
    out["mixed_fp32_polish_saturated"] = mixed
    say(f"serve: saturated, FP32 + FP64 polish {mixed['requests_per_s']:.1f} req/s, "
        f"max rel diff {mixed['max_rel_diff_served_vs_alone']:.1e}")
    rate = seq_fraction * mixed["requests_per_s"]
    mp = run_server_mixed(reqs, poisson_arrivals(count, rate), cell=cell, rounds=rounds,
                          pool_bytes=pool_bytes)
    mp["arrival_rate_per_s"] = rate
    out["mixed_fp32_polish_poisson"] = {str(seq_fraction): mp}
    say(f"serve: FP32 + polish at {seq_fraction}x: p50 {mp['p50_ms']:.1f} p99 {mp['p99_ms']:.1f}")
    seq_sat = run_sequential(reqs, np.zeros(count), cell=cell)
    out["one_at_a_time_saturated"] = seq_sat
    say(f"serve: one-at-a-time {seq_sat['requests_per_s']:.1f} req/s")
    rate = seq_fraction * sat["requests_per_s"]
    seq = run_sequential(reqs, poisson_arrivals(count, rate), cell=cell)
    seq["arrival_rate_per_s"] = rate
    out["one_at_a_time_poisson"] = {str(seq_fraction): seq}
    say(f"serve: one-at-a-time at {seq_fraction}x: p50 {seq['p50_ms']:.1f} p99 {seq['p99_ms']:.1f}")
    del reqs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rounds", type=int, default=8, help="worklist rounds per server step")
    ap.add_argument("--cell", type=int, default=8)
    ap.add_argument("--pool-gib", type=float, default=16.0)
    a = ap.parse_args()
    res = serve_benchmark(a.requests, a.rounds, a.cell, pool_bytes=int(a.pool_gib * (1 << 30)),
                          log=sys.stderr)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
