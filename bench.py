#!/usr/bin/env python3
"""Benchmark: solved nodes/s of the cell-scheduled Eikonal solver on one MI355X.

One step = one complete solve through the C ABI (stage the speeds into the cell-blocked layout,
seed the exit nodes, run the persistent cell-sweep kernel until the worklist is empty, write the
row-major result), with the speed field already resident in HBM.  The default workload is the
513^3 barrier maze (4 exit nodes, cell side 8, FP64 arithmetic, tol 0).

Prints one JSON line with the throughput, the roofline of the dominant kernel (the persistent
solve kernel, timed with HIP events on the stream it runs on) and the serial oracle timed on one
host core on the same workload, whose result the GPU's is compared with node by node.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-node updates/s and solved nodes/s at 1e-10 rel err; serving p50/p99"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP64_VECTOR_PEAK_TF = 78.6   # MI355X FP64 vector, published
# LDS: 256 CUs x 256 bytes per clock x 2.4 GHz.  128 B per clock per CU is the older CDNA
# figure; on this chip a plain 16-byte read stream (libeik_probe.so) already exceeds it (about
# 160 B per clock per CU), consistent with the doubled LDS read path of CDNA4.
LDS_PEAK_GBS = 256 * 256 * 2.4
# The fraction of the HBM roofline the solve kernel is meant to reach on the 513^3 maze; the
# line reports whether it does (it does not: the kernel is bound by the chain of cell hops and
# the length of each visit, not by bandwidth).
TARGET_FRAC = 0.5


def lds_bytes_per_update(s_u: int = 8) -> int:
    """Algorithmic LDS bytes of one local solve in a sweep step: the node, its six neighbours
    and s read, the node written back (the activations of neighbours are extra)."""
    return s_u * 9


def bytes_per_visit(cell: int, s_u: int = 8, s_f: int = 4) -> int:
    """Algorithmic HBM bytes of one cell visit: read the cell and its one-node halo, read the
    speeds, write the cell back: s_u (2 r^3 + 6 r^2) + s_F r^3."""
    r3, r2 = cell ** 3, cell ** 2
    return s_u * (2 * r3 + 6 * r2) + s_f * r3


def measured_traffic(workload_name: str, cell: int):
    """HBM bytes per launch of the solve kernel from the committed FETCH_SIZE / WRITE_SIZE
    summary, scaled by the plain-copy calibration; None unless the summary was taken on the
    kernel source as it is now (sha256 prefix match) and on this workload."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1306_4743_amd", "csrc", "eik_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", f"k_solve_{workload_name}_pmc*.md")):
        for line in open(path):
            if not line.startswith("machine-readable:"):
                continue
            kv = dict(item.split("=", 1) for item in line.split(":", 1)[1].split())
            if kv.get("sha") != sha or cell != 8:
                continue
            return (float(kv["fetch_kib"]) * float(kv["fetch_scale"])
                    + float(kv["write_kib"]) * float(kv["write_scale"])) * 1024.0
    return None


def cell_hop_chain(u, src, cell: int) -> int:
    """Longest chain of cell crossings along the characteristics of the solution u (torch
    float64 [nz, ny, nx] on the device): each node's parent is its smallest axis neighbour (the
    first term of its local solve, always upwind), an edge costs 1 where it crosses a cell face,
    and the chain of a node is the sum along its parents up to an exit (pointer doubling).  A
    cell can only be final after every cell on such a chain before it, and a round moves
    information about one cell (a face published early in a round can be read later in the same
    round, so sometimes further), so the solve needs about this many rounds."""
    import torch
    nz, ny, nx = u.shape
    inf = float("inf")
    idx = torch.arange(u.numel(), device=u.device, dtype=torch.int64).view(nz, ny, nx)
    best = torch.full_like(u, inf)
    parent = idx.clone()
    cross = torch.zeros(u.shape, dtype=torch.int32, device=u.device)
    coord = {2: torch.arange(nx, device=u.device).view(1, 1, nx),
             1: torch.arange(ny, device=u.device).view(1, ny, 1),
             0: torch.arange(nz, device=u.device).view(nz, 1, 1)}
    stride = {2: 1, 1: nx, 0: nx * ny}
    for ax in (0, 1, 2):
        n = u.shape[ax]
        for step in (-1, 1):
            nb = torch.full_like(u, inf)
            dst = [slice(None)] * 3
            srcs = [slice(None)] * 3
            if step < 0:
                dst[ax], srcs[ax] = slice(1, n), slice(0, n - 1)
            else:
                dst[ax], srcs[ax] = slice(0, n - 1), slice(1, n)
            nb[tuple(dst)] = u[tuple(srcs)]
            better = nb < best
            best = torch.where(better, nb, best)
            parent = torch.where(better, idx + step * stride[ax], parent)
            c = coord[ax]
            crosses = (c % cell == 0) if step < 0 else ((c + 1) % cell == 0)
            cross = torch.where(better, crosses.to(torch.int32).expand_as(cross), cross)
            del nb, better
    root = ~(best < u) | ~torch.isfinite(u)  # exits (no smaller neighbour), unreachable nodes
    if len(src):
        s = torch.as_tensor(src, device=u.device)
        root[s[:, 2], s[:, 1], s[:, 0]] = True
    parent = torch.where(root, idx, parent).view(-1)
    cross = torch.where(root, torch.zeros_like(cross), cross).view(-1)
    del best, root, idx
    for _ in range(40):
        cross = cross + cross[parent]
        nxt = parent[parent]
        if torch.equal(nxt, parent):
            break
        parent = nxt
    return int(cross.max())


def workload(name: str):
    from paper_1306_4743_amd import workloads as W
    if name == "maze513":
        return W.maze(513, seed=3)
    if name == "osc257":
        return W.oscillatory(257, periods=4)
    if name == "const65":
        return W.constant(65)
    if name == "maze257":
        return W.maze(257, seed=3)
    raise SystemExit(f"unknown workload {name}")


def _oracle_request(i):
    """One request of the serving stream recipe solved by the oracle (a worker process)."""
    import oracle
    from paper_1306_4743_amd import serve, workloads as W
    n, ns = serve.request_shape(i)
    p = W.maze(n, seed=5000 + i, n_sources=ns)
    t0 = time.perf_counter()
    oracle.fmm(p.F, p.h, p.src, p.q)
    return p.nodes, time.perf_counter() - t0


def cpu_serving_sample(count: int = 48):
    """The oracle on the first `count` requests of the serving stream, one request per host
    core at a time (the serial FMM cannot use more than one core per request)."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_request, range(count))
    wall = time.perf_counter() - t0
    nodes = sum(r[0] for r in res)
    return {"requests": count, "cores": cores, "wall_s": wall, "requests_per_s": count / wall,
            "solved_nodes_per_s": nodes / wall, "cpu_seconds": sum(r[1] for r in res)}


def host_cpu():
    """Model name of the host CPU and the number of cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(args, p, got):
    """The serial oracle (FMM) on the benchmark's own workload: one full solve of the same
    problem (same float32 speeds, same exits) on one host core -- the FMM is serial -- and the
    GPU result of the timed steps compared with it node by node."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    want = oracle.fmm(p.F, p.h, p.src, p.q)
    dt = time.perf_counter() - t0
    fin = np.isfinite(want) & (want > 0)
    rel = float(np.max(np.abs(got[fin] - want[fin]) / want[fin]))
    same_inf = bool(np.array_equal(np.isinf(got), np.isinf(want)))
    s = p.src
    exits_exact = bool(np.array_equal(got[s[:, 2], s[:, 1], s[:, 0]], want[s[:, 2], s[:, 1], s[:, 0]]))
    del want, fin
    model, ncpu = host_cpu()
    serving = cpu_serving_sample() if args.serving_requests > 0 else None
    return {"value": p.nodes / dt, "unit": "solved nodes/s", "cores": 1, "kind": "oracle",
            "serving_sample": serving,
            "sample": f"serial FP64 FMM, one full solve of the benchmark workload itself "
                      f"({p.meta['workload']}, {p.nodes} nodes), {dt:.1f} s on one host core "
                      f"(FMM is serial)",
            "seconds": dt, "host_cpu": model, "host_cores_available": ncpu,
            "gpu_max_rel_err_vs_oracle": rel, "inf_masks_equal": same_inf,
            "exits_exact": exits_exact}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="maze513")
    ap.add_argument("--cell", type=int, default=8)
    ap.add_argument("--delta", type=float, default=0.0)
    ap.add_argument("--inner", type=int, default=0,
                    help="in-cell solver: 0 default, 1 sweeps, 2 active-list, 3 dual sweeps")
    ap.add_argument("--schedule", type=int, default=0,
                    help="0 auto (rounds in one cooperative launch), 1 cooperative, "
                         "2 host-driven rounds, 3 no rounds (ring of queued cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the mixed-size serving stream (0: skip the serving leg)")
    ap.add_argument("--serving-rounds", type=int, default=16,
                    help="worklist rounds per server step in the serving leg (with "
                         "--no-serving-tune)")
    ap.add_argument("--no-serving-tune", action="store_true",
                    help="serve with --cell and --serving-rounds instead of the tuned server "
                         "configuration (tuning cache, measured on a sample of the stream)")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache file (JSON); default: a fresh file for this run")
    ap.add_argument("--precision-n", type=int, default=1025,
                    help="side of the Gaussian-bumps grid of the precision leg (0: skip it)")
    ap.add_argument("--copy-reference-mib", type=int, default=0,
                    help="only run plain device-to-device copies of this many MiB (calibrates "
                         "the HBM byte counters of a profiler against a known size)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent solves shard across GPUs, one process and one server per GPU, with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1306_4743_amd import eik

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_reference_mib:
        n = args.copy_reference_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(max(args.steps, 1)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_read": n * 8, "copy_reference_bytes_written": n * 8,
                          "copies": max(args.steps, 1)}), flush=True)
        return
    eik.load()
    p = workload(args.workload)
    F = torch.from_numpy(p.F).to(dev)
    u = torch.empty(F.shape, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def solve(timing=False):
        eik.solve(F, p.h, p.src, p.q, cell=args.cell, tol=p.tol, u_out=u, delta=args.delta,
                  timing=timing, inner=args.inner, schedule=args.schedule)

    for _ in range(args.warmup):
        solve()
    rc, st = eik.status()
    if rc != 0:
        raise SystemExit(f"warmup solve failed: {eik.strerror(rc)}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solve(timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rc, st = eik.status()
    if rc != 0:
        raise SystemExit(f"timed solve failed: {eik.strerror(rc)}")
    solve_ms, total_ms = eik.kernel_times(args.steps)

    ms_per_step = 1000.0 * wall / args.steps
    value = p.nodes * args.steps / wall
    upd_per_s = st["updates"] / (ms_per_step / 1000.0)
    kern_ms = float(np.mean(solve_ms))
    s_f = 4 if p.F.dtype == np.float32 else 8
    bpv = bytes_per_visit(args.cell, 8, s_f)
    visits = st["visits"]
    achieved = visits * bpv / (kern_ms / 1000.0) / 1e9
    floor_bytes = st["cells"] * bpv
    traffic = measured_traffic(args.workload, args.cell)
    tot_cyc = sum(st[k] for k in ("cycles_pop", "cycles_stage", "cycles_sweep", "cycles_write",
                                  "cycles_wait"))
    phases = {k[7:]: round(st[k] / max(tot_cyc, 1), 4) for k in
              ("cycles_pop", "cycles_stage", "cycles_sweep", "cycles_write", "cycles_wait")}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solved nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.meta["workload"], "grid": list(p.dims), "h": p.h,
                   "cell": args.cell, "tol": p.tol, "sources": int(len(p.src)),
                   "f_dtype": str(p.F.dtype), "delta": args.delta or "inf",
                   "inner": args.inner or "default",
                   "schedule": ["auto", "cooperative", "host loop", "no rounds"][args.schedule]},
        "grid_node_updates_per_s": upd_per_s,
        "visits_per_cell": visits / st["cells"],
        "sweeps_per_visit": st["sweeps"] / max(visits, 1),
        "updates_per_node": st["updates"] / p.nodes,
        "rounds": st["rounds"],
        "solve_kernel_ms": kern_ms,
        "whole_call_ms": float(np.mean(total_ms)),
        "worker_phase_fractions": phases,
        "roofline": {"bound": "hbm", "kernel": "k_solve", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_visit": bpv, "visits_per_launch": visits,
                     "frac_at_one_visit_per_cell": floor_bytes / (kern_ms / 1000.0) / 1e9
                     / HBM_PEAK_GBS,
                     # counter-measured bytes (FETCH_SIZE + WRITE_SIZE, calibrated) per launch
                     # over the same kernel time, when the committed counters match the source
                     "traffic_gbs": (traffic / (kern_ms / 1000.0) / 1e9) if traffic else None,
                     "traffic_frac": (traffic / (kern_ms / 1000.0) / 1e9 / HBM_PEAK_GBS)
                     if traffic else None,
                     "target_frac": TARGET_FRAC,
                     "target_met": achieved / HBM_PEAK_GBS >= TARGET_FRAC},
        "lds_roofline": {"achieved": st["updates"] * lds_bytes_per_update() / (kern_ms / 1000.0)
                         / 1e9, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                         "frac": st["updates"] * lds_bytes_per_update() / (kern_ms / 1000.0) / 1e9
                         / LDS_PEAK_GBS, "bytes_per_update": lds_bytes_per_update()},
    }
    # Latency floor: rounds cannot be fewer than the longest chain of cell crossings, and each
    # round lasts at least one visit.
    chain = cell_hop_chain(u, p.src, args.cell)
    busy = sum(st[k] for k in ("cycles_stage", "cycles_sweep", "cycles_write"))
    visit_us = kern_ms * 1000.0 * st["workers"] * (busy / max(tot_cyc, 1)) / max(visits, 1)
    line["latency_floor"] = {
        "cell_hop_chain": chain, "rounds": st["rounds"], "mean_visit_us": visit_us,
        "floor_ms": (chain + 1) * visit_us / 1000.0,
        "frac": (chain + 1) * visit_us / 1000.0 / kern_ms,
        "visits_per_round_per_worker": visits / max(st["rounds"], 1) / max(st["workers"], 1)}
    from paper_1306_4743_amd import probes
    line["device_probes"] = probes.measure(dev)
    line["roofline"]["frac_of_probe_copy"] = achieved / line["device_probes"]["hbm_copy_gbs"]
    line["lds_roofline"]["frac_of_probe_read"] = (line["lds_roofline"]["achieved"]
                                                  / line["device_probes"]["lds_read_gbs"])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args, p, u.cpu().numpy())
    del F, u
    torch.cuda.empty_cache()
    if args.precision_n > 0:
        line["precision"] = precision_leg(args, dev)
        torch.cuda.empty_cache()
    if args.serving_requests > 0:
        line["serving"] = serving_leg(args)
    print(json.dumps(line), flush=True)


def precision_leg(args, dev):
    """The precision workload: Gaussian bumps (32 bumps, clamp [0.2, 2], centre exit, seed 4)
    at n^3, FP32 speeds, solved in FP64, FP32 and mixed precision; differences to the FP64
    result (which the test suite holds to eq. (2) at every node)."""
    import torch
    from paper_1306_4743_amd import eik, workloads as W
    p = W.bumps(args.precision_n, seed=4, device=dev)
    F = torch.from_numpy(p.F).to(dev)
    nodes = p.nodes
    del p.F
    out = {"workload": f"Gaussian bumps {args.precision_n}^3, 32 bumps, seed 4, FP32 speeds, "
                       f"cell {args.cell}, tol 0"}
    ref = None
    for name, mode in (("fp64", eik.EIK_MODE_FP64), ("fp32", eik.EIK_MODE_FP32),
                       ("mixed", eik.EIK_MODE_MIXED)):
        u = eik.solve(F, p.h, p.src, p.q, cell=args.cell, mode=mode)  # warm-up (workspace)
        eik.status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = eik.solve(F, p.h, p.src, p.q, cell=args.cell, mode=mode, u_out=u, timing=True)
        rc, st = eik.status()
        wall = time.perf_counter() - t0
        if rc != 0:
            raise SystemExit(f"precision leg ({name}) failed: {eik.strerror(rc)}")
        ks, _ = eik.kernel_times(1)
        r = {"ms": 1000.0 * wall, "solved_nodes_per_s": nodes / wall,
             "solve_kernel_ms": float(ks[0]), "visits_per_cell": st["visits"] / st["cells"]}
        if ref is None:
            ref = u
        else:
            fin = ref > 0
            rel = (u[fin] - ref[fin]).abs() / ref[fin]
            r["max_rel_diff_vs_fp64"] = float(rel.max())
            r["mean_rel_diff_vs_fp64"] = float(rel.mean())
            del rel, fin, u
        out[name] = r
    del ref, F
    return out


def serving_leg(args):
    """The mixed-size request stream (33..257 nodes per side, barrier mazes, 1-4 exits) through
    the continuous-batching servers, against one-at-a-time solves of the same stream."""
    from paper_1306_4743_amd import serve
    cache = args.tune_cache
    if cache is None and not args.no_serving_tune:
        import tempfile
        cache = os.path.join(tempfile.mkdtemp(prefix="eik_tune_"), "tuning.json")
    r = serve.serve_benchmark(args.serving_requests, rounds=args.serving_rounds, cell=args.cell,
                              log=sys.stderr, tune=not args.no_serving_tune, tune_cache=cache)
    sat, one = r["saturated"], r["one_at_a_time_saturated"]
    mix = r["mode_mix"]
    pick = ("p50_ms", "p99_ms", "requests_per_s", "arrival_rate_per_s")
    return {
        "workload": f"{r['requests']} requests, n uniform over {r['sizes']}, barrier mazes seed "
                    f"5000+i, 1-4 exits, FP32 speeds, FP64 values, tol 0, inputs resident",
        "rounds_per_step": r["rounds_per_step"], "cell": r["cell"],
        "pool_bytes": r["pool_bytes"], "tuned_configuration": r["tuned"],
        "mode_mix": {
            "modes": f"fair coin per request: FP64 or FP32 + FP64 polish "
                     f"({mix['saturated']['polish_requests']} of {r['requests']} polish)",
            "saturated_requests_per_s": mix["saturated"]["requests_per_s"],
            "saturated_solved_nodes_per_s": mix["saturated"]["solved_nodes_per_s"],
            "max_rel_diff_served_vs_alone": mix["saturated"]["max_rel_diff_served_vs_alone"],
            "poisson": {f: {k: v[k] for k in pick} for f, v in mix["poisson"].items()},
            "one_at_a_time_requests_per_s": mix["one_at_a_time_saturated"]["requests_per_s"],
        },
        "fp64": {
            "saturated_requests_per_s": sat["requests_per_s"],
            "saturated_solved_nodes_per_s": sat["solved_nodes_per_s"],
            "max_rel_diff_served_vs_alone": r["max_rel_diff_served_vs_alone"],
            "poisson": {f: {k: v[k] for k in pick} for f, v in r["poisson"].items()},
            "one_at_a_time_requests_per_s": one["requests_per_s"],
            "one_at_a_time_solved_nodes_per_s": one["solved_nodes_per_s"],
            "one_at_a_time_poisson": {f: {k: v[k] for k in pick}
                                      for f, v in r["one_at_a_time_poisson"].items()},
        },
        "all_fp32_polish_saturated_requests_per_s":
            r["mixed_fp32_polish_saturated"]["requests_per_s"],
        "fp32_mode_saturated_requests_per_s": r["saturated_fp32_mode"]["requests_per_s"],
    }


if __name__ == "__main__":
    main()
