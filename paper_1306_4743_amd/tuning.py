"""Persistent autotuning: picks of ``eik_autotune`` (single solves) and of a server sweep (request
streams), kept in a JSON file keyed by problem class.

The best cell size, in-cell solver, worker count and band width depend on the problem (the
paper finds the best cell size problem-dependent, Section 6), so they are measured once per
problem class and reused:

* a single-solve key is (size class, speed class, mode): the size class is the longest side
  rounded up to a power of two; the speed class is "constant" (max F = min F), "smooth" (max/min
  <= 10) or "contrast" (max/min > 10), taken from the speeds on the device; the mode is the
  arithmetic mode;
* a server key names the stream (its sizes, speed class, mode) and holds the cell size and the
  worklist rounds per server step that served a sample of it fastest.

The cache holds configuration only; every solve still runs in the HIP library.
"""
from __future__ import annotations

import json
import math
import os
import time

DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "eik_mi355x_tuning.json")


def size_class(dims) -> int:
    """Longest side rounded up to a power of two."""
    n = max(int(d) for d in dims)
    return 1 << max(0, math.ceil(math.log2(n)))


def speed_class(F) -> str:
    """'constant', 'smooth' (max/min <= 10) or 'contrast', from the speeds (torch tensor)."""
    fmin = float(F.min())
    fmax = float(F.max())
    if fmax == fmin:
        return "constant"
    return "smooth" if fmax <= 10.0 * fmin else "contrast"


def solve_key(dims, F, mode: int) -> str:
    return f"solve/n{size_class(dims)}/{speed_class(F)}/mode{int(mode)}"


class TuneCache:
    """A JSON file of tuned configurations: {key: {config..., "measured": {...}}}."""

    def __init__(self, path: str = DEFAULT_PATH):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, entry: dict):
        self.data[key] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def tuned_solve_options(F, h, idx3, q, mode: int = 0, cache: TuneCache | None = None,
                        reps: int = 2):
    """Options (cell, inner, workers, delta) for problems of this class: from the cache, or
    measured with ``eik_autotune`` on this problem and stored.  Returns (options dict, key,
    whether it was measured now)."""
    from . import eik
    cache = cache or TuneCache()
    nz, ny, nx = F.shape
    key = solve_key((nx, ny, nz), F, mode)
    hit = cache.get(key)
    if hit is not None:
        return {k: hit[k] for k in ("cell", "inner", "workers", "delta")}, key, False
    best, table = eik.autotune(F, h, idx3, q, reps=reps)
    entry = {k: best[k] for k in ("cell", "inner", "workers", "delta")}
    entry["measured"] = {"ms": best["ms"], "configs_tried": len(table),
                         "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    cache.put(key, entry)
    return {k: entry[k] for k in ("cell", "inner", "workers", "delta")}, key, True


def server_key(sizes, speed: str, mode: int) -> str:
    return f"server/sizes{'-'.join(str(s) for s in sizes)}/{speed}/mode{int(mode)}"


def tune_server(reqs, cells=(8, 4, 16), rounds=(4, 8, 16, 32), sample: int = 96,
                pool_bytes: int = 32 << 30, log=None):
    """Serves the first `sample` requests of a stream, all arriving at once, through a server of
    every (cell, rounds per step) configuration; returns (best config, table) where the table
    lists requests/s per configuration."""
    import numpy as np
    from . import serve
    sub = reqs[:sample]
    table = []
    for cell in cells:
        for r in rounds:
            serve.run_server(sub[:8], np.zeros(8), cell=cell, rounds=r, pool_bytes=pool_bytes)
            res = serve.run_server(sub, np.zeros(len(sub)), cell=cell, rounds=r,
                                   pool_bytes=pool_bytes)
            table.append({"cell": cell, "rounds_per_step": r,
                          "requests_per_s": res["requests_per_s"]})
            if log:
                print(f"tune server: cell {cell} rounds {r}: "
                      f"{res['requests_per_s']:.1f} req/s", file=log, flush=True)
    best = max(table, key=lambda t: t["requests_per_s"])
    return {"cell": best["cell"], "rounds_per_step": best["rounds_per_step"]}, table


def tuned_server_config(reqs, sizes, mode: int = 0, cache: TuneCache | None = None,
                        log=None, **kw):
    """The server configuration for a stream: from the cache, or measured with ``tune_server``
    on a sample of it and stored.  Returns (config, key, table or None)."""
    cache = cache or TuneCache()
    speed = speed_class(reqs[0].F)
    key = server_key(sizes, speed, mode)
    hit = cache.get(key)
    if hit is not None:
        return {k: hit[k] for k in ("cell", "rounds_per_step")}, key, None
    best, table = tune_server(reqs, log=log, **kw)
    cache.put(key, dict(best, table=table, when=time.strftime("%Y-%m-%d %H:%M:%S")))
    return best, key, table
