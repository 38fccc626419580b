"""A seeded sweep of small random problems against the oracle.

Each case draws grid extents (2..40 per axis, so ragged and degenerate cells appear), i.i.d.
speeds over one of three ranges, 1-6 exits with random q, and a solver configuration (cell size,
in-cell solver, priority band, shuffled pop order, sweep cap, speed dtype, precision mode or a
polish of the FP32 result), and larger grids in a random schedule with or without jittered visit
orders.  The discrete solution of eq. (2) is unique and reached by every
configuration (Section 4), so every case is compared node by node with the serial FMM: same
+inf mask, exits exact, relative error <= 1e-10 (FP32 mode: 4 n 2^-24)."""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = 160


def draw(case: int):
    rng = np.random.default_rng(70_000 + case)
    nx, ny, nz = (int(v) for v in rng.integers(2, 41, size=3))
    lo, hi = [(0.2, 2.0), (0.9, 1.1), (0.01, 5.0)][int(rng.integers(3))]
    F = rng.uniform(lo, hi, size=(nz, ny, nx))
    ns = int(rng.integers(1, 7))
    src = {(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(ns)}
    src = np.array(sorted(src), dtype=np.int64)
    q = rng.uniform(0.0, 0.2, size=len(src))
    h = float(rng.choice([1.0 / 32, 0.1, 0.37]))
    cfg = {
        "cell": int(rng.choice([4, 8])),
        "inner": int(rng.integers(1, 4)),
        "delta": float(rng.choice([0.0, 0.0, 0.05, 0.5])),
        "shuffle": int(rng.integers(0, 2)) * int(rng.integers(1, 1000)),
        "max_sweeps": int(rng.choice([0, 0, 1, 3])),
        "f32": bool(rng.integers(0, 2)),
        "mode": str(rng.choice(["fp64", "fp64", "fp32", "mixed", "polish"])),
    }
    p = W.Problem(f"rand{case}", F.astype(np.float32) if cfg["f32"] else F, h, src, q,
                  cfg["cell"], 0.0, {"workload": "random sweep"})
    return p, cfg


def draw16(case: int):
    """A case of the same recipe with cells of 16 (sweeps or the list relaxation)."""
    p, cfg = draw(90_000 + case)
    cfg["cell"] = 16
    cfg["inner"] = 1 + case % 2
    p.cell = 16
    return p, cfg


@pytest.mark.parametrize("case", range(CASES))
def test_random_configuration_matches_oracle(orc, case):
    run_case(orc, *draw(case))


@pytest.mark.parametrize("case", range(40))
def test_random_configuration_cell16_matches_oracle(orc, case):
    run_case(orc, *draw16(case))


def draw_pair(case: int):
    """A case of the same recipe swept two cells per wave (cells of 4 and 8)."""
    p, cfg = draw(80_000 + case)
    cfg["inner"] = 4
    return p, cfg


@pytest.mark.parametrize("case", range(40))
def test_random_configuration_pair_matches_oracle(orc, case):
    run_case(orc, *draw_pair(case))


def draw_sched(case: int):
    """A larger grid (40..120 nodes per axis, FP32 speeds over [0.2, 2], 1-4 exits) in a random
    schedule -- rounds in one launch, rounds driven from the host, or the round-free ring --
    with or without jittered visit orders, so that the rounds' lists span many lengths against
    the pop segments."""
    rng = np.random.default_rng(300_000 + case)
    nx, ny, nz = (int(v) for v in rng.integers(40, 121, size=3))
    F = rng.uniform(0.2, 2.0, size=(nz, ny, nx)).astype(np.float32)
    ns = int(rng.integers(1, 5))
    src = {(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(ns)}
    src = np.array(sorted(src), dtype=np.int64)
    q = rng.uniform(0.0, 0.2, size=len(src))
    sched = int(rng.choice([0, 0, 2, 3]))
    cfg = {
        "cell": int(rng.choice([4, 8, 8])),
        "inner": int(rng.choice([1, 1, 2, 4])) if sched != 3 else int(rng.choice([1, 2])),
        "delta": 0.0, "shuffle": 0, "max_sweeps": 0, "f32": True, "mode": "fp64",
        "schedule": sched, "jitter": int(rng.choice([0, 0, 1 + case])),
    }
    p = W.Problem(f"sched{case}", F, 1.0 / 64, src, q, cfg["cell"], 0.0,
                  {"workload": "random sweep, schedules"})
    return p, cfg


@pytest.mark.parametrize("case", range(60))
def test_random_schedule_matches_oracle(orc, case):
    run_case(orc, *draw_sched(case))


def run_case(orc, p, cfg):
    import torch
    from paper_1306_4743_amd import eik
    dev = torch.device("cuda:0")
    F = torch.from_numpy(np.ascontiguousarray(p.F)).to(dev)
    kw = dict(cell=cfg["cell"], inner=cfg["inner"], delta=cfg["delta"], shuffle=cfg["shuffle"],
              max_sweeps=cfg["max_sweeps"], schedule=cfg.get("schedule", 0),
              jitter=cfg.get("jitter", 0))
    mode = cfg["mode"]
    if mode == "polish":
        u = eik.solve(F, p.h, p.src, p.q, mode=eik.EIK_MODE_FP32, **kw)
        assert eik.status()[0] == 0
        u = eik.solve(F, p.h, p.src, p.q, u_out=u, u_approx=u, **kw)
    else:
        m = {"fp64": eik.EIK_MODE_FP64, "fp32": eik.EIK_MODE_FP32,
             "mixed": eik.EIK_MODE_MIXED}[mode]
        u = eik.solve(F, p.h, p.src, p.q, mode=m, **kw)
    rc, stats = eik.status()
    assert rc == 0, (cfg, stats)
    got = u.cpu().numpy()
    want = orc.fmm(p.F, p.h, p.src, p.q)
    assert np.array_equal(np.isinf(got), np.isinf(want)), cfg
    s = p.src
    exits = got[s[:, 2], s[:, 1], s[:, 0]]
    if mode == "fp32":
        assert np.array_equal(exits, p.q.astype(np.float32).astype(np.float64)), cfg
        tol = 4.0 * max(p.F.shape) * 2.0 ** -24
    else:
        assert np.array_equal(exits, want[s[:, 2], s[:, 1], s[:, 0]]), cfg
        tol = 1e-10
    fin = np.isfinite(want) & (want > 0)
    if fin.any():
        err = float(np.max(np.abs(got[fin] - want[fin]) / want[fin]))
        assert err <= tol, (cfg, err)
