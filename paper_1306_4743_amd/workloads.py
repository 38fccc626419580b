"""Seeded synthetic Eikonal problems (speed field F, exit nodes, exit values).

This module only builds inputs: speed arrays and source lists.  It contains none of the
solver's arithmetic, so the GPU solver and the serial oracle can both consume its output as
plain data.  Arrays are indexed ``F[k, j, i]`` (z, y, x) with x fastest, node (i, j, k) at
(i h, j h, k h) on the unit cube, h = 1 / (n - 1).

Workloads (the paper's benchmark problems and the synthetic stand-ins derived from them):

* ``constant``     -- F = 1, one centre source (Section 6, Example 1, with one centre node
                      because the grids here have an odd number of nodes per side).
* ``oscillatory``  -- F = 1 + amp sin(2 pi p x) sin(2 pi p y) sin(2 pi p z) (Section 6,
                      Example 2 has amp = 0.5 and p = 10; the 257^3 benchmark uses p = 4).
* ``curved``       -- Example 3: F = 1 + 0.99 sin(2 pi x) sin(2 pi y) sin(2 pi z).
* ``maze``         -- axis-aligned slowly permeable slab barriers with gaps, a stand-in for
                      the spherical-shell maze of the "maze speed functions" subsection
                      (barriers of low speed whose openings pinch the level sets).
* ``bumps``        -- 1 + a sum of Gaussian bumps, clamped (precision workload).
* ``checkerboard`` -- the K^3 checkerboard with F in {1, 2} ("checkerboard speed functions").
* ``shell_maze``   -- the spherical-shell maze of the "maze speed functions" subsection.

Every generator is deterministic in its arguments (numpy PCG64 seeded generators).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Problem:
    """One Eikonal problem: speeds F[k,j,i], grid step h, exit nodes (i,j,k) and values q."""

    name: str
    F: np.ndarray
    h: float
    src: np.ndarray  # int64 [n, 3] node indices (i, j, k)
    q: np.ndarray  # float64 [n]
    cell: int = 8
    tol: float = 0.0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.F.shape
        return (nx, ny, nz)

    @property
    def nodes(self) -> int:
        return int(self.F.size)


def _grid_h(n: int) -> float:
    return 1.0 / (n - 1)


def centre_source(n: int):
    c = (n - 1) // 2
    return np.array([[c, c, c]], dtype=np.int64), np.zeros(1)


def constant(n: int = 65, cell: int = 8, tol: float = 1e-14, dtype=np.float64) -> Problem:
    """Plain method, small: F = 1, one point source u = 0 at the centre node."""
    src, q = centre_source(n)
    return Problem(f"constant{n}", np.ones((n, n, n), dtype=dtype), _grid_h(n), src, q, cell, tol,
                   {"workload": f"constant speed F=1, {n}^3, centre source"})


def _axis_coords(n: int):
    h = _grid_h(n)
    return np.arange(n, dtype=np.float64) * h


def oscillatory(n: int = 257, periods: float = 4.0, amp: float = 0.5, cell: int = 8,
                tol: float = 0.0, dtype=np.float64) -> Problem:
    """F(x,y,z) = 1 + amp sin(2 pi periods x) sin(2 pi periods y) sin(2 pi periods z),
    evaluated in FP64 at x = i h; one centre source."""
    x = _axis_coords(n)
    sx = np.sin(2.0 * math.pi * periods * x)
    F = 1.0 + amp * (sx[:, None, None] * sx[None, :, None]) * sx[None, None, :]
    src, q = centre_source(n)
    return Problem(f"oscillatory{n}", np.ascontiguousarray(F.astype(dtype)), _grid_h(n), src, q,
                   cell, tol, {"workload": f"oscillatory speed 1+{amp}sin^3 x {periods} periods, "
                                           f"{n}^3, centre source"})


def curved(n: int = 129, cell: int = 8, tol: float = 0.0) -> Problem:
    """Example 3 of the paper: F = 1 + 0.99 sin(2 pi x) sin(2 pi y) sin(2 pi z)."""
    p = oscillatory(n, periods=1.0, amp=0.99, cell=cell, tol=tol)
    p.name = f"curved{n}"
    p.meta["workload"] = f"curved speed 1+0.99 sin^3 (one period), {n}^3, centre source"
    return p


def maze_layout(n: int = 513, seed: int = 3, n_sources: int = 4, slabs_per_axis: int = 6,
                thickness: int | None = None, gap: int | None = None,
                gaps_per_slab: int = 2) -> dict:
    """The random part of the barrier maze, drawn once: slab positions, openings and sources.

    Slab m (m = 0..slabs_per_axis-1) on axis a covers the nodes [s_m, s_m + thickness) along
    a, s_m = round((m+1) (n-1) / (slabs_per_axis+1)) - thickness // 2, across the whole grid in
    the other two axes.  Each slab has ``gaps_per_slab`` openings of gap x gap nodes at uniform
    random in-plane offsets (o1, o2) over the slab's two in-plane axes in increasing order; an
    opening restores F = 1 only inside its own slab.  At n = 513 thickness is 4 and gap 16; at
    other sizes both scale with (n-1)/512, floored at 1 and 2.  Sources: ``n_sources`` distinct
    nodes drawn uniformly among the nodes outside every barrier.
    """
    scale = (n - 1) / 512.0
    if thickness is None:
        thickness = max(1, int(round(4 * scale)))
    if gap is None:
        gap = max(2, int(round(16 * scale)))
    rng = np.random.default_rng(seed)
    slabs = []  # (axis, start, [(o1, o2), ...]) with axis 0 = x, 1 = y, 2 = z
    for axis in range(3):
        for m in range(slabs_per_axis):
            s = int(round((m + 1) * (n - 1) / (slabs_per_axis + 1))) - thickness // 2
            s = min(max(s, 0), n - thickness)
            holes = []
            for _ in range(gaps_per_slab):
                o1 = int(rng.integers(0, n - gap + 1))
                o2 = int(rng.integers(0, n - gap + 1))
                holes.append((o1, o2))
            slabs.append((axis, s, holes))

    def in_barrier(i, j, k):
        p = (i, j, k)
        for axis, s, holes in slabs:
            if not (s <= p[axis] < s + thickness):
                continue
            a, b = [p[x] for x in range(3) if x != axis]
            if not any(o1 <= a < o1 + gap and o2 <= b < o2 + gap for o1, o2 in holes):
                return True
        return False

    src = []
    while len(src) < n_sources:
        i, j, k = (int(v) for v in rng.integers(0, n, size=3))
        if in_barrier(i, j, k) or [i, j, k] in src:
            continue
        src.append([i, j, k])
    return {"n": n, "seed": seed, "thickness": thickness, "gap": gap, "slabs": slabs,
            "slabs_per_axis": slabs_per_axis, "gaps_per_slab": gaps_per_slab,
            "src": np.array(src, dtype=np.int64)}


def _maze_barrier(layout, xp, zeros, ones):
    """Boolean barrier mask [z][y][x] of a layout with array module ``xp`` (numpy or torch)."""
    n, t, gap = layout["n"], layout["thickness"], layout["gap"]
    barrier = zeros((n, n, n))
    for axis, s, holes in layout["slabs"]:
        plane = ones((n, n))  # indexed by the two in-plane axes in increasing order
        for o1, o2 in holes:
            plane[o1:o1 + gap, o2:o2 + gap] = False
        pt = plane.T
        # storage order is [z][y][x]: axis x -> dim 2, y -> dim 1, z -> dim 0
        if axis == 0:    # plane[y, z] -> view [z][y]
            barrier[:, :, s:s + t] |= pt[:, :, None]
        elif axis == 1:  # plane[x, z] -> view [z][x]
            barrier[:, s:s + t, :] |= pt[:, None, :]
        else:            # plane[x, y] -> view [y][x]
            barrier[s:s + t, :, :] |= pt[None, :, :]
    return barrier


def maze(n: int = 513, seed: int = 3, n_sources: int = 4, slabs_per_axis: int = 6,
         thickness: int | None = None, gap: int | None = None, gaps_per_slab: int = 2,
         barrier_speed: float = 0.01, cell: int = 8, tol: float = 0.0,
         dtype=np.float32) -> Problem:
    """Barrier maze: F = 1 except on axis-aligned slabs of speed ``barrier_speed`` with square
    openings (layout in ``maze_layout``), q = 0 at the sources.  F is returned in ``dtype``
    (float32 by default) and both solvers read exactly those values."""
    L = maze_layout(n, seed, n_sources, slabs_per_axis, thickness, gap, gaps_per_slab)
    barrier = _maze_barrier(L, np, lambda sh: np.zeros(sh, dtype=bool),
                            lambda sh: np.ones(sh, dtype=bool))
    F = np.where(barrier, dtype(barrier_speed), dtype(1.0)).astype(dtype)
    return Problem(f"maze{n}", F, _grid_h(n), L["src"], np.zeros(n_sources), cell, tol,
                   {"workload": f"barrier maze {n}^3 ({slabs_per_axis} slabs/axis, thickness "
                                f"{L['thickness']}, {gaps_per_slab} gaps {L['gap']}x{L['gap']}, "
                                f"F=1/{barrier_speed}), {n_sources} sources, seed {seed}",
                    "seed": seed, "thickness": L["thickness"], "gap": L["gap"]})


def maze_torch(n: int, seed: int, n_sources: int, device, barrier_speed: float = 0.01):
    """The same maze built directly in device memory (float32 F, bit-identical to ``maze``).

    Returns (F tensor [n, n, n], h, sources int64 [k, 3], q float64 [k])."""
    import torch
    L = maze_layout(n, seed, n_sources)
    barrier = _maze_barrier(L, torch,
                            lambda sh: torch.zeros(sh, dtype=torch.bool, device=device),
                            lambda sh: torch.ones(sh, dtype=torch.bool, device=device))
    F = torch.where(barrier, torch.tensor(barrier_speed, dtype=torch.float32, device=device),
                    torch.tensor(1.0, dtype=torch.float32, device=device))
    return F.contiguous(), _grid_h(n), L["src"], np.zeros(n_sources)


def shell_maze(n: int = 257, cell: int = 8, tol: float = 0.0, dtype=np.float32,
               barrier_speed: float = 0.001, t: float = 1.0 / 12.0, w: float = 0.1) -> Problem:
    """The spherical-shell maze of the "maze speed functions" subsection of Section 6.

    Domain [-1, 1]^3 with n nodes per side (h = 2 / (n - 1)), one exit node at the origin
    (q = 0).  F = 1 except inside four concentric shells of thickness t with inner radii 0.3,
    0.5, 0.7, 0.9, where F = ``barrier_speed``; each shell has a cylindrical opening
    x^2 + y^2 < w on alternating sides (z < 0 for the first and third, z > 0 for the second and
    fourth).  F is returned in ``dtype`` and both solvers read exactly those values.
    """
    c = np.linspace(-1.0, 1.0, n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    rad = np.sqrt(x * x + y * y + z * z)
    hole = x * x + y * y < w
    barrier = np.zeros((n, n, n), dtype=bool)
    for k, r0 in enumerate((0.3, 0.5, 0.7, 0.9)):
        side = (z < 0) if k % 2 == 0 else (z > 0)
        barrier |= (rad > r0) & (rad < r0 + t) & ~(hole & side)
    F = np.where(barrier, dtype(barrier_speed), dtype(1.0)).astype(dtype)
    m = (n - 1) // 2
    src = np.array([[m, m, m]], dtype=np.int64)
    return Problem(f"shellmaze{n}", F, 2.0 / (n - 1), src, np.zeros(1), cell, tol,
                   {"workload": f"spherical-shell maze {n}^3 on [-1,1]^3 (4 shells, t=1/12, "
                                f"w=1/10, F=1/{barrier_speed}), exit at the origin"})


def bumps(n: int = 1025, seed: int = 4, n_bumps: int = 32, cell: int = 8, tol: float = 0.0,
          dtype=np.float32, device=None) -> Problem:
    """F = clamp(1 + sum_m A_m exp(-|x - c_m|^2 / (2 w_m^2)), 0.2, 2) with c_m ~ U[0,1]^3,
    A_m ~ U[-0.5, 0.5], w_m ~ U[0.02, 0.1]; centre source.  Evaluated in FP64 and stored in
    ``dtype``.  The Gaussian is separable: its per-axis factors are evaluated on the host with
    numpy; the 3-D sum then takes, for each bump, the products (g_z g_y) g_x, the scaling by A_m
    and the addition, each correctly rounded, in that order -- with numpy on the host, or with
    torch on ``device`` (returned as a numpy array) -- so both give the same field bit for bit."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=(n_bumps, 3))
    A = rng.uniform(-0.5, 0.5, size=n_bumps)
    w = rng.uniform(0.02, 0.1, size=n_bumps)
    x = _axis_coords(n)
    g = [[np.exp(-(x - c[m, a]) ** 2 / (2 * w[m] ** 2)) for a in range(3)]
         for m in range(n_bumps)]
    if device is None:
        F = np.ones((n, n, n), dtype=np.float64)
        buf = np.empty_like(F)
        for m in range(n_bumps):
            gx, gy, gz = g[m]
            np.multiply(gz[:, None, None] * gy[None, :, None], gx[None, None, :], out=buf)
            buf *= A[m]
            F += buf
        del buf
        np.clip(F, 0.2, 2.0, out=F)
        F = F.astype(dtype)
    else:
        import torch
        Ft = torch.ones((n, n, n), dtype=torch.float64, device=device)
        buf = torch.empty_like(Ft)
        for m in range(n_bumps):
            gx, gy, gz = (torch.from_numpy(v).to(device) for v in g[m])
            torch.mul(gz[:, None, None] * gy[None, :, None], gx[None, None, :], out=buf)
            buf.mul_(float(A[m]))
            Ft.add_(buf)
        del buf
        Ft.clamp_(0.2, 2.0)
        F = Ft.to(torch.float32 if dtype == np.float32 else torch.float64).cpu().numpy()
        del Ft
    src, q = centre_source(n)
    return Problem(f"bumps{n}", F, _grid_h(n), src, q, cell, tol,
                   {"workload": f"Gaussian bumps {n}^3 ({n_bumps} bumps, clamp [0.2,2]), "
                                f"centre source, seed {seed}", "seed": seed})


def checkerboard(n: int = 89, K: int = 11, cell: int = 8, tol: float = 0.0) -> Problem:
    """K^3 checkerboard: F = 2 on 'black' cubes, 1 on 'white' cubes, centre source."""
    x = _axis_coords(n)
    b = np.minimum((x * K).astype(np.int64), K - 1)
    parity = (b[:, None, None] + b[None, :, None] + b[None, None, :]) % 2
    F = np.where(parity == 0, 2.0, 1.0)
    src, q = centre_source(n)
    return Problem(f"checker{K}_{n}", F, _grid_h(n), src, q, cell, tol,
                   {"workload": f"checkerboard K={K}, {n}^3, centre source"})


def random_small(n: int, seed: int, n_sources: int = 3, fmin: float = 0.2, fmax: float = 2.0,
                 nx: int | None = None, ny: int | None = None) -> Problem:
    """Tiny random problem: F ~ U[fmin, fmax] i.i.d., random distinct sources, q ~ U[0, 0.1]."""
    rng = np.random.default_rng(seed)
    nx = nx or n
    ny = ny or n
    F = rng.uniform(fmin, fmax, size=(n, ny, nx))
    src = set()
    while len(src) < n_sources:
        src.add((int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, n))))
    src = np.array(sorted(src), dtype=np.int64)
    q = rng.uniform(0.0, 0.1, size=len(src))
    return Problem(f"random{nx}x{ny}x{n}_s{seed}", F, 1.0 / max(nx - 1, 1), src, q, 8, 0.0,
                   {"workload": f"random speeds U[{fmin},{fmax}] {nx}x{ny}x{n}", "seed": seed})


def by_name(name: str, **kw) -> Problem:
    table = {"constant": constant, "oscillatory": oscillatory, "curved": curved, "maze": maze,
             "bumps": bumps, "checkerboard": checkerboard, "shell_maze": shell_maze}
    return table[name](**kw)
