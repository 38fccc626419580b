"""Properties of eq. (2) that hold at any size, checked on the GPU without the oracle.

* Mirroring an axis, or permuting the axes, of the speeds and the exits mirrors / permutes the
  discrete solution (the update of Section 1.1 treats the six directions alike).  The kernels
  do not: they sweep in eight reflected directions, stage six faces and lay cells out with a
  halo, so a wrong reflection, face or stride shows up as a broken symmetry.
* F -> 2F gives U -> U / 2, and h -> 2h with q -> 2q gives U -> 2U (s = h/F scales by a power
  of two, so every local solve scales exactly; only the rounding of the order of the updates
  may differ).
Compared to 1e-13 relative with identical +inf masks, at 129^3 in the three schedules and on the
513^3 maze.
"""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1306_4743_amd import eik
    eik.load()
    return torch.device("cuda:0")


def solve(dev, F, h, src, q, **kw):
    import torch
    from paper_1306_4743_amd import eik
    u = eik.solve(torch.from_numpy(np.ascontiguousarray(F)).to(dev), h, src, q, **kw)
    rc, _ = eik.status()
    assert rc == 0
    return u.cpu().numpy()


def close(a, b):
    assert np.array_equal(np.isinf(a), np.isinf(b)), "+inf masks differ"
    fin = np.isfinite(a) & (a > 0)
    rel = float(np.max(np.abs(a[fin] - b[fin]) / a[fin]))
    assert rel <= TOL, rel
    return rel


def transformed(p, perm, flip):
    """Speeds and exits of problem p with the axes (x, y, z) permuted by perm (new axis a is old
    axis perm[a]) and then the new axes in flip mirrored; returns (F', src', back) where back
    maps a solution on the new grid to the old one."""
    F = p.F  # [z][y][x]
    nx, ny, nz = F.shape[2], F.shape[1], F.shape[0]
    old_dims = (nx, ny, nz)
    # numpy axis of coordinate a (x=0, y=1, z=2) is 2 - a
    Fp = np.transpose(F, [2 - perm[2], 2 - perm[1], 2 - perm[0]])
    for a in flip:
        Fp = np.flip(Fp, axis=2 - a)
    src = p.src[:, list(perm)].copy()
    new_dims = tuple(old_dims[perm[a]] for a in range(3))
    for a in flip:
        src[:, a] = new_dims[a] - 1 - src[:, a]

    def back(U):
        for a in flip:
            U = np.flip(U, axis=2 - a)
        inv = [perm.index(a) for a in range(3)]
        return np.transpose(U, [2 - inv[2], 2 - inv[1], 2 - inv[0]])
    return np.ascontiguousarray(Fp), src, back


CASES = [((0, 1, 2), (0,)), ((0, 1, 2), (2,)), ((0, 1, 2), (0, 1, 2)), ((2, 1, 0), ()),
         ((1, 0, 2), (1,)), ((1, 2, 0), (0, 2))]


@pytest.mark.parametrize("perm,flip", CASES)
@pytest.mark.parametrize("cell,schedule", [(8, 0), (4, 0), (8, 2), (8, 3)])
def test_mirror_and_permutation_invariance(dev, cell, schedule, perm, flip):
    p = W.maze(129, seed=6, n_sources=3)
    # a box that is not a cube, so a permutation changes the cell grid too
    p.F = np.ascontiguousarray(p.F[:, :97, :113])
    p.src = np.array([[10, 20, 30], [100, 90, 5], [60, 7, 120]], dtype=np.int64)
    p.q = np.array([0.0, 0.01, 0.02])
    ref = solve(dev, p.F, p.h, p.src, p.q, cell=cell, schedule=schedule)
    Fp, srcp, back = transformed(p, perm, flip)
    got = back(solve(dev, Fp, p.h, srcp, p.q, cell=cell, schedule=schedule))
    close(ref, got)


@pytest.mark.parametrize("cell", [8, 4])
def test_power_of_two_scaling(dev, cell):
    p = W.oscillatory(129, periods=3)
    ref = solve(dev, p.F, p.h, p.src, p.q, cell=cell)
    close(ref / 2.0, solve(dev, 2.0 * p.F, p.h, p.src, p.q, cell=cell))
    close(2.0 * ref, solve(dev, p.F, 2.0 * p.h, p.src, 2.0 * p.q, cell=cell))


def test_maze_513_mirrored(dev):
    """The benchmark's workload at full size, mirrored in x and with y and z exchanged, in the
    benchmark's configuration."""
    p = W.maze(513, seed=3)
    ref = solve(dev, p.F, p.h, p.src, p.q, cell=8)
    Fp, srcp, back = transformed(p, (0, 2, 1), (0,))
    del p.F
    got = back(solve(dev, Fp, p.h, srcp, p.q, cell=8))
    rel = close(ref, got)
    print(f"513^3 maze mirrored and transposed: max rel diff {rel:.2e}", flush=True)
