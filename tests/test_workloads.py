"""The seeded input generators: determinism, the maze recipe, and the device-side maze builder
being bit-identical to the host one (both solvers and the serving stream rely on that)."""
import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W


@pytest.mark.parametrize("n,seed,ns", [(33, 5000, 1), (65, 5001, 4), (49, 22, 2), (97, 3, 4)])
def test_maze_torch_matches_numpy(n, seed, ns):
    import torch
    p = W.maze(n, seed=seed, n_sources=ns)
    F, h, src, q = W.maze_torch(n, seed, ns, torch.device("cpu"))
    assert F.dtype == torch.float32 and tuple(F.shape) == p.F.shape
    assert np.array_equal(F.numpy(), p.F)
    assert np.array_equal(src, p.src) and np.array_equal(q, p.q) and h == p.h


def test_maze_recipe():
    """513^3 maze: 18 slabs of thickness 4 with two 16x16 openings each, speeds {0.01, 1} in
    FP32, four distinct sources outside the barriers with q = 0."""
    L = W.maze_layout(513, 3, 4)
    assert L["thickness"] == 4 and L["gap"] == 16 and len(L["slabs"]) == 18
    assert all(len(h) == 2 for _, _, h in L["slabs"])
    starts = sorted({s for _, s, _ in L["slabs"]})
    assert starts == [int(round((m + 1) * 512 / 7)) - 2 for m in range(6)]
    p = W.maze(65, seed=3)
    assert set(np.unique(p.F).tolist()) == {np.float32(0.01), np.float32(1.0)}
    assert len({tuple(s) for s in p.src}) == 4
    for i, j, k in p.src:
        assert p.F[k, j, i] == 1.0
    assert np.all(p.q == 0.0)
    # scaled sizes with floors
    small = W.maze_layout(33, 1, 1)
    assert small["thickness"] == 1 and small["gap"] == 2


def test_generators_deterministic():
    a, b = W.maze(33, seed=9, n_sources=3), W.maze(33, seed=9, n_sources=3)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.src, b.src)
    c = W.maze(33, seed=10, n_sources=3)
    assert not np.array_equal(a.F, c.F) or not np.array_equal(a.src, c.src)


def test_shell_maze_recipe():
    """Four shells of speed 0.001 between radii r0 and r0 + 1/12 (r0 = .3, .5, .7, .9), openings
    x^2 + y^2 < 1/10 on alternating sides, exit at the origin."""
    p = W.shell_maze(65)
    n = 65
    c = np.linspace(-1, 1, n)
    assert p.h == 2.0 / 64 and list(p.src[0]) == [32, 32, 32]
    assert p.F[32, 32, 32] == 1.0
    # along the x axis (y = z = 0) the openings never apply (they need x^2 < 1/10 and z != 0)
    line = p.F[32, 32, :]
    for i, v in enumerate(c):
        in_shell = any(r0 < abs(v) < r0 + 1 / 12 for r0 in (0.3, 0.5, 0.7, 0.9))
        assert line[i] == (np.float32(0.001) if in_shell else 1.0), (i, v)
    # along -z through the first shell's opening (x = y = 0, z < 0): open; along +z: closed
    colz = p.F[:, 32, 32]
    for k, v in enumerate(c):
        r = abs(v)
        if 0.3 < r < 0.3 + 1 / 12:
            assert colz[k] == (1.0 if v < 0 else np.float32(0.001))
        if 0.5 < r < 0.5 + 1 / 12:
            assert colz[k] == (1.0 if v > 0 else np.float32(0.001))
