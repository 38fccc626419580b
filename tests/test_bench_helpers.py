"""CPU checks of the measurement helpers in bench.py: the algorithmic bytes of a visit, the LDS
bytes of a local solve, and the longest chain of cell crossings of a solution (the latency
floor), on solutions from the oracle whose chains can be counted by hand."""
import numpy as np
import pytest


def test_bytes_per_visit_and_update():
    import bench
    # s_u (2 r^3 + 6 r^2) + s_F r^3 at r = 8, FP64 values, FP32 speeds
    assert bench.bytes_per_visit(8, 8, 4) == 8 * (2 * 512 + 6 * 64) + 4 * 512 == 13312
    assert bench.bytes_per_visit(4, 8, 8) == 8 * (2 * 64 + 6 * 16) + 8 * 64
    assert bench.bytes_per_visit(16, 8, 8) == 8 * (2 * 4096 + 6 * 256) + 8 * 4096 == 110592
    assert bench.lds_bytes_per_update() == 72


def _chain(u, src, cell):
    import torch
    import bench
    return bench.cell_hop_chain(torch.from_numpy(u), src, cell)


def test_cell_hop_chain_corner_source(orc):
    """Corner exit of a 17^3 unit-speed grid: the farthest node (16, 16, 16) is reached through
    two cell faces per axis at r = 8 (16 -> 15 and 8 -> 7), six in all; at r = 4 four per axis,
    at r = 16 one."""
    F = np.ones((17, 17, 17))
    src = np.array([[0, 0, 0]])
    u = orc.fmm(F, 1 / 16, src, np.zeros(1))
    assert _chain(u, src, 8) == 6
    assert _chain(u, src, 4) == 12
    assert _chain(u, src, 16) == 3  # one face per axis (16 -> 15)


def test_cell_hop_chain_line_and_unreachable(orc):
    """A thin 33 x 2 x 2 grid with the exit at x = 0: the chain runs along x, crossing
    32 / r cell faces; a grid without exits has no chain."""
    F = np.ones((2, 2, 33))
    src = np.array([[0, 0, 0]])
    u = orc.fmm(F, 1 / 32, src, np.zeros(1))
    assert _chain(u, src, 8) == 4
    assert _chain(u, src, 4) == 8
    assert _chain(u, src, 16) == 2
    none = np.full((5, 5, 5), np.inf)
    assert _chain(none, np.zeros((0, 3), np.int64), 4) == 0
