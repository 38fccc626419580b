"""Pins of the serial FP64 oracle against what the paper and the mathematics fix.

The oracle (``oracle/``) claims to compute the unique solution of the first-order upwind system,
eq. (2) of Section 1.1: at each node outside the exit set, sum over axes of
max(D^-U, -D^+U, 0)^2 = 1/F^2, with values beyond the grid +inf and exit nodes fixed at q.
None of the checks below re-uses the oracle's own local-solve code:

* closed forms of the local solve (hand-derived fixture, tests/golden);
* exact axis values k h/F of a constant-speed point source (bitwise, h a power of two);
* the diagonal closed forms h(1 + 1/sqrt 2) and h(1 + 1/sqrt 2 + 1/sqrt 3);
* the 1D reduction of a plane source: U_i = sum h/F exactly;
* eq. (2) itself, evaluated per node in numpy (residual);
* brute-force Jacobi iteration to an exact fixed point (Section 1.1) on tiny grids;
* invariants: monotone causality, the local bounds s/sqrt(3) <= U - min_nbr <= s, neighbour
  Lipschitz bound, cube symmetry, first-order convergence to |x - x0| as h -> 0;
* planted mistakes in the local solve are caught by these pins.
"""
import math
import os

import numpy as np
import pytest

from paper_1306_4743_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_closed_forms():
    rows = []
    with open(os.path.join(GOLDEN, "local_solve_closed_forms.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split(None, 4)
            m = [float(v) for v in parts[:4]]
            env = {"sqrt": math.sqrt, "inf": math.inf}
            rows.append((*m, float(eval(parts[4], {"__builtins__": {}}, env))))
    return rows


@pytest.mark.parametrize("row", _load_closed_forms())
def test_local_solve_closed_forms(orc, row):
    m0, m1, m2, s, want = row
    got = orc.gamma(m0, m1, m2, s)
    if math.isinf(want):
        assert math.isinf(got)
    else:
        assert abs(got - want) <= 2 * np.spacing(want), (row, got)


def test_local_solve_satisfies_equation(orc):
    """Random inputs: the returned U solves sum max(U-m,0)^2 = s^2 and is its smallest root."""
    rng = np.random.default_rng(11)
    for _ in range(20000):
        m = rng.uniform(0, 3, size=3)
        m[rng.uniform(size=3) < 0.15] = np.inf
        s = rng.uniform(0.01, 2.0)
        u = orc.gamma(*m, s)
        if np.all(np.isinf(m)):
            assert math.isinf(u)
            continue
        d = np.maximum(u - m, 0.0)
        lhs = float(np.sum(d * d))
        assert abs(lhs - s * s) <= 16 * np.finfo(float).eps * s * max(u, s), (m, s, u)
        # smallest root: any smaller value gives a strictly smaller left-hand side
        assert u > np.min(m)
        slack = 4 * np.finfo(float).eps * u
        assert u - np.min(m) <= s + slack
        assert u - np.min(m) >= s / math.sqrt(3) - slack


@pytest.mark.parametrize("n", [17, 33, 65])
def test_axis_values_exact(orc, n):
    """Constant speed, centre source, h = 1/(n-1) a power of two: U at k steps along an axis is
    exactly k h (only one upwind neighbour is smaller there), bitwise."""
    p = W.constant(n)
    U = orc.fmm(p.F, p.h, p.src, p.q)
    c = (n - 1) // 2
    k = np.arange(-c, c + 1)
    want = np.abs(k) * p.h
    assert np.array_equal(U[c, c, :], want)
    assert np.array_equal(U[c, :, c], want)
    assert np.array_equal(U[:, c, c], want)


def test_diagonal_closed_forms(orc):
    p = W.constant(33)
    U = orc.fmm(p.F, p.h, p.src, p.q)
    c, h = 16, p.h
    a2 = h * (1 + 1 / math.sqrt(2))
    a3 = h * (1 + 1 / math.sqrt(2) + 1 / math.sqrt(3))
    for dj, dk in [(1, 1), (-1, 1), (1, -1), (-1, -1)]:
        assert abs(U[c, c + dj, c + dk] - a2) <= 2 * np.spacing(a2)
        assert abs(U[c + dk, c + dj, c] - a2) <= 2 * np.spacing(a2)
    for d in [(1, 1, 1), (-1, 1, 1), (1, -1, -1), (-1, -1, -1)]:
        got = U[c + d[2], c + d[1], c + d[0]]
        assert abs(got - a3) <= 2 * np.spacing(a3)


def test_plane_source_1d_reduction(orc):
    """All nodes with i = 0 are exits with q = 0 and F depends on i only: by symmetry every
    node of a plane i = const has the same value, so only the x-neighbour is upwind and
    U_i = U_{i-1} + h/F_i.  Powers of two make every partial sum exact."""
    nx, ny, nz = 24, 5, 4
    h = 1.0 / 32
    rng = np.random.default_rng(5)
    fx = 2.0 ** rng.integers(-2, 3, size=nx)
    F = np.broadcast_to(fx[None, None, :], (nz, ny, nx)).copy()
    src = np.array([[0, j, k] for k in range(nz) for j in range(ny)], dtype=np.int64)
    U = orc.fmm(F, h, src, np.zeros(len(src)))
    want = np.concatenate([[0.0], np.cumsum(h / fx[1:])])
    for k in range(nz):
        for j in range(ny):
            assert np.array_equal(U[k, j, :], want)


@pytest.mark.parametrize("seed", range(8))
def test_jacobi_fixed_point_matches_fmm(orc, seed):
    """Brute force: Jacobi iteration from +inf to an exact fixed point equals FMM."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 12))
    nx = int(rng.integers(3, 13))
    p = W.random_small(n, seed, n_sources=int(rng.integers(1, 4)), nx=nx, ny=n)
    U = orc.fmm(p.F, p.h, p.src, p.q)
    V, sweeps = orc.jacobi(p.F, p.h, p.src, p.q)
    assert sweeps > 1
    assert np.all(np.isfinite(U))
    rel = np.abs(U - V) / np.maximum(np.abs(V), 1e-300)
    assert rel.max() <= 1e-13


@pytest.mark.parametrize("mk", [
    lambda: W.maze(33, seed=3, n_sources=2),
    lambda: W.oscillatory(17, periods=2),
    lambda: W.checkerboard(13, K=3),
])
def test_jacobi_matches_fmm_structured(orc, mk):
    p = mk()
    U = orc.fmm(p.F, p.h, p.src, p.q)
    V, _ = orc.jacobi(p.F, p.h, p.src, p.q)
    assert np.max(np.abs(U - V) / V.clip(1e-300)) <= 1e-13


@pytest.mark.parametrize("mk", [
    lambda: W.constant(33),
    lambda: W.oscillatory(65),
    lambda: W.curved(33),
    lambda: W.maze(65, seed=3),
    lambda: W.checkerboard(45, K=11),
    lambda: W.random_small(20, 3, n_sources=4),
])
def test_residual_of_eq2(orc, mk):
    """Eq. (2) holds at every non-exit node to rounding; exits hold q exactly; C and numpy
    evaluations of the residual agree."""
    p = mk()
    U = orc.fmm(p.F, p.h, p.src, p.q)
    rho = orc.residual_numpy(p.F, p.h, p.src, U)
    assert rho.max() <= 2e-14
    r_c, nbad = orc.residual(p.F, p.h, p.src, p.q, U, 2e-14)
    assert nbad == 0
    assert abs(r_c - rho.max()) <= 1e-16 + 1e-12 * rho.max()
    assert np.array_equal(U[p.src[:, 2], p.src[:, 1], p.src[:, 0]], p.q)


def test_residual_detects_perturbation(orc):
    p = W.oscillatory(33)
    U = orc.fmm(p.F, p.h, p.src, p.q)
    U2 = U.copy()
    U2[3, 20, 7] *= 1 + 1e-9
    r, nbad = orc.residual(p.F, p.h, p.src, p.q, U2, 1e-12)
    assert r > 1e-9 and nbad >= 1


@pytest.mark.parametrize("mk", [lambda: W.oscillatory(65), lambda: W.maze(65, seed=7)])
def test_bounds_and_causality(orc, mk):
    """At every non-exit node: s/sqrt(3) <= U - min_nbr <= s (monotone causality: the node is
    strictly larger than the neighbours it depends on), and |U_x - U_y| <= s at the larger of
    two neighbours."""
    p = mk()
    U = orc.fmm(p.F, p.h, p.src, p.q)
    s = p.h / p.F.astype(np.float64)
    ms = orc.upwind_minima(U)
    mn = np.minimum(np.minimum(ms[0], ms[1]), ms[2])
    mask = np.ones(U.shape, bool)
    mask[p.src[:, 2], p.src[:, 1], p.src[:, 0]] = False
    d = (U - mn)[mask]
    sm = s[mask]
    tol = 8 * np.finfo(float).eps * U[mask]
    assert np.all(d >= sm / math.sqrt(3) - tol)
    assert np.all(d <= sm + tol)
    for axis in range(3):
        a = np.moveaxis(U, axis, 0)
        sa = np.moveaxis(s, axis, 0)
        diff = a[1:] - a[:-1]
        s_big = np.where(diff > 0, sa[1:], sa[:-1])
        assert np.all(np.abs(diff) <= s_big * (1 + 1e-12) + 8 * np.finfo(float).eps * a[1:])


def test_cube_symmetry(orc):
    """Constant speed and a centre source are invariant under the 48 symmetries of the cube;
    FMM's index tie-break evaluates mirrored nodes in different orders, so agreement is to a
    few ulp rather than bitwise."""
    p = W.constant(33)
    U = orc.fmm(p.F, p.h, p.src, p.q)
    import itertools
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product([False, True], repeat=3):
            V = np.transpose(U, perm)
            for ax, f in enumerate(flips):
                if f:
                    V = np.flip(V, ax)
            assert np.max(np.abs(V - U) / np.maximum(U, p.h)) <= 4e-16 * 8


def test_first_order_convergence(orc):
    """Scheme sanity (not parity): with F = 1 the error against the Euclidean distance to the
    source shrinks as h -> 0 (first-order upwind scheme, O(h log 1/h))."""
    errs = []
    for n in (17, 33, 65, 129):
        p = W.constant(n)
        U = orc.fmm(p.F, p.h, p.src, p.q)
        x = np.arange(n) * p.h - 0.5
        d = np.sqrt(x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2)
        errs.append(np.max(np.abs(U - d)))
    assert all(errs[i + 1] < errs[i] for i in range(3))
    assert errs[-1] < 0.6 * errs[0] and errs[-1] < 0.02


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_planted_mistakes_are_caught(orc, variant):
    """A dropped three-term branch (1), the wrong root (2) or the cancellation-prone expanded
    discriminant (3) in the local solve must fail at least one pin above."""
    caught = []
    p = W.constant(33)
    U = orc.fmm_planted(p.F, p.h, p.src, p.q, variant)
    c, h = 16, p.h
    a3 = h * (1 + 1 / math.sqrt(2) + 1 / math.sqrt(3))
    caught.append(abs(U[c + 1, c + 1, c + 1] - a3) > 2 * np.spacing(a3))
    big = W.oscillatory(65)
    Ub = orc.fmm_planted(big.F, big.h, big.src, big.q, variant)
    caught.append(orc.residual_numpy(big.F, big.h, big.src, Ub).max() > 2e-14)
    assert any(caught), variant


def test_unreachable_and_invalid(orc):
    p = W.constant(9)
    with pytest.raises(ValueError):
        orc.fmm(p.F, p.h, np.array([[9, 0, 0]]), [0.0])
    with pytest.raises(ValueError):
        orc.fmm(p.F, p.h, p.src, [-1.0])
    F = p.F.copy()
    F[0, 0, 0] = 0.0
    with pytest.raises(ValueError):
        orc.fmm(F, p.h, p.src, p.q)
    # no sources: everything unreachable
    U = orc.fmm(p.F, p.h, np.zeros((0, 3), np.int64), np.zeros(0))
    assert np.all(np.isinf(U))


def test_duplicate_sources_keep_min(orc):
    p = W.constant(9)
    src = np.array([[4, 4, 4], [4, 4, 4], [0, 0, 0]])
    U = orc.fmm(p.F, p.h, src, [0.5, 0.25, 0.0])
    assert U[4, 4, 4] == 0.25 and U[0, 0, 0] == 0.0


def test_progress_variant_is_the_same_fmm(orc, capfd):
    """The FMM with progress lines returns the plain FMM's array bit for bit and reports every
    `progress` accepted nodes on stderr."""
    p = W.oscillatory(33)
    want = orc.fmm(p.F, p.h, p.src, p.q)
    got = orc.fmm(p.F, p.h, p.src, p.q, progress=4096)
    assert np.array_equal(got, want)
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("oracle FMM:")]
    assert len(lines) == 33 ** 3 // 4096
    assert lines[-1] == f"oracle FMM: {len(lines) * 4096} of {33 ** 3} nodes accepted"


def _diagonal_plane_source(n: int):
    """F = 1, h = 1/(n - 1), exits with q = 0 on every node of the plane i + j + k = n - 1."""
    K = n - 1
    src = np.array([(i, j, K - i - j) for i in range(n) for j in range(n) if 0 <= K - i - j < n],
                   dtype=np.int64)
    return np.ones((n, n, n)), 1.0 / (n - 1), src, np.zeros(len(src)), K


def _diagonal_layer_error(U, h, K, n):
    """Largest relative deviation from |m| h / sqrt(3) over the nodes m layers off the plane
    whose three upwind neighbours lie one layer closer (far side: i, j, k >= m; near side:
    i, j, k <= n - 1 - |m|), and how many such nodes there are."""
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    m = i + j + k - K
    far = (m > 0) & (np.minimum(np.minimum(i, j), k) >= m)
    near = (m < 0) & (np.maximum(np.maximum(i, j), k) <= n - 1 + m)
    sel = far | near
    want = np.abs(m[sel]) * h / math.sqrt(3.0)
    return float(np.max(np.abs(U[sel] - want) / want)), int(sel.sum())


def test_diagonal_plane_source_closed_form(orc):
    """A node m layers off an exit plane i + j + k = const whose three upwind neighbours all lie
    one layer closer has three equal axis values a, so eq. (2) gives U = a + h/(F sqrt(3)) (the
    three-term case), and by induction U = |m| h / sqrt(3) exactly up to the square root's
    rounding: the three-term branch along chains of up to 16 nodes, on both sides of the plane.
    A dropped three-term branch or the wrong root fails it (pinned below)."""
    n = 17
    F, h, src, q, K = _diagonal_plane_source(n)
    err, count = _diagonal_layer_error(orc.fmm(F, h, src, q), h, K, n)
    assert count > 500
    assert err <= 2.0 ** -50, err
    for variant in (1, 2):
        bad, _ = _diagonal_layer_error(orc.fmm_planted(F, h, src, q, variant), h, K, n)
        assert bad > 1e-3, (variant, bad)


def test_axis_pair_plane_source_closed_form(orc):
    """Exits on the plane i + j = n - 1 through every k (F = 1, q = 0): a node m layers off it
    whose x and y upwind neighbours both lie one layer closer has two equal axis values a, and
    its z neighbours lie in its own layer, so they add nothing (they sit exactly where eq. (2)
    switches from two to three terms): U = a + h/(F sqrt(2)), and by induction |m| h / sqrt(2)
    up to rounding -- the two-term branch and the tie between two and three terms."""
    n = 17
    K, h = n - 1, 1.0 / (n - 1)
    src = np.array([(i, K - i, k) for i in range(n) for k in range(n)], dtype=np.int64)
    F, q = np.ones((n, n, n)), np.zeros(len(src))
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    m = i + j - K
    sel = ((m > 0) & (np.minimum(i, j) >= m)) | ((m < 0) & (np.maximum(i, j) <= n - 1 + m))
    want = np.abs(m[sel]) * h / math.sqrt(2.0)
    U = orc.fmm(F, h, src, q)
    assert sel.sum() > 4000
    assert float(np.max(np.abs(U[sel] - want) / want)) <= 2.0 ** -50
    bad = orc.fmm_planted(F, h, src, q, 2)  # the wrong root
    assert float(np.max(np.abs(bad[sel] - want) / want)) > 1e-3
