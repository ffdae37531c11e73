"""Pins of the oracle's 1D C-HiDeNN basis against what the paper's definitions fix.

Sec. 2.1: Kronecker delta, partition of unity and reproduction of polynomials
up to order p; special cases that reduce to textbook functions.
"""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import basis

CASES = [(2, 20.0, 2), (2, 20.0, 1), (1, 10.0, 1), (3, 30.0, 3), (2, 20.0, 0), (0, 5.0, 0)]


def _grid(n, nonuniform, seed=0):
    x = np.linspace(0.0, 1.0, n)
    if nonuniform:
        rng = np.random.Generator(np.random.PCG64(seed))
        x[1:-1] += rng.uniform(-0.25, 0.25, n - 2) / (n - 1)
    return x


@pytest.mark.parametrize("s,a,p", CASES)
@pytest.mark.parametrize("nonuniform", [False, True])
def test_partition_of_unity_and_reproduction(s, a, p, nonuniform):
    x = _grid(13, nonuniform)
    pts = np.linspace(0, 1, 157)
    N, B = (m.toarray() for m in basis.shape_matrices(x, s, a, p, pts))
    # reproduction of x^q for q <= p (s = 0 leaves the linear hats: q <= 1)
    for q in range((p if s > 0 else 1) + 1):
        assert np.abs(N @ x ** q - pts ** q).max() < 1e-12
        dq = q * pts ** (q - 1) if q > 0 else 0.0 * pts
        assert np.abs(B @ x ** q - dq).max() < 1e-10


@pytest.mark.parametrize("s,a,p", CASES)
def test_kronecker_delta_and_continuity(s, a, p):
    x = _grid(11, True, seed=3)
    N, _ = basis.shape_matrices(x, s, a, p, x)
    assert np.abs(N.toarray() - np.eye(len(x))).max() < 1e-12
    # C0: limits from both sides of each interior node agree
    eps = 1e-9
    left = basis.shape_matrices(x, s, a, p, x[1:-1] - eps)[0].toarray()
    right = basis.shape_matrices(x, s, a, p, x[1:-1] + eps)[0].toarray()
    assert np.abs(left - right).max() < 1e-6


def test_s0_p0_is_linear_hat():
    x = _grid(9, True, seed=1)
    pts = np.linspace(0, 1, 101)
    N, B = (m.toarray() for m in basis.shape_matrices(x, 0, 3.0, 0, pts))
    for k in range(len(x)):
        hat = np.interp(pts, x, np.eye(len(x))[k])
        assert np.abs(N[:, k] - hat).max() < 1e-14


@pytest.mark.parametrize("s", [1, 2, 3])
def test_boundary_patch_with_p_plus_1_nodes_is_lagrange(s):
    # the truncated patch of node 0 has s+1 nodes; with p = s the patch function
    # is the Lagrange cardinal polynomial on those nodes (independent of the kernel)
    x = _grid(12, True, seed=s)
    js = list(range(s + 1))
    for t in np.linspace(x[0], x[s], 17):
        got_js, W, dW = basis.patch_function(x, 0, s, 20.0, s, t)
        assert got_js == js
        for j in js:
            others = [k for k in js if k != j]
            lag = np.prod([(t - x[k]) / (x[j] - x[k]) for k in others])
            assert abs(W[j] - lag) < 1e-9


@pytest.mark.parametrize("s", [1, 2, 3])
def test_p1_patch_function_is_natural_cubic_spline(s):
    # when a*h is at least twice the patch span every kernel argument stays in
    # the first (cubic) branch, the constant and quadratic parts of the kernel are
    # absorbed by the reproduction conditions, and with linear reproduction the
    # patch interpolant is the cubic polyharmonic = natural cubic spline
    x = _grid(15, True, seed=7)
    i = 7
    js = basis.patch(len(x), i, s)
    xp = x[js]
    ts = np.linspace(xp[0], xp[-1], 23)
    for jj, j in enumerate(js):
        data = np.zeros(len(js))
        data[jj] = 1.0
        spline = CubicSpline(xp, data, bc_type="natural")
        for t in ts:
            _, W, dW = basis.patch_function(x, i, s, 5.0 * s + 2.0, 1, t)
            assert abs(W[jj] - spline(t)) < 1e-9
            assert abs(dW[jj] - spline(t, 1)) < 1e-6


@pytest.mark.parametrize("p", [1, 2])
def test_dilation_inert_when_large(p):
    x = _grid(10, True, seed=2)
    pts = np.linspace(0, 1, 61)
    A = basis.shape_matrices(x, 2, 20.0, p, pts)[0].toarray()
    B = basis.shape_matrices(x, 2, 40.0, p, pts)[0].toarray()
    assert np.abs(A - B).max() < 1e-9


def test_derivative_matches_finite_difference():
    x = _grid(10, True, seed=4)
    pts = np.linspace(0.03, 0.97, 40)
    h = 1e-6
    _, B = basis.shape_matrices(x, 2, 20.0, 2, pts)
    Np = basis.shape_matrices(x, 2, 20.0, 2, pts + h)[0].toarray()
    Nm = basis.shape_matrices(x, 2, 20.0, 2, pts - h)[0].toarray()
    # points chosen away from nodes, where Ntilde is smooth
    assert np.abs((Np - Nm) / (2 * h) - B.toarray()).max() < 1e-5


def test_abs_term_sum_of_reconstruction():
    # sum_m |w_m prod_d Phi_d[i_d, m]| written out by hand on a tiny case; it
    # bounds the reconstructed value and equals it when every term is positive
    from oracle import reconstruct
    P0 = np.array([[1.0, -2.0], [0.5, 3.0]])
    P1 = np.array([[2.0, 1.0], [-1.0, 4.0], [0.25, -0.5]])
    P2 = np.array([[3.0, -1.0]])
    w = np.array([0.5, -2.0])
    idx = np.array([[i, j, 0] for i in range(2) for j in range(3)])
    got = reconstruct.abs_term_sum([P0, P1, P2], idx, w)
    want = [abs(0.5 * P0[i, 0] * P1[j, 0] * 3.0) + abs(-2.0 * P0[i, 1] * P1[j, 1] * -1.0) for i, j, _ in idx]
    assert np.array_equal(got, np.array(want))
    val = reconstruct.reconstruct_points([P0, P1, P2], idx, w)
    assert np.all(np.abs(val) <= got * (1 + 1e-15))
    pos = [np.abs(P0), np.abs(P1), np.abs(P2)]
    assert np.allclose(reconstruct.abs_term_sum(pos, idx), reconstruct.reconstruct_points(pos, idx), rtol=1e-15)
