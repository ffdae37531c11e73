"""Pins of the oracle's separated operator, dim solve and Algorithm 1.

What the paper's definitions fix: the projected Galerkin residual of Sec. 2.5
equals the projection of the explicit full-tensor residual; with as many modes
as free nodes one dim solve is the full Galerkin solve; manufactured solutions
inside the discrete space are reproduced exactly; the Galerkin energy does not
rise under subspace iteration on an SPD problem; the energy-norm ordering of
Sec. 2.7; the L2 convergence rate set by p.
"""
import numpy as np
import pytest

import taps_workloads as W
from oracle import als, basis, fulltensor, problems, reconstruct, separated
from oracle.assemble import Dim1D


def _rand_U(prob, M, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    U = []
    for d in range(prob.D):
        u = rng.standard_normal((prob.n[d], M))
        u[list(prob.fixed[d])] = 0.0
        U.append(u)
    return U


def _tiny_heat():
    case = W.heat_slab(8, 7, 6, 7, M=3)
    return case, problems.heat_slab(case)


def test_projected_residual_matches_full_tensor_heat():
    _, prob = _tiny_heat()
    U = _rand_U(prob, 3, 11)
    Rs, _ = separated.residuals(prob, U)
    for d in range(prob.D):
        ref = fulltensor.projected_residual(prob, U, d)
        assert np.linalg.norm(Rs[d] - ref) <= 1e-11 * np.linalg.norm(ref)


def test_projected_residual_matches_full_tensor_poisson():
    case = W.poisson2d(9, M=4)
    prob = problems.poisson2d(case)
    U = _rand_U(prob, 4, 5)
    Rs, _ = separated.residuals(prob, U)
    for d in range(2):
        ref = fulltensor.projected_residual(prob, U, d)
        assert np.linalg.norm(Rs[d] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("dense_limit", [10 ** 9, 0])
def test_dim_solve_backward_error(dense_limit):
    _, prob = _tiny_heat()
    U = _rand_U(prob, 3, 2)
    for d in range(prob.D):
        C = separated.couplings(prob, U, d)
        Q = separated.force(prob, U, d)
        X = separated.solve_dim(prob, d, C, Q, dense_limit=dense_limit)
        free = prob.free(d)
        R = (separated.apply_dim(prob, d, C, X) - Q)[free]
        assert np.linalg.norm(R) <= 1e-12 * np.linalg.norm(Q[free])
        assert np.all(X[~free] == 0.0)


def test_full_rank_2d_one_solve_is_full_galerkin():
    case = W.poisson2d(10, M=9)
    prob = problems.poisson2d(case)
    uf = fulltensor.solve_full(prob)
    U = _rand_U(prob, 9, 1)          # 9 = free nodes of y
    C = separated.couplings(prob, U, 0)
    U[0] = separated.solve_dim(prob, 0, C, separated.force(prob, U, 0))
    assert np.abs(fulltensor.td_tensor(U) - uf).max() <= 1e-11 * np.abs(uf).max()


def test_full_galerkin_by_fast_diagonalisation():
    # second route to the full 2D solution: K_x X M_y + M_x X K_y = F solved in
    # the eigenbasis of the generalised problem K v = lambda M v on free nodes
    case = W.poisson2d(12, M=1)
    prob = problems.poisson2d(case)
    uf = fulltensor.solve_full(prob)
    fr = [prob.free(d) for d in range(2)]
    Kx, Mx = (prob.mats[0][k].toarray()[np.ix_(fr[0], fr[0])] for k in ("stiff", "mass"))
    Ky, My = (prob.mats[1][k].toarray()[np.ix_(fr[1], fr[1])] for k in ("stiff", "mass"))
    F = sum(np.outer(prob.F[0][fr[0], r], prob.F[1][fr[1], r]) for r in range(prob.R))
    from scipy.linalg import eigh
    lx, Vx = eigh(Kx, Mx)
    ly, Vy = eigh(Ky, My)
    G = Vx.T @ F @ Vy
    X = Vx @ (G / (lx[:, None] + ly[None, :])) @ Vy.T
    assert np.abs(X - uf[np.ix_(fr[0], fr[1])]).max() <= 1e-11 * np.abs(uf).max()


def test_rank_one_poisson_reproduced_exactly():
    case = W.poisson2d(16, M=1)
    dims = problems.dims_of(case)
    prob = problems.poisson2d_polynomial(dims)
    U, hist, ok = als.solve(prob, W.initial_factors(case.axes, 1, 0), tol=1e-13, iter_max=50)
    assert ok
    x, y = dims[0].nodes, dims[1].nodes
    u = np.outer(U[0][:, 0], U[1][:, 0])
    assert np.abs(u - np.outer(x * (1 - x), y * (1 - y))).max() < 1e-12


def test_space_time_rank_one_reproduced_exactly():
    x = np.linspace(0, 1, 13)
    t = np.linspace(0, 0.5, 9)
    dx = Dim1D(x, 2, 20.0, 2, 5, fixed=(0, 12))
    dt = Dim1D(t, 1, 20.0, 1, 5, fixed=(0,))
    prob = problems.spacetime_polynomial(dx, dt)
    rng = np.random.Generator(np.random.PCG64(9))
    U0 = [rng.standard_normal((13, 1)), rng.standard_normal((9, 1))]
    U0[0][[0, 12]] = 0.0
    U0[1][0] = 0.0
    U, hist, ok = als.solve(prob, U0, tol=1e-13, iter_max=100)
    assert ok
    u = np.outer(U[0][:, 0], U[1][:, 0])
    assert np.abs(u - np.outer(x * (1 - x), t)).max() < 1e-12


def test_energy_non_increasing_per_dim_solve():
    case = W.poisson2d(24, M=4)
    prob = problems.poisson2d(case)
    U = _rand_U(prob, 4, 3)
    J = separated.energy(prob, U)
    for _ in range(4):
        for d in range(2):
            C = separated.couplings(prob, U, d)
            U[d] = separated.solve_dim(prob, d, C, separated.force(prob, U, d))
            Jn = separated.energy(prob, U)
            assert Jn <= J + 1e-10 * abs(J)   # Gram-expanded J carries rounding
            J = Jn


def _energy_error(dims, U, uex_dx, uex_dy, uex):
    """||grad(u_h - u)||_L2^2 on the Gauss grid (the Poisson energy norm)."""
    x, y = dims
    Nx, Bx = x.Ng.toarray(), x.Bg.toarray()
    Ny, By = y.Ng.toarray(), y.Bg.toarray()
    ux = (Bx @ U[0]) @ (Ny @ U[1]).T
    uy = (Nx @ U[0]) @ (By @ U[1]).T
    X, Y = np.meshgrid(x.xg, y.xg, indexing="ij")
    w = np.outer(x.wg, y.wg)
    return float(np.sum(w * ((ux - uex_dx(X, Y)) ** 2 + (uy - uex_dy(X, Y)) ** 2)))


def test_energy_norm_ordering():
    pi = np.pi
    dux = lambda X, Y: pi * np.cos(pi * X) * np.sin(pi * Y) + (1 - 2 * X) * Y * (1 - Y)
    duy = lambda X, Y: pi * np.sin(pi * X) * np.cos(pi * Y) + X * (1 - X) * (1 - 2 * Y)
    n_el = 8
    # full C-HiDeNN (no decomposition): node values of the full Galerkin solve as a
    # rank-(n) factorisation U_x = I, U_y = u^T
    case = W.poisson2d(n_el, M=5, s=2, p=2)
    dims = problems.dims_of(case)
    prob = problems.poisson2d(case, dims)
    uf = fulltensor.solve_full(prob)
    e_full = _energy_error(dims, [np.eye(n_el + 1), uf.T], dux, duy, None)
    U, _, _ = als.solve(prob, W.initial_factors(case.axes, 5, 0), tol=1e-10, iter_max=100)
    e_taps = _energy_error(dims, U, dux, duy, None)
    lin = W.poisson2d(n_el, M=1, s=0, p=0, a=3.0)
    ldims = problems.dims_of(lin)
    lprob = problems.poisson2d(lin, ldims)
    ul = fulltensor.solve_full(lprob)
    e_fem = _energy_error(ldims, [np.eye(n_el + 1), ul.T], dux, duy, None)
    assert e_full <= e_taps * (1 + 1e-9)
    assert e_taps <= e_fem


def test_l2_convergence_rate_p2():
    errs = []
    els = [8, 16, 32]
    for n_el in els:
        case = W.poisson2d(n_el, M=2)      # the exact field has rank 2
        dims = problems.dims_of(case)
        prob = problems.poisson2d(case, dims)
        U, _, ok = als.solve(prob, W.initial_factors(case.axes, 2, 0), tol=1e-10, iter_max=100)
        assert ok
        x, y = dims
        uh = (x.Ng.toarray() @ U[0]) @ (y.Ng.toarray() @ U[1]).T
        X, Y = np.meshgrid(x.xg, y.xg, indexing="ij")
        ue = problems.poisson2d_exact(X, Y)
        w = np.outer(x.wg, y.wg)
        errs.append(np.sqrt(np.sum(w * (uh - ue) ** 2) / np.sum(w * ue ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.7), (errs, rates)


def test_last_solved_dim_residual_zero_and_balance_keeps_field():
    _, prob = _tiny_heat()
    U = _rand_U(prob, 3, 4)
    als.sweep(prob, U)
    Rs, Qs = separated.residuals(prob, U)
    assert np.linalg.norm(Rs[-1]) <= 1e-12 * np.linalg.norm(Qs[-1])
    before = fulltensor.td_tensor(U)
    als.balance(U)
    after = fulltensor.td_tensor(U)
    assert np.abs(after - before).max() <= 1e-13 * np.abs(before).max()
    norms = np.array([[np.linalg.norm(u[:, m]) for m in range(3)] for u in U])
    assert np.allclose(norms, norms[0][None, :], rtol=1e-13)


def test_reconstruction_at_nodes_is_td_tensor():
    case, prob = _tiny_heat()
    U = _rand_U(prob, 3, 6)
    Phis = [reconstruct.factor_at(ax.nodes(), ax.s, ax.a, ax.p, U[d], ax.nodes())
            for d, ax in enumerate(case.axes)]
    for d in range(4):
        assert np.abs(Phis[d] - U[d]).max() < 1e-12
    full = reconstruct.reconstruct_grid(Phis)
    assert np.abs(full - fulltensor.td_tensor(U)).max() <= 1e-12 * np.abs(full).max()
    idx = np.array([[1, 2, 3, 4], [7, 6, 5, 6], [0, 0, 0, 0]])
    vals = reconstruct.reconstruct_points(Phis, idx)
    assert np.allclose(vals, full[tuple(idx.T)], rtol=1e-14, atol=0)


def test_heat_source_integral():
    # total source power of load term j equals amplitude * (Gaussian area in x, y)
    # * depth (top layer), all in closed form
    from scipy.special import erf
    case = W.heat_slab(200, 150, 60, 5, M=1)
    prob = problems.heat_slab(case)
    amp = 2 * case.eta * case.power / (np.pi * case.radius ** 2 * case.depth)
    s2 = np.sqrt(2.0) / case.radius
    area = lambda c, lo, hi: np.sqrt(np.pi) / (2 * s2) * (erf(s2 * (hi - c)) - erf(s2 * (lo - c)))
    x0 = case.x_start + case.speed * case.axes[3].nodes()
    for j in range(5):
        assert abs(prob.F[0][:, j].sum() - amp * area(x0[j], 0, 1)) < 1e-8 * amp
    assert abs(prob.F[1][:, 0].sum() - area(case.y0, 0, 1)) < 1e-10
    # the top-layer indicator: 5-point Gauss across the step is not exact; within one element
    hz = case.axes[2].hi / (case.axes[2].n - 1)
    assert abs(prob.F[2][:, 0].sum() - case.depth) < hz


def test_heat_operator_rank_one_reproduced_exactly():
    # u = z (2H - z) t lies in the p = 2 space, satisfies the slab's boundary and
    # initial conditions, and is rank one: TAPS with M = 1 reproduces it exactly,
    # which pins the heat term table (rho c_p on the time derivative, k on each
    # stiffness, the time-derivative matrix in t)
    case = W.heat_slab(9, 8, 10, 7, M=1)
    dims = problems.dims_of(case)
    prob = problems.heat_polynomial(case, dims)
    U, hist, ok = als.solve(prob, W.initial_factors(case.axes, 1, 5), tol=1e-13, iter_max=200)
    assert ok
    z, t = dims[2].nodes, dims[3].nodes
    H = case.height
    u = fulltensor.td_tensor(U)
    ref = np.einsum("i,j,k,l->ijkl", np.ones(9), np.ones(8), z * (2 * H - z), t)
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


def test_dim_system_by_complex_schur_route():
    # the fast-diagonalisation reading of a two-kind dim system (Sec. 2.6):
    # A1 X C1^T + A2 X C2^T = Q with (A1, C1) the mass kind; E = C2^T C1^{-T}
    # = Z T Z^H (complex Schur), P = Z Wv (eigenvectors), M banded systems
    # (A1 + lambda_m A2) y_m = (Q C1^{-T} P)_m, X = Re(Y P^{-1}) -- must equal
    # the plain solve of the dim system, non-symmetric time dim included
    from scipy.linalg import schur, solve_triangular
    case = W.heat_slab(10, 9, 8, 9, M=5, seed=3)
    prob = problems.heat_slab(case)
    rng = np.random.Generator(np.random.PCG64(8))
    U = []
    for d in range(prob.D):
        u = rng.standard_normal((prob.n[d], 5))
        u[list(prob.fixed[d])] = 0.0
        U.append(u)
    for d in range(prob.D):
        C = separated.couplings(prob, U, d)
        Q = separated.force(prob, U, d)
        ref = separated.solve_dim(prob, d, C, Q)
        k1 = "mass"
        k2 = [k for k in prob.kinds(d) if k != "mass"][0]
        A1, A2 = prob.mats[d][k1].toarray(), prob.mats[d][k2].toarray()
        fx = list(prob.fixed[d])
        A1[fx, :] = 0.0
        A1[:, fx] = 0.0
        A1[fx, fx] = 1.0
        A2[fx, :] = 0.0
        A2[:, fx] = 0.0
        C1inv = np.linalg.inv(C[k1])
        E = C[k2].T @ C1inv.T
        T, Z = schur(E.astype(complex), output="complex")
        M = E.shape[0]
        Wv = np.eye(M, dtype=complex)
        for k in range(M):
            for i in range(k - 1, -1, -1):
                Wv[i, k] = -(T[i, i + 1:k + 1] @ Wv[i + 1:k + 1, k]) / (T[i, i] - T[k, k])
        P = Z @ Wv
        R = Q.copy()
        R[fx] = 0.0
        R = R @ C1inv.T @ P
        Y = np.column_stack([np.linalg.solve(A1 + T[m, m] * A2, R[:, m]) for m in range(M)])
        X = (Y @ solve_triangular(Wv, np.eye(M), lower=False) @ Z.conj().T).real
        assert np.abs(X - ref).max() <= 1e-10 * np.abs(ref).max(), d


def test_relative_change_by_hand():
    # the stop rule of Sec. 2.6: change of all solution matrices relative to
    # the new ones, sqrt(sum_d ||U_d - U_d^prev||^2 / sum_d ||U_d||^2)
    old = [np.array([[3.0, 0.0]]), np.array([[0.0], [0.0]])]
    new = [np.array([[3.0, 0.0]]), np.array([[4.0], [0.0]])]
    assert als.relative_change(old, new) == pytest.approx(0.8, rel=0, abs=1e-15)
    assert als.relative_change(new, new) == 0.0
    # a swapped argument order is not the same rule
    assert als.relative_change(new, old) == pytest.approx(4.0 / 3.0, abs=1e-15)
