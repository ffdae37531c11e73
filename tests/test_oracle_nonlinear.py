"""Pins of the global-local loop for solution-dependent coefficients
(Algorithm 2; appendix on nonlinear S-P-T PDEs): a manufactured field the
discrete space holds exactly is a fixed point of the loop and is reached with
one mode; with zero slopes the loop is Algorithm 1 on the linear problem; the
TD inner product equals the dense one."""
import numpy as np

import taps_workloads as W
from oracle import als, fulltensor, nonlinear, problems


def _poly_case(**kw):
    return W.nonlinear_heat(9, 6, 6, 7, M=1, Lx=1.0, Ly=1.0, H=0.5, T=1.0, source="poly", amp=20.0,
                            m_k=1e-3, n_k=1e-2, m_c=1e-3, n_c=2e-2, **kw)


def test_manufactured_field_is_reached():
    # u = a x (1 - x) t: degree 2 in x, 1 in t, zero at x = 0, 1 and t = 0; the
    # load is d/dt((m_c u + n_c) u) - d/dx((m_k u + n_k) du/dx) written out, so
    # a wrong product rule in W_G, a misplaced weight or a dropped m_k term
    # would move the fixed point
    c = _poly_case()
    dims = problems.dims_of(c)
    U0 = W.initial_factors(c.axes, 1, 3)
    U, V, ch = nonlinear.global_local(c, dims, U0, Rc=1, outer=25, sweeps=3, comp_sweeps=3)
    u = fulltensor.td_tensor(U)
    x, t = dims[0].nodes, dims[3].nodes
    ref = np.einsum("i,j,k,l->ijkl", 20 * x * (1 - x), np.ones(6), np.ones(6), t)
    assert np.abs(u - ref).max() < 1e-9 * np.abs(ref).max()
    assert ch[-1] <= 1e-7 and ch[1] > 1e-4


def test_zero_slopes_give_the_linear_problem():
    c = W.nonlinear_heat(10, 8, 6, 9, M=3, Lx=2.0, Ly=2.0, H=0.5, T=0.004, radius=0.3, speed=200.0, y0=1.0,
                         x_start=0.5, m_k=0.0, m_c=0.0)
    dims = problems.dims_of(c)
    U0 = W.initial_factors(c.axes, 3, 4)
    U, V, ch = nonlinear.global_local(c, dims, U0, Rc=1, outer=1, sweeps=2)
    lin = nonlinear.coefficient_problem(c, dims, None)
    Ul = [u.copy() for u in U0]
    for _ in range(2):
        als.sweep(lin, Ul)
        als.balance(Ul)
    for a, b in zip(U, Ul):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_td_inner_is_the_mass_inner_product():
    c = _poly_case()
    dims = problems.dims_of(c)
    rng = np.random.Generator(np.random.PCG64(2))
    A = [rng.standard_normal((D.n, 3)) for D in dims]
    B = [rng.standard_normal((D.n, 2)) for D in dims]
    Mk = [D.matrix("mass").toarray() for D in dims]
    ta, tb = fulltensor.td_tensor(A), fulltensor.td_tensor(B)
    dense = np.einsum("abcd,ai,bj,ck,dl,ijkl->", ta, *Mk, tb)
    assert abs(nonlinear.td_inner(dims, A, B) - dense) < 1e-12 * abs(dense)
