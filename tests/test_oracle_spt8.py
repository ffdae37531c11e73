"""Pins of the eight-dimensional space-parameter-time convergence problem's
oracle (second results section): the derived source against the PDE applied
to the closed-form field by finite differences (the printed source agrees
with this one), the lifting against the face data, and convergence."""
import numpy as np

import st_error
import taps_workloads as W
from oracle import als, problems


def test_source_is_the_pde_applied_to_the_exact_field():
    c = W.spt8_convergence(6, M=2)
    rng = np.random.Generator(np.random.PCG64(5))
    h = 1e-4
    for _ in range(20):
        x, y = rng.uniform(-1, 1, 2)
        k, P, rho, cp = rng.uniform(1, 2, 4)
        t = rng.uniform(0.01, 0.2)
        u = lambda x, y, t: problems.spt8_exact(c, x, y, k, P, rho, cp, t)
        d1 = lambda f: (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
        d2 = lambda f: (-f(2) + 16 * f(1) - 30 * f(0) + 16 * f(-1) - f(-2)) / (12 * h * h)
        lhs = rho * cp * d1(lambda q: u(x, y, t + q * h)) - k * (d2(lambda q: u(x + q * h, y, t))
                                                                  + d2(lambda q: u(x, y + q * h, t)))
        E = np.exp(-25 * (x * x + y * y))
        a = 1 - np.exp(-15 * k * t)
        printed = 15 * rho ** 2 * cp ** 2 * k * P * np.exp(-15 * k * t) * E + 50 * rho * cp * k * P * a * E * (
            (1 - 50 * x * x) + (1 - 50 * y * y))
        assert abs(lhs - printed) <= 1e-5 * max(1.0, abs(printed))


def test_lifting_carries_the_face_data():
    c = W.spt8_convergence(5, M=2)
    dims = problems.dims_of(c)
    lift = problems.spt8_field_factors(c, dims, [np.zeros((D.n, 0)) for D in dims])
    g = np.einsum("am,bm,cm,dm,em,fm,gm,hm->abcdefgh", *lift)
    nodes = [D.nodes for D in dims]
    grids = np.meshgrid(*nodes, indexing="ij")
    ex = problems.spt8_exact(c, grids[0], grids[1], grids[3], grids[4], grids[5], grids[6], grids[7])
    face = np.ones(g.shape, dtype=bool)
    face[1:-1, 1:-1, 1:-1] = False
    assert np.abs(g[face] - ex[face]).max() < 1e-14 * np.abs(ex).max()
    assert np.all(g[~face] == 0.0)


def test_error_falls_under_refinement():
    errs = []
    for n in (6, 10, 16):
        c = W.spt8_convergence(n, M=6)
        dims = problems.dims_of(c)
        prob = problems.spt8_convergence(c, dims)
        U = W.initial_factors(c.axes, 6, 1)
        for _ in range(4):
            als.sweep(prob, U)
            als.balance(U)
        errs.append(st_error.spt8_l2_error(c, dims, problems.spt8_field_factors(c, dims, U)))
    assert errs[0] > errs[1] > errs[2], errs
