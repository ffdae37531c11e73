"""Pins of the space-time convergence problem's oracle (first results
section): the derived source against the PDE applied to the exact field by
finite differences, the nodal lifting against the face data, the separated
L2 error against the dense quadrature, and convergence under refinement."""
import numpy as np

import st_error
import taps_workloads as W
from oracle import als, fulltensor, problems


def test_source_is_the_pde_applied_to_the_exact_field():
    c = W.st_convergence(12, 10, M=4)
    rng = np.random.Generator(np.random.PCG64(3))
    h = 1e-4
    u = lambda x, y, t: problems.st_exact(c, x, y, t)
    for _ in range(20):
        x, y, t = rng.uniform(0, 10), rng.uniform(-5, 5), rng.uniform(0.002, 0.05)
        # fourth-order central differences
        d2 = lambda f: (-f(2) + 16 * f(1) - 30 * f(0) + 16 * f(-1) - f(-2)) / (12 * h * h)
        d1 = lambda f: (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
        ut = d1(lambda k: u(x, y, t + k * h))
        uxx = d2(lambda k: u(x + k * h, y, t))
        uyy = d2(lambda k: u(x, y + k * h, t))
        f = problems.st_source(c, x, y, t)
        assert abs(f - (ut - uxx - uyy)) <= 1e-6 * max(1.0, abs(f))


def test_lifting_carries_the_face_data():
    c = W.st_convergence(9, 7, M=2)
    dims = problems.dims_of(c)
    lift = problems.st_field_factors(c, dims, [np.zeros((D.n, 0)) for D in dims])
    g = fulltensor.td_tensor(lift)
    x, y, z, t = (D.nodes for D in dims)
    ex = problems.st_exact(c, x[:, None, None, None], y[None, :, None, None], t[None, None, None, :])
    ex = np.broadcast_to(ex, g.shape)
    inner = np.zeros(g.shape, dtype=bool)
    inner[1:-1, 1:-1, 1:-1, :] = True
    assert np.abs(g[~inner] - ex[~inner]).max() < 1e-15
    assert np.all(g[inner] == 0.0)


def test_separated_error_equals_dense_quadrature():
    c = W.st_convergence(10, 8, M=3)
    dims = problems.dims_of(c)
    rng = np.random.Generator(np.random.PCG64(4))
    U = [rng.standard_normal((D.n, 3)) * 0.1 for D in dims]
    Uf = problems.st_field_factors(c, dims, U)
    a, b = st_error.l2_error(c, dims, Uf), st_error.l2_error_dense(c, dims, Uf)
    assert abs(a - b) < 1e-10 * b


def test_error_falls_under_refinement():
    errs = []
    for n, nt, M in ((12, 9, 8), (24, 17, 12), (48, 33, 16)):
        c = W.st_convergence(n, nt, M=M)
        dims = problems.dims_of(c)
        prob = problems.st_convergence(c, dims)
        U = W.initial_factors(c.axes, M, 1)
        for _ in range(5):
            als.sweep(prob, U)
            als.balance(U)
        errs.append(st_error.l2_error(c, dims, problems.st_field_factors(c, dims, U)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.02, errs
