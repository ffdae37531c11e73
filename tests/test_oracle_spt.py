"""Pins of the space-parameter-time oracle problem (Sec. 2.3 variables;
Sec. 2.5 1D integrals, the conductivity through the k-weighted mass)."""
import numpy as np

import taps_workloads as W
from oracle import als, fulltensor, problems, separated


def test_exact_field_reproduced_with_one_mode():
    # u = z (2H - z) t P lies in the discrete space (degree <= 2 per dim) and
    # satisfies the fixed rows, so the Galerkin solution is u itself; a
    # misplaced k weighting, a wrong term coefficient or a transposed time
    # derivative would leave Algorithm 1 at another field
    c = W.spt_slab(7, 6, 8, 7, n_param=6, M=1, seed=4)
    p = problems.spt_polynomial(c)
    U = W.initial_factors(c.axes, 1, 4)
    for _ in range(60):
        als.sweep(p, U)
        als.balance(U)
        if separated.residual_norm(p, U) < 1e-13:
            break
    u = fulltensor.td_tensor(U)
    z, t, P = c.axes[2].nodes(), c.axes[6].nodes(), c.axes[3].nodes()
    ref = np.einsum("a,b,c,d,e,f,g->abcdefg", np.ones(7), np.ones(6), z * (2 * c.height - z), P,
                    np.ones(6), np.ones(6), t)
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


def test_source_at_parameter_nodes_is_the_heat_slab_source():
    # load term (j, l): x and y factors are the heat slab's beam of radius r_l
    # at time node j (times P / P at the power factor), so every index of the
    # (j, l) -> column maps is checked against the plain heat slab
    c = W.spt_slab(14, 11, 9, 7, n_param=6, M=2, seed=1, y0=0.42)
    p = problems.spt_slab(c)
    rn, nr = c.axes[4].nodes(), c.axes[4].n
    for l in (0, 2, 5):
        hc = W.heat_slab(14, 11, 9, 7, M=2, power=1.0, radius=float(rn[l]), y0=0.42, eta=c.eta, depth=c.depth)
        hp = problems.heat_slab(hc)
        for j in range(c.axes[6].n):
            q = j * nr + l
            assert p.load_col[0][q] == q and p.load_col[1][q] == l and p.load_col[6][q] == j
            assert p.load_col[4][q] == l
            np.testing.assert_allclose(p.F[0][:, q], hp.F[0][:, j], rtol=1e-13, atol=1e-13 * np.abs(hp.F[0]).max())
        np.testing.assert_allclose(p.F[1][:, l], hp.F[1][:, 0], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(p.F[2], hp.F[2], rtol=0, atol=0)
    # the P factor integrates P against the basis, the k factor integrates 1
    Pn = c.axes[3].nodes()
    assert abs(np.sum(p.F[3]) - (Pn[-1] ** 2 - Pn[0] ** 2) / 2) < 1e-9
    kn = c.axes[5].nodes()
    assert abs(np.sum(p.F[5]) - (kn[-1] - kn[0])) < 1e-15
