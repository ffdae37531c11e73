"""TD interpolation of the rank-M field (oracle).

Paper Sec. 2.3, TD interpolation with C-HiDeNN: at a point x,
    u(x) = sum_m prod_d ( sum_{I_d} Ntilde^[d]_{I_d}(x_d) U_d[I_d, m] ).
The inner sum is Phi_d = Ntilde_d(pts_d) U_d (points x modes); the outer sum
over modes is accumulated with compensated (Kahan) summation so the FP64 value
is a reference for reduced-precision reconstructions.
"""
import numpy as np

from . import basis


def factor_at(nodes, s, a, p, U, pts):
    """Phi = Ntilde(pts) U  (n_pts x M)."""
    Nm, _ = basis.shape_matrices(nodes, s, a, p, pts)
    return np.asarray(Nm @ U)


def reconstruct_grid(Phis, mode_w=None):
    """Full tensor u[i_1, .., i_D] = sum_m w_m prod_d Phi_d[i_d, m] (Kahan over m)."""
    M = Phis[0].shape[1]
    shape = tuple(P.shape[0] for P in Phis)
    total = np.zeros(shape)
    comp = np.zeros(shape)
    for m in range(M):
        term = np.ones(shape) * (1.0 if mode_w is None else mode_w[m])
        for d, P in enumerate(Phis):
            sh = [1] * len(Phis)
            sh[d] = P.shape[0]
            term = term * P[:, m].reshape(sh)
        y = term - comp
        t = total + y
        comp = (t - total) - y
        total = t
    return total


def reconstruct_points(Phis, idx, mode_w=None):
    """Values at index tuples idx (n_samples x D), Kahan over modes."""
    idx = np.asarray(idx)
    M = Phis[0].shape[1]
    total = np.zeros(len(idx))
    comp = np.zeros(len(idx))
    for m in range(M):
        term = np.ones(len(idx)) * (1.0 if mode_w is None else mode_w[m])
        for d, P in enumerate(Phis):
            term = term * P[idx[:, d], m]
        y = term - comp
        t = total + y
        comp = (t - total) - y
        total = t
    return total


def abs_term_sum(Phis, idx, mode_w=None):
    """sum_m |w_m prod_d Phi_d[i_d, m]| at index tuples (scale of the rounding bound)."""
    idx = np.asarray(idx)
    out = np.zeros(len(idx))
    for m in range(Phis[0].shape[1]):
        term = np.ones(len(idx)) * (1.0 if mode_w is None else mode_w[m])
        for d, P in enumerate(Phis):
            term = term * P[idx[:, d], m]
        out += np.abs(term)
    return out
