"""Relative L2 error of a TD field against the closed-form field of the
space-time convergence problem (the paper's space-time L2 error: the L2
norm over the whole space-time domain of u_TD - u_ex over that of u_ex).

Every integral is Gauss quadrature on each dim's elements (five points):
||u||^2 from the Gram products of the factors' values at the Gauss points,
(u, u_ex) from the separable y and z parts times a two-dimensional (x, t)
quadrature of the travelling Gaussian, ||u_ex||^2 likewise."""
import numpy as np

from oracle import problems


def l2_error(case, dims, U):
    dx, dy, dz, dt = dims
    Phi = [np.asarray(D.Ng @ u) for D, u in zip(dims, U)]        # factor values at the Gauss points
    W = [D.wg for D in dims]
    uu = np.ones((U[0].shape[1],) * 2)
    for P, w in zip(Phi, W):
        uu = uu * (P.T @ (w[:, None] * P))
    norm_u = float(np.sum(uu))
    a = 1.0 - np.exp(-case.decay * dt.xg)
    H = a[None, :] * np.exp(-(dx.xg[:, None] - case.speed * dt.xg[None, :] - case.x0) ** 2)   # (x_g, t_g)
    gy = np.exp(-dy.xg ** 2)
    iy = (W[1] * gy) @ Phi[1]
    iz = W[2] @ Phi[2]
    ixt = np.einsum("im,ij,jm->m", W[0][:, None] * Phi[0], H, W[3][:, None] * Phi[3])
    cross = float(np.sum(iy * iz * ixt))
    norm_ex = float(np.sum(W[1] * gy ** 2) * np.sum(W[2]) * (W[0] @ (H ** 2) @ W[3]))
    err2 = max(norm_u - 2.0 * cross + norm_ex, 0.0)
    return np.sqrt(err2 / norm_ex)


def l2_error_dense(case, dims, U):
    """The same on the tensor of Gauss points (small grids only): a check of
    the separated evaluation above."""
    dx, dy, dz, dt = dims
    Phi = [np.asarray(D.Ng @ u) for D, u in zip(dims, U)]
    u = np.einsum("im,jm,km,lm->ijkl", *Phi)
    ex = problems.st_exact(case, dx.xg[:, None, None, None], dy.xg[None, :, None, None], dt.xg[None, None, None, :])
    ex = np.broadcast_to(ex, u.shape)
    w = np.einsum("i,j,k,l->ijkl", *[D.wg for D in dims])
    return np.sqrt(np.sum(w * (u - ex) ** 2) / np.sum(w * ex ** 2))


def spt8_l2_error(case, dims, U):
    """Relative L2 error of a TD field against the eight-dimensional closed
    form over the whole space-parameter-time domain (the paper's S-P-T L2
    error), by Gauss quadrature: Gram products for ||u||^2, separable
    factors times a (k, t) quadrature for the cross term and ||u_ex||^2."""
    dx, dy, dz, dk, dP, dr, dc, dt = dims
    Phi = [np.asarray(D.Ng @ u) for D, u in zip(dims, U)]
    W = [D.wg for D in dims]
    uu = np.ones((U[0].shape[1],) * 2)
    for P, w in zip(Phi, W):
        uu = uu * (P.T @ (w[:, None] * P))
    norm_u = float(np.sum(uu))
    E = lambda v: np.exp(-case.width * v ** 2)
    g = [E(dx.xg), E(dy.xg), np.ones_like(dz.xg), None, dP.xg, dr.xg, dc.xg, None]
    A = 1.0 - np.exp(-case.decay * dk.xg[:, None] * dt.xg[None, :])           # (k_g, t_g)
    cross = np.ones(U[0].shape[1])
    ex2 = 1.0
    for d in (0, 1, 2, 4, 5, 6):
        cross = cross * ((W[d] * g[d]) @ Phi[d])
        ex2 *= float(np.sum(W[d] * g[d] ** 2))
    cross = cross * np.einsum("im,ij,jm->m", W[3][:, None] * Phi[3], A, W[7][:, None] * Phi[7])
    ex2 *= float(W[3] @ (A ** 2) @ W[7])
    err2 = max(norm_u - 2.0 * float(np.sum(cross)) + ex2, 0.0)
    return np.sqrt(err2 / ex2)
