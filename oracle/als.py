"""Subspace iteration, Algorithm 1 of the paper (oracle).

Sec. 2.6: starting from random factors, for each sweep and each dimension d in
order, hold every other factor fixed, solve the linear dim-d system
K^[d](others) U^[d] = Q^[d](others), and use the new U^[d] when forming the
next dimension's system; after each sweep check convergence.

Readings (the paper is silent on them):
  * stop rule: the projected Galerkin residual rho (Sec. 2.5, the block-diagonal
    system; zero exactly at a fixed point of the iteration) at or below tol;
    the paper's "relative change of all solution matrices" is also reported;
  * after each sweep the mode norms are balanced across dimensions (per mode m,
    scale U_e[:, m] by g / ||U_e[:, m]|| with g the geometric mean of the D
    norms; skipped if any norm is below 1e-300).  This leaves the field, and
    hence every later iterate, unchanged in exact arithmetic.
"""
import numpy as np

from . import separated


def balance(U):
    """Equalise per-mode column norms across dimensions in place."""
    D = len(U)
    M = U[0].shape[1]
    for m in range(M):
        norms = np.array([np.linalg.norm(U[e][:, m]) for e in range(D)])
        if np.any(norms < 1e-300):
            continue
        g = np.exp(np.mean(np.log(norms)))
        for e in range(D):
            U[e][:, m] *= g / norms[e]
    return U


def sweep(prob, U):
    """One pass of Algorithm 1 over d = 1..D (in place); returns U."""
    for d in range(prob.D):
        C = separated.couplings(prob, U, d)
        Q = separated.force(prob, U, d)
        U[d] = separated.solve_dim(prob, d, C, Q)
    return U


def relative_change(U_old, U_new):
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(U_old, U_new))
    den = sum(float(np.sum(b * b)) for b in U_new)
    return np.sqrt(num / den) if den > 0 else np.inf


def solve(prob, U0, tol=1e-8, iter_max=500, on_sweep=None):
    """Run Algorithm 1 to tolerance.  Returns (U, history, converged) with
    history = list of (rho, relative change) per sweep."""
    U = [np.array(u, dtype=np.float64, copy=True) for u in U0]
    history = []
    for it in range(iter_max):
        U_old = [u.copy() for u in U]
        sweep(prob, U)
        balance(U)
        rho = separated.residual_norm(prob, U)
        history.append((rho, relative_change(U_old, U)))
        if on_sweep is not None:
            on_sweep(it, U, rho)
        if rho <= tol:
            return U, history, True
    return U, history, False
