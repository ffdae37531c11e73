"""Comparison helpers of the GPU parity tests and the per-case parity bar.

Every FP64 comparison is made twice: in norm (relative Frobenius difference)
and element by element (largest entry difference over the largest reference
entry).  The bar is 1e-10 unless the case itself amplifies rounding more
than that.  Two measures of that amplification are taken on the oracle
alone (nothing from the GPU enters a bar):

* kappa, the largest 1-norm condition estimate (Hager-Higham on a sparse LU)
  of the case's dim systems: a backward-stable solve of a system with
  condition kappa is accurate to about kappa x eps, so two correct FP64
  solvers agree to c x kappa x eps;
* the iteration's own response: Algorithm 1 (Sec. 2.6) carries every
  rounding error of one dim solve into the couplings of the next, so the
  same sweeps are run again with every coupling matrix and force perturbed
  by eta = 1e-14 of its RMS entry (about twice what reordering the sums of
  one contraction moves them by) and the difference this makes is measured.

The bar is max(1e-10, c x kappa x eps, c x response) with c = 10.
"""
import contextlib

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import als, separated

TOL = 1e-10
EPS = np.finfo(np.float64).eps


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def maxrel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0)) if b.size else 0.0


def check(a, b, bar, what=""):
    """Both the norm-wise and the element-wise difference within bar; returns them."""
    r, m = rel(a, b), maxrel(a, b)
    assert r <= bar and m <= bar, f"{what}: rel {r:.3e}, max entry {m:.3e}, bar {bar:.3e}"
    return r, m


@contextlib.contextmanager
def perturbed(eta=1e-14, seed=0):
    """Within the block every dim solve of the oracle (separated.solve_dim,
    which Algorithm 1 and the chain call) first perturbs its couplings and
    force by eta times their RMS entry (Gaussian, seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    exact = separated.solve_dim

    def solve(prob, d, C, Q, *a, **k):
        C = {nm: c + eta * np.sqrt(np.mean(c ** 2)) * rng.standard_normal(c.shape) for nm, c in C.items()}
        Q = Q + eta * np.sqrt(np.mean(Q ** 2)) * rng.standard_normal(Q.shape)
        return exact(prob, d, C, Q, *a, **k)

    separated.solve_dim = solve
    try:
        yield
    finally:
        separated.solve_dim = exact


def perturbed_sweeps(prob, U0, sweeps, eta=1e-14, seed=0):
    """The oracle's Algorithm 1 with every coupling matrix and force perturbed."""
    U = [np.array(u, dtype=np.float64, copy=True) for u in U0]
    with perturbed(eta, seed):
        for _ in range(sweeps):
            als.sweep(prob, U)
            als.balance(U)
    return U


def oracle_sweeps(prob, U0, sweeps):
    """Algorithm 1 on the oracle: factors, rho and relative change after every sweep."""
    U = [np.array(u, dtype=np.float64, copy=True) for u in U0]
    rhos, changes = [], []
    for _ in range(sweeps):
        old = [u.copy() for u in U]
        als.sweep(prob, U)
        als.balance(U)
        rhos.append(separated.residual_norm(prob, U))
        changes.append(als.relative_change(old, U))
    return U, rhos, changes


def sweep_bars(prob, U0, Uo, sweeps, rho_o, change_o, eta=1e-14, c=10.0):
    """Per-case bars after `sweeps` sweeps: relative bar of every dim's factor,
    absolute bar of rho, relative bar of the change, and the kappa used."""
    kappa = max(cond_estimate(prob, d, separated.couplings(prob, Uo, d)) for d in range(prob.D))
    Up = perturbed_sweeps(prob, U0, sweeps, eta)
    floor = max(TOL, c * kappa * EPS)
    f = [max(floor, c * max(rel(a, b), maxrel(a, b))) for a, b in zip(Up, Uo)]
    rho_p = separated.residual_norm(prob, Up)
    r = max(TOL * rho_o, c * abs(rho_p - rho_o), c * kappa * EPS)
    # the change compares two iterates: it moves by about the end point's own
    # perturbation, relative to the change's size
    d_end = max(als.relative_change(Up, Uo), kappa * EPS)
    ch = max(TOL, c * d_end / max(change_o, 1e-300))
    return f, r, ch, kappa


def dim_system_sparse(prob, d, C):
    """The node-major dim-d system sum_k A^k (x) C^k on free rows and columns."""
    free = prob.free(d)
    idx = np.nonzero(free)[0]
    return sp.csc_matrix(sum(sp.kron(prob.mats[d][k][idx][:, idx], sp.csr_matrix(Ck)) for k, Ck in C.items()))


def cond_estimate(prob, d, C):
    """1-norm condition estimate of the dim-d system (Hager-Higham on a sparse LU)."""
    A = dim_system_sparse(prob, d, C)
    lu = spla.splu(A)
    inv = spla.LinearOperator(A.shape, matvec=lu.solve, rmatvec=lambda x: lu.solve(x, trans="T"),
                              dtype=np.float64)
    return float(spla.onenormest(A) * spla.onenormest(inv))
