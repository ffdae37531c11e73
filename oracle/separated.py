"""Separated operator, Grams, Hadamard couplings, force and the dim-d system (oracle).

Paper Sec. 2.5 (discretized matrix form).  The operator is a sum of T
separable terms  sum_tau gamma_tau (x)_d A^tau_d  (one 1D matrix per dimension
and term) and the load a sum of R separable terms  sum_r (x)_d F^r_d.
With the trial field u = sum_m prod_d U_d[:,m] (CP form, Sec. 2.2) and the test
function varied in dimension d only (Sec. 2.4, variational test function), the
1D integrals of the other dimensions collapse into M x M coefficient matrices
(the paper's C^[k], C^[t]) that multiply entrywise -- the Hadamard product
C^[x]_mn = C^[k]_mn C^[t]_mn with no sum over (m, n).  Written out:

  Gram            G^A_e[m, n] = U_e[:, m]^T A_e U_e[:, n]     (test mode m first)
  load Gram       L_e[r, m]   = F^r_e . U_e[:, m]
  coupling        C^tau_d     = gamma_tau * prod_{e != d} G^{A^tau_e}_e   (entrywise)
  force           Q_d[i, m]   = sum_r F^r_d[i] prod_{e != d} L_e[r, m]
  dim-d system    sum_tau A^tau_d U_d (C^tau_d)^T = Q_d

The last line is the paper's K^[d] U^[d] = Q^[d] (Sec. 2.6, per-dimension
linear system) with the 4th-order tensor A_{i j m n} = A_d[i, j] C_d[m, n]
reshaped node-major (I = i*M + m).  Rows of fixed nodes (Dirichlet faces, the
initial-condition row in time; Sec. 2.1 Kronecker-delta property) carry U = 0:
their test functions are dropped and their unknowns are known zeros.
Couplings are reported grouped by the dim-d matrix (sum over the terms that
share it), which is the same linear system.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class SeparatedProblem:
    """A separated S-P-T problem on D dimensions.

    mats[d]   : dict name -> sparse n_d x n_d 1D matrix
    terms     : list of (gamma, names) with names[d] a key of mats[d]
    F[d]      : n_d x R_d dense load columns
    load_col[d]: length-R int array, load term r uses column load_col[d][r] of F[d]
    fixed[d]  : tuple of fixed node indices
    """

    def __init__(self, mats, terms, F, load_col, fixed):
        self.mats = mats
        self.terms = [(float(g), tuple(names)) for g, names in terms]
        self.F = [np.asarray(f, dtype=np.float64) for f in F]
        self.load_col = [np.asarray(c, dtype=np.int64) for c in load_col]
        self.fixed = [tuple(f) for f in fixed]
        self.D = len(mats)
        self.n = [next(iter(m.values())).shape[0] for m in mats]
        R = {len(c) for c in self.load_col}
        assert len(R) == 1, "every dim needs one column index per load term"
        self.R = R.pop()

    def kinds(self, d):
        """Distinct dim-d matrix names in first-use order."""
        out = []
        for _, names in self.terms:
            if names[d] not in out:
                out.append(names[d])
        return out

    def free(self, d):
        mask = np.ones(self.n[d], dtype=bool)
        mask[list(self.fixed[d])] = False
        return mask


def gram(A, U):
    """U^T A U (M x M), test mode first."""
    return U.T @ (A @ U)


def load_gram(F, U):
    """F^T U (R_cols x M)."""
    return F.T @ U


def couplings(prob, U, d):
    """dict name -> C^{(k)}_d = sum over terms using matrix k in dim d of
    gamma * Hadamard product of the other dims' Grams."""
    M = U[0].shape[1]
    out = {k: np.zeros((M, M)) for k in prob.kinds(d)}
    for gamma, names in prob.terms:
        C = np.full((M, M), gamma)
        for e in range(prob.D):
            if e != d:
                C = C * gram(prob.mats[e][names[e]], U[e])
        out[names[d]] += C
    return out


def force(prob, U, d):
    """Q_d = sum_r F^r_d (prod_{e != d} F^r_e . U_e[:, m])  (n_d x M)."""
    M = U[0].shape[1]
    W = np.ones((prob.R, M))
    for e in range(prob.D):
        if e != d:
            L = load_gram(prob.F[e], U[e])
            W = W * L[prob.load_col[e], :]
    return prob.F[d][:, prob.load_col[d]] @ W


def apply_dim(prob, d, C, X):
    """sum_k A^k_d X (C^k)^T  (the dim-d operator applied to a factor)."""
    out = np.zeros_like(X)
    for k, Ck in C.items():
        out += prob.mats[d][k] @ X @ Ck.T
    return out


def dim_matrix_dense(prob, d, C):
    """The (n_d M) x (n_d M) node-major system matrix, fixed rows/cols removed."""
    free = prob.free(d)
    Kd = sum(np.kron(prob.mats[d][k].toarray()[np.ix_(free, free)], Ck) for k, Ck in C.items())
    return Kd


def _half_bandwidth(prob, d):
    w = 0
    for A in prob.mats[d].values():
        coo = A.tocoo()
        if coo.nnz:
            w = max(w, int(np.max(np.abs(coo.row - coo.col))))
    return w


def solve_dim(prob, d, C, Q, dense_limit=2000):
    """Exact solution U_d of the dim-d system (fixed rows = 0).

    Dense LU (numpy) when n_d*M <= dense_limit, else LAPACK banded LU with
    partial pivoting on the node-major matrix (half-bandwidth (w+1)M-1)."""
    n, M = prob.n[d], Q.shape[1]
    free = prob.free(d)
    U = np.zeros((n, M))
    nf = int(free.sum())
    if nf * M <= dense_limit:
        K = dim_matrix_dense(prob, d, C)
        U[free] = np.linalg.solve(K, Q[free].reshape(-1)).reshape(nf, M)
        return U
    w = _half_bandwidth(prob, d)
    bw = (w + 1) * M - 1
    N = n * M
    ab = np.zeros((2 * bw + 1, N))
    fixed_rows = ~free
    for k, Ck in C.items():
        coo = prob.mats[d][k].tocoo()
        for i, j, a in zip(coo.row, coo.col, coo.data):
            if fixed_rows[i] or fixed_rows[j]:
                continue
            for m in range(M):
                I = i * M + m
                J = j * M + np.arange(M)
                ab[bw + I - J, J] += a * Ck[m, :]
    rhs = Q.reshape(-1).copy()
    for i in np.nonzero(fixed_rows)[0]:
        for m in range(M):
            I = i * M + m
            ab[bw, I] = 1.0
            rhs[I] = 0.0
    x = sla.solve_banded((bw, bw), ab, rhs)
    return x.reshape(n, M)


def residuals(prob, U):
    """Per-dim projected Galerkin residuals R_d = sum_k A^k_d U_d C^k^T - Q_d on
    free rows, and the matching Q_d.  Zero at a fixed point of Algorithm 1."""
    Rs, Qs = [], []
    for d in range(prob.D):
        C = couplings(prob, U, d)
        Q = force(prob, U, d)
        R = apply_dim(prob, d, C, U[d]) - Q
        free = prob.free(d)
        Rs.append(R[free])
        Qs.append(Q[free])
    return Rs, Qs


def residual_norm(prob, U):
    """rho = sqrt(sum_d ||R_d||_F^2) / sqrt(sum_d ||Q_d||_F^2)."""
    Rs, Qs = residuals(prob, U)
    num = sum(float(np.sum(R * R)) for R in Rs)
    den = sum(float(np.sum(Q * Q)) for Q in Qs)
    return np.sqrt(num) / np.sqrt(den) if den > 0 else np.sqrt(num)


def energy(prob, U):
    """J(u) = 1/2 a(u, u) - l(u) of the separated field (symmetric operators)."""
    M = U[0].shape[1]
    a = 0.0
    for gamma, names in prob.terms:
        P = np.full((M, M), gamma)
        for e in range(prob.D):
            P = P * gram(prob.mats[e][names[e]], U[e])
        a += P.sum()
    W = np.ones((prob.R, M))
    for e in range(prob.D):
        W = W * load_gram(prob.F[e], U[e])[prob.load_col[e], :]
    return 0.5 * a - W.sum()
