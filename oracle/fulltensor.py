"""Full-tensor Galerkin solve on tiny grids (oracle pin).

Paper Sec. 2.7, error estimates: the TAPS solution approaches the Galerkin
solution of the full (undecomposed) C-HiDeNN space as modes are added.  That
solution is computed here directly: the operator sum_tau gamma_tau
A^tau_1 (x) ... (x) A^tau_D assembled as one sparse Kronecker matrix over all
nodes (first dimension slowest), fixed nodes removed, solved by a dense LU (sparse LU beyond 8000 unknowns).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _kron_all(mats):
    out = sp.csr_matrix(np.ones((1, 1)))
    for A in mats:
        out = sp.kron(out, sp.csr_matrix(A), format="csr")
    return out


def free_mask(prob):
    mask = np.ones(1, dtype=bool)
    for d in range(prob.D):
        mask = np.kron(mask, prob.free(d)).astype(bool)
    return mask


def full_operator(prob):
    return sum(g * _kron_all([prob.mats[d][names[d]] for d in range(prob.D)])
               for g, names in prob.terms)


def full_load(prob):
    f = 0.0
    for r in range(prob.R):
        v = np.ones(1)
        for d in range(prob.D):
            v = np.kron(v, prob.F[d][:, prob.load_col[d][r]])
        f = f + v
    return f


def solve_full(prob):
    """Nodal tensor of the full Galerkin solution (zeros at fixed nodes)."""
    A = full_operator(prob).tocsr()
    f = full_load(prob)
    mask = free_mask(prob)
    u = np.zeros(len(f))
    Af = A[mask][:, mask]
    if Af.shape[0] <= 8000:
        u[mask] = np.linalg.solve(Af.toarray(), f[mask])
    else:
        u[mask] = spla.spsolve(Af.tocsc(), f[mask])
    return u.reshape(prob.n)


def td_tensor(U):
    """Nodal tensor sum_m prod_d U_d[:, m]."""
    M = U[0].shape[1]
    out = 0.0
    for m in range(M):
        t = np.ones(1)
        for Ud in U:
            t = np.kron(t, Ud[:, m])
        out = out + t
    return np.asarray(out).reshape([Ud.shape[0] for Ud in U])


def projected_residual(prob, U, d):
    """Galerkin projection of the explicit full residual A u - f onto the dim-d
    test space {delta U_d (x) others}: R_d[i, m] = sum_{other idx} r[..] prod_{e!=d} U_e[i_e, m]."""
    A = full_operator(prob)
    u = td_tensor(U).reshape(-1)
    r = (A @ u - full_load(prob)).reshape(prob.n)
    M = U[0].shape[1]
    out = np.zeros((prob.n[d], M))
    for m in range(M):
        t = r
        # contract the other dims, highest index first so axis numbers stay valid
        for e in reversed(range(prob.D)):
            if e != d:
                t = np.tensordot(t, U[e][:, m], axes=([e], [0]))
        out[:, m] = t
    return out[prob.free(d)]
