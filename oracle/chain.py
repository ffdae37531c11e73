"""Space-time slab chain with a carried initial condition and mode compression
(oracle; test infrastructure only).

Paper, LPBF section and the mode-compression appendix.  A long scan is split
into space-time slabs.  Slab T+1 solves for u = u_c(x_s) + u_0(x_s, t), where
u_c is slab T's field at its last time node and u_0 has a homogeneous initial
condition (fixed t = 0 row).  Because u_c does not depend on t, substituting it
into rho c_p du/dt - k lap u = f leaves, in weak form,

    a(u_0, v) = l(v) - k int grad u_c . grad v,

and for u_c = sum_r prod_{d in x,y,z} V_d[:, r] the extra term is separable:
for each r, three load terms (one per spatial dim carrying the stiffness
matrix), e.g.  -k (K_x V_x[:,r]) (x) (M_y V_y[:,r]) (x) (M_z V_z[:,r]) (x) w_t
with w_t[l] = int Ntilde_l(t) dt (the time test function against the constant
1).  The discrete statement behind it: G 1 = 0 (partition of unity) and
M_t 1 = w_t, so A (u_c (x) 1_t) is exactly the sum of those terms.

The end state u(x_s, t_max) = u_c + sum_m U_x U_y U_z U_t[n_t - 1, m] has
K_c + M modes; mode compression replaces it by K_c modes through the weighted
residual statement  int du_F (u_F - u_TD) dx = 0, i.e. Algorithm 1 on the
mass-only operator M (x) M (x) M with the load M_d W_d built from the factors
W of u_TD (the z = 0 Dirichlet row stays fixed, so the carried field keeps the
boundary condition).
"""
import numpy as np

from . import als, problems
from .separated import SeparatedProblem


def time_weights(dt):
    """w_t[l] = int Ntilde_l(t) dt."""
    return dt.load(lambda t: np.ones_like(t))


def carried_terms(case, dims, V):
    """Load columns of -k int grad u_c . grad v for u_c = sum_r prod V_d[:, r]
    (V = [V_x, V_y, V_z]).  Returns (F_x, F_y, F_z, F_t) with 3 K_c columns in
    space (term j carries the stiffness matrix in space dim j, the factor -k
    sits in x) and one time column w_t."""
    dx, dy, dz, dt = dims
    Kc = V[0].shape[1]
    mats = [(d.matrix("mass"), d.matrix("stiff")) for d in (dx, dy, dz)]
    cols = [[], [], []]
    for j in range(3):
        for r in range(Kc):
            for e in range(3):
                Mm, Kk = mats[e]
                col = (Kk if e == j else Mm) @ V[e][:, r]
                cols[e].append(-case.k * col if e == 0 else col)
    F = [np.stack(c, axis=1) if Kc else np.zeros((dims[e].n, 0)) for e, c in enumerate(cols)]
    return F + [time_weights(dt)[:, None]]


def slab_problem(case, dims, V):
    """The heat slab of ``case`` (moving source) plus the carried field's load terms."""
    base = problems.heat_slab(case, dims)
    if V is None or V[0].shape[1] == 0:
        return base
    Fc = carried_terms(case, dims, V)
    nc = Fc[0].shape[1]
    F, cols = [], []
    for d in range(4):
        off = base.F[d].shape[1]
        F.append(np.concatenate([base.F[d], Fc[d]], axis=1))
        extra = off + (np.arange(nc) if d < 3 else np.zeros(nc, np.int64))
        cols.append(np.concatenate([base.load_col[d], extra]))
    return SeparatedProblem(base.mats, base.terms, F, cols, base.fixed)


def end_state(V, U):
    """Factors of u(x_s, t_max) = u_c + sum_m prod U_d[:, m] U_t[-1, m]:
    [V_x | U_x diag(U_t[-1])], [V_y | U_y], [V_z | U_z]."""
    scale = U[3][-1, :]
    W = [U[0] * scale[None, :], U[1], U[2]]
    if V is not None and V[0].shape[1]:
        W = [np.concatenate([V[d], W[d]], axis=1) for d in range(3)]
    return W


def compression_problem(dims, W):
    """Algorithm 1 problem of the mode compression: operator M (x) M (x) M,
    load sum_r prod_d M_d W_d[:, r], fixed rows as in the slab (z = 0)."""
    mats = [{"mass": d.matrix("mass")} for d in dims[:3]]
    F = [mats[e]["mass"] @ W[e] for e in range(3)]
    R = W[0].shape[1]
    cols = [np.arange(R)] * 3
    return SeparatedProblem(mats, [(1.0, ("mass", "mass", "mass"))], F, cols, [d.fixed for d in dims[:3]])


def compress(dims, W, U0, tol=1e-10, iter_max=200):
    """K_c-mode approximation of the field with factors W (Algorithm 1 from U0)."""
    prob = compression_problem(dims, W)
    U, hist, ok = als.solve(prob, U0, tol=tol, iter_max=iter_max)
    return U, hist


def run_chain(cases, dims, U0s, C0s, sweeps, comp_sweeps, V0=None):
    """Solve slabs in order, carrying a K_c-mode initial condition (K_c = the
    mode count of C0s[T]); V0 is the field carried into the first slab.

    cases[T]   slab T's parameters (one grid); U0s[T] its initial factors;
    C0s[T]     initial factors of slab T's compression; fixed sweep counts.
    Returns per slab (U, V_carried_into_slab, V_carried_out)."""
    out = []
    V = V0
    for T, case in enumerate(cases):
        prob = slab_problem(case, dims, V)
        U = [np.array(u, dtype=np.float64, copy=True) for u in U0s[T]]
        for _ in range(sweeps):
            als.sweep(prob, U)
            als.balance(U)
        W = end_state(V, U)
        Vn = [np.array(u, dtype=np.float64, copy=True) for u in C0s[T]]
        cprob = compression_problem(dims, W)
        for _ in range(comp_sweeps):
            als.sweep(cprob, Vn)
            als.balance(Vn)
        out.append((U, V, Vn))
        V = Vn
    return out
