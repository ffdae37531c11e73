"""Solution-dependent material coefficients and the global-local loop,
Algorithm 2 of the paper (oracle; test infrastructure only).

Appendix on solution-dependent coefficients: the weak form is
    int v d/dt (rho c_p(u) u) + int grad v . k(u) grad u = int v f,
and with the linear fits of the third results section the coefficients
k = m_k u + n_k, rho c_p = m_c u + n_c are themselves in TD form whenever u
is.  Global stage: with the coefficients frozen the problem is linear and is
solved by Algorithm 1.  Local stage: the coefficients are updated from the
new u (for linear fits exactly, at every Gauss point, through the TD form).
The loop stops when the coefficients change by at most a positive tolerance
(tol = 0: every one of the given outer stages runs).

Readings:
  * the coefficient field is the TD of u compressed to R_c modes by the
    paper's mode compression (Algorithm 1 on the mass-only operator with u as
    load, fixed rows kept), so the operator has 4 (R_c + 1) separable terms:
      n_c (M, M, M, G),  m_c (W[v_x], W[v_y], W[v_z], W_G[v_t]) per mode v,
      n_k (K, M, M, M) and its y, z analogues,
      m_k (W_K[v_x], W[v_y], W[v_z], W[v_t]) and its y, z analogues,
    with W[c] = int c N N, W_K[c] = int c B B, W_G[c] = int N d/dt (c N);
  * the first global stage uses the constant coefficients (u = 0), the
    solution's factors start from the seeded random draw;
  * a global stage runs a fixed number of sweeps from the current factors;
  * the change measured is that of the compressed field in the mass norm,
    ||u_c(new) - u_c(old)||_M / ||u_c(new)||_M (the coefficients are affine
    in it).
"""
import numpy as np

from . import als, problems, separated
from .separated import SeparatedProblem


def td_inner(dims, A, B):
    """Mass-norm inner product of two TD fields: sum_{m,m'} prod_d A_d[:,m]^T M_d B_d[:,m']."""
    G = np.ones((A[0].shape[1], B[0].shape[1]))
    for D, a, b in zip(dims, A, B):
        G = G * (a.T @ (D.matrix("mass") @ b))
    return float(np.sum(G))


def compress(case, dims, U, Rc, V0, sweeps):
    """Rank-R_c field closest to u = prod_d U_d in the mass norm (mode
    compression: Algorithm 1 on M (x) M (x) M (x) M with load M_d U_d)."""
    mats = [{"mass": D.matrix("mass")} for D in dims]
    F = [np.asarray(D.matrix("mass") @ u) for D, u in zip(dims, U)]
    R = U[0].shape[1]
    prob = SeparatedProblem(mats, [(1.0, ("mass",) * 4)], F, [np.arange(R)] * 4, [D.fixed for D in dims])
    V = [np.array(v, copy=True) for v in V0]
    for _ in range(sweeps):
        als.sweep(prob, V)
        als.balance(V)
    return V


def coefficient_problem(case, dims, V):
    """The linear problem of one global stage: operator with the coefficients
    n + m u_c, u_c = prod_d V_d (R_c modes), and the case's load."""
    dx, dy, dz, dt = dims
    Rc = V[0].shape[1] if V is not None else 0
    mats = [{"mass": D.matrix("mass"), "stiff": D.matrix("stiff")} for D in (dx, dy, dz)]
    mats.append({"mass": dt.matrix("mass"), "ddt": dt.matrix("ddt")})
    terms = [(case.n_c, ("mass", "mass", "mass", "ddt")), (case.n_k, ("stiff", "mass", "mass", "mass")),
             (case.n_k, ("mass", "stiff", "mass", "mass")), (case.n_k, ("mass", "mass", "stiff", "mass"))]
    for r in range(Rc):
        for d, D in enumerate(dims):
            c = np.asarray(D.Ng @ V[d][:, r]).ravel()
            mats[d][f"w{r}"] = D.matrix("wmass", coef=c)
            if d < 3:
                mats[d][f"wk{r}"] = D.matrix("wstiff", coef=c)
            else:
                mats[d][f"wg{r}"] = D.matrix("wddt", coef=c, dcoef=np.asarray(D.Bg @ V[d][:, r]).ravel())
        w = f"w{r}"
        terms.append((case.m_c, (w, w, w, f"wg{r}")))
        terms.append((case.m_k, (f"wk{r}", w, w, w)))
        terms.append((case.m_k, (w, f"wk{r}", w, w)))
        terms.append((case.m_k, (w, w, f"wk{r}", w)))
    F, cols = loads(case, dims)
    return SeparatedProblem(mats, terms, F, cols, [D.fixed for D in dims])


def loads(case, dims):
    dx, dy, dz, dt = dims
    one = lambda v: np.ones_like(v)
    if case.source == "poly":
        # f = 2 m_c a^2 X^2 t + n_c a X - m_k a^2 t^2 (L^2 - 6 L x + 6 x^2) + 2 n_k a t,  X = x (L - x)
        L, a = dx.nodes[-1], case.amp
        X = lambda x: x * (L - x)
        fx = [lambda x: 2 * case.m_c * a * a * X(x) ** 2, lambda x: case.n_c * a * X(x),
              lambda x: -case.m_k * a * a * (L * L - 6 * L * x + 6 * x * x), lambda x: 2 * case.n_k * a * one(x)]
        ft = [lambda t: t, one, lambda t: t * t, lambda t: t]
        F = [dx.loads(fx), dy.loads([one] * 4), dz.loads([one] * 4), dt.loads(ft)]
        return F, [np.arange(4)] * 4
    amp = 2.0 * case.eta * case.power / (np.pi * case.radius ** 2 * dz.nodes[-1])
    r2 = case.radius ** 2
    x0 = case.x_start + case.speed * dt.nodes
    Fx = np.stack([dx.load(lambda x, c=c: amp * np.exp(-2.0 * (x - c) ** 2 / r2)) for c in x0], axis=1)
    Fy = dy.load(lambda y: np.exp(-2.0 * (y - case.y0) ** 2 / r2))[:, None]
    Fz = dz.load(one)[:, None]
    Ft = dt.matrix("mass").toarray()
    nt = dt.n
    zero = np.zeros(nt, np.int64)
    return [Fx, Fy, Fz, Ft], [np.arange(nt), zero, zero, np.arange(nt)]


def global_local(case, dims, U0, Rc, outer, sweeps, comp_sweeps=4, tol=0.0, seed=0):
    """Algorithm 2: returns the factors of u, the compressed coefficient
    field's factors and the change of the compressed field per global stage."""
    U = [np.array(u, copy=True) for u in U0]
    V = None
    rng = np.random.Generator(np.random.PCG64(seed))
    Vinit = []
    for D in dims:
        v = rng.standard_normal((D.n, Rc))
        v[list(D.fixed)] = 0.0
        Vinit.append(v)
    changes = []
    for it in range(outer):
        prob = coefficient_problem(case, dims, V)           # global stage: frozen coefficients
        for _ in range(sweeps):
            als.sweep(prob, U)
            als.balance(U)
        Vn = compress(case, dims, U, Rc, V if V is not None else Vinit, comp_sweeps)   # local stage
        if V is None:
            change = 1.0
        else:
            nn = td_inner(dims, Vn, Vn)
            change = np.sqrt(max(nn + td_inner(dims, V, V) - 2 * td_inner(dims, Vn, V), 0.0) / nn)
        changes.append(change)
        V = Vn
        if tol > 0.0 and change <= tol:
            break
    return U, V, changes
