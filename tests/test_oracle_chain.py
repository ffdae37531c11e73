"""Pins of the slab-chain oracle (carried initial condition, mode compression).

Each pin compares the separated construction with something computed another
way: the explicit Kronecker operator, a full-tensor solve with the initial
condition imposed directly, and exact representability of low-rank fields.
"""
import numpy as np

import taps_workloads as W
from oracle import als, chain, fulltensor, problems


def tiny_case(power=200.0, seed=0):
    # s = 1, p = 1 keeps the full tensor small (n >= 2s + 2 = 4 per axis)
    return W.heat_slab(6, 5, 5, 4, M=3, seed=seed, s=1, p=1, power=power)


def rand_field(dims, K, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    V = [rng.standard_normal((d.n, K)) for d in dims[:3]]
    V[2][0, :] = 0.0                      # carried field vanishes on z = 0
    return V


def test_carried_load_is_operator_on_constant_in_time_field():
    """-A (u_c (x) 1_t) written with the full Kronecker operator equals the
    separated carried load (uses G 1 = 0 and M_t 1 = w_t)."""
    case = tiny_case()
    dims = problems.dims_of(case)
    V = rand_field(dims, 2, 1)
    heat = problems.heat_slab(case, dims)
    A = fulltensor.full_operator(heat)
    uc = fulltensor.td_tensor(V)                              # (nx, ny, nz)
    u = np.einsum("ijk,l->ijkl", uc, np.ones(dims[3].n)).reshape(-1)
    Fc = chain.carried_terms(case, dims, V)
    nc = Fc[0].shape[1]
    from oracle.separated import SeparatedProblem
    carried = SeparatedProblem(heat.mats, heat.terms, Fc,
                               [np.arange(nc)] * 3 + [np.zeros(nc, np.int64)], heat.fixed)
    lhs = fulltensor.full_load(carried)
    rhs = -(A @ u)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_split_solution_equals_directly_imposed_initial_condition():
    """Full Galerkin solve of the homogenised slab plus u_c equals the full
    Galerkin solve with the t = 0 nodal values set to u_c."""
    case = tiny_case(power=150.0)
    dims = problems.dims_of(case)
    V = rand_field(dims, 2, 2)
    u0 = fulltensor.solve_full(chain.slab_problem(case, dims, V))
    uc = fulltensor.td_tensor(V)
    split = u0 + uc[..., None]
    heat = problems.heat_slab(case, dims)
    A = fulltensor.full_operator(heat).toarray()
    f = fulltensor.full_load(heat)
    shape = heat.n
    known = np.zeros(shape)
    known[..., 0] = uc                     # initial condition (z = 0 rows are zero in uc)
    free = fulltensor.free_mask(heat)
    x = known.reshape(-1).copy()
    x[free] = np.linalg.solve(A[free][:, free], f[free] - A[free][:, ~free] @ x[~free])
    direct = x.reshape(shape)
    assert np.abs(split - direct).max() <= 1e-10 * np.abs(direct).max()


def test_compression_reproduces_field_of_lower_rank():
    """A field with rank <= K_c is its own mass-weighted projection."""
    case = tiny_case()
    dims = problems.dims_of(case)
    Wf = rand_field(dims, 2, 3)
    U0 = W.initial_factors(case.axes[:3], 3, 5)
    V, hist = chain.compress(dims, Wf, U0, tol=1e-12, iter_max=500)
    got, ref = fulltensor.td_tensor(V), fulltensor.td_tensor(Wf)
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_rank_one_compression_exact_after_one_sweep():
    """Rank-one target, rank-one compression: one sweep of Algorithm 1 lands
    on it (each dim solve is a scalar multiple of the target factor)."""
    case = tiny_case()
    dims = problems.dims_of(case)
    Wf = rand_field(dims, 1, 4)
    V = W.initial_factors(case.axes[:3], 1, 6)
    als.sweep(chain.compression_problem(dims, Wf), V)
    got, ref = fulltensor.td_tensor(V), fulltensor.td_tensor(Wf)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_end_state_is_field_at_last_time_node():
    case = tiny_case()
    dims = problems.dims_of(case)
    rng = np.random.Generator(np.random.PCG64(7))
    U = [rng.standard_normal((d.n, 3)) for d in dims]
    V = rand_field(dims, 2, 8)
    Wf = chain.end_state(V, U)
    ref = fulltensor.td_tensor(U)[..., -1] + fulltensor.td_tensor(V)
    assert np.abs(fulltensor.td_tensor(Wf) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_chain_runs_and_carries_modes():
    cases = [tiny_case(seed=s) for s in range(3)]
    cases = [W.replace(c, x_start=0.1 + 0.3 * T) for T, c in enumerate(cases)] if hasattr(W, "replace") else cases
    dims = problems.dims_of(cases[0])
    U0s = [W.initial_factors(c.axes, 3, 10 + T) for T, c in enumerate(cases)]
    C0s = [W.initial_factors(c.axes[:3], 2, 20 + T) for T, c in enumerate(cases)]
    out = chain.run_chain(cases, dims, U0s, C0s, sweeps=3, comp_sweeps=3)
    assert out[0][1] is None
    for T in range(1, 3):
        assert out[T][1] is out[T - 1][2]
        assert out[T][2][0].shape[1] == 2 and np.all(out[T][2][2][0] == 0.0)


def test_compression_is_mass_weighted_best_rank_one():
    """K_c = 1 on a rank-2 field with one dominant mode: the converged
    compression equals the best rank-one approximation in the L2 (mass) norm,
    computed independently by a higher-order power iteration on the dense
    tensor after the change of variables M_d = L_d L_d^T (z restricted to the
    free rows, where the carried field lives)."""
    case = tiny_case()
    dims = problems.dims_of(case)
    Wf = rand_field(dims, 2, 12)
    Wf[0][:, 1] *= 0.3
    target = fulltensor.td_tensor(Wf)[:, :, 1:]
    Ls = [np.linalg.cholesky(d.matrix("mass").toarray()) for d in dims[:2]]
    Ls.append(np.linalg.cholesky(dims[2].matrix("mass").toarray()[1:, 1:]))
    t = np.einsum("ijk,ia,jb,kc->abc", target, *Ls)        # coordinates with the M-inner product
    # the problem has more than one stationary point: take the best of a few
    # seeded starts on both sides
    cands = []
    for start in range(4):
        rng = np.random.Generator(np.random.PCG64(start))
        vecs = [rng.standard_normal(n) for n in t.shape]
        for _ in range(1000):
            vecs[0] = np.einsum("abc,b,c->a", t, vecs[1], vecs[2]); vecs[0] /= np.linalg.norm(vecs[0])
            vecs[1] = np.einsum("abc,a,c->b", t, vecs[0], vecs[2]); vecs[1] /= np.linalg.norm(vecs[1])
            vecs[2] = np.einsum("abc,a,b->c", t, vecs[0], vecs[1])
        bt = np.einsum("a,b,c->abc", *vecs)
        cands.append((np.linalg.norm(t - bt), bt))
    best_t = min(cands, key=lambda c: c[0])[1]
    best = np.einsum("abc,ia,jb,kc->ijk", best_t, *[np.linalg.inv(L).T for L in Ls])
    Ms = [d.matrix("mass").toarray() for d in dims[:3]]
    full = fulltensor.td_tensor(Wf)
    runs = []
    for seed in (13, 14, 15):
        V, hist = chain.compress(dims, Wf, W.initial_factors(case.axes[:3], 1, seed), tol=1e-13, iter_max=2000)
        g = fulltensor.td_tensor(V)
        e = full - g
        runs.append((np.einsum("ijk,ia,jb,kc,abc->", e, *Ms, e), g))
    got = min(runs, key=lambda r: r[0])[1]
    assert np.abs(got[:, :, 0]).max() == 0.0
    assert np.abs(got[:, :, 1:] - best).max() <= 1e-7 * np.abs(best).max()
