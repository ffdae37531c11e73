"""Solution-dependent coefficients on the GPU: the library's weighted kinds
(WMASS, WSTIFF, WDDT), its TD inner product, and the global-local loop of
Algorithm 2 built on them, against the oracle; the manufactured field; and
the paper's nonlinear moving-source set-up (10 mm x 10 mm x 1 mm, Inconel
718 linear fits, beam radius 0.5 mm at 500 mm/s, 10 elements per beam
diameter, time increment 1.6e-4 s): the coefficient change per global stage
and how far the nonlinear field moves from the linear one."""
import math
import time

import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import assemble, fulltensor, nonlinear as onl, problems

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[nonlinear]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, nonlinear
    h = capi.Handle()
    yield torch, capi, nonlinear, h
    h.close()


@pytest.mark.parametrize("s,p", [(2, 2), (1, 1)])
def test_weighted_kinds_match_oracle(env, s, p):
    torch, capi, nonlinear, h = env
    from paper_2503_13933_amd.problem import DeviceAxis
    ax = W.Axis("t", 0.0, 1.3, 23, s, 20.0, p, 5)
    A = DeviceAxis(h, ax, [capi.WMASS, capi.WSTIFF, capi.WDDT], "cuda")
    rng = np.random.Generator(np.random.PCG64(s))
    v = torch.tensor(rng.standard_normal((ax.n, 1)), device="cuda")
    val, der = nonlinear._gauss_values(h, A, v)
    coef = torch.cat([val[0], der[0]]).contiguous()
    capi.taps_assemble1d(h, A.basis, [capi.WMASS, capi.WSTIFF, capi.WDDT], A.band, coef_g=coef)
    torch.cuda.synchronize()
    D = assemble.Dim1D(ax.nodes(), s, 20.0, p, 5)
    vh = v.cpu().numpy()[:, 0]
    c, dc = D.Ng @ vh, D.Bg @ vh
    ref = [D.matrix("wmass", coef=c), D.matrix("wstiff", coef=c), D.matrix("wddt", coef=c, dcoef=dc)]
    band = A.band.cpu().numpy()
    w = 2 * s + 1
    for k in range(3):
        dense = np.zeros((ax.n, ax.n))
        for i in range(ax.n):
            for o in range(2 * w + 1):
                j = i + o - w
                if 0 <= j < ax.n:
                    dense[i, j] = band[k, i, o]
        pu.check(dense, ref[k].toarray(), pu.TOL, f"kind {k}")


def test_td_inner_matches_oracle(env):
    torch, capi, nonlinear, h = env
    c = W.nonlinear_heat(12, 9, 7, 11, M=3)
    dims = problems.dims_of(c)
    prob = nonlinear.coefficient_problem(h, c, None)
    rng = np.random.Generator(np.random.PCG64(3))
    A = [rng.standard_normal((D.n, 3)) for D in dims]
    B = [rng.standard_normal((D.n, 2)) for D in dims]
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    capi.taps_td_inner(h, [a.s for a in c.axes], [ax.band[0] for ax in prob.axes], prob.factors(A), prob.factors(B),
                       out)
    torch.cuda.synchronize()
    G = np.ones((3, 2))
    for D, a, b in zip(dims, A, B):
        G = G * (a.T @ (D.matrix("mass") @ b))
    pu.check(out.cpu().numpy()[:6].reshape(3, 2), G, pu.TOL, "Gram product")
    assert abs(out[6].item() - onl.td_inner(dims, A, B)) <= pu.TOL * abs(G).sum()


def test_global_local_matches_oracle(env):
    torch, capi, nonlinear, h = env
    c = W.nonlinear_heat(14, 10, 6, 11, M=4, Lx=2.0, Ly=2.0, H=0.5, T=0.004, radius=0.3, speed=200.0, y0=1.0,
                         x_start=0.5)
    dims = problems.dims_of(c)
    U0 = W.initial_factors(c.axes, 4, 5)
    rng = np.random.Generator(np.random.PCG64(6))
    V0 = []
    for D in dims:
        v = rng.standard_normal((D.n, 2))
        v[list(D.fixed)] = 0.0
        V0.append(v)
    _say("global-local loop 14x10x6x11, M=4, R_c=2, 3 global stages: GPU vs oracle")
    Ug, Vg, chg = nonlinear.global_local(h, c, U0, Rc=2, outer=3, sweeps=2, comp_sweeps=3, V_init=V0)
    torch.cuda.synchronize()
    # the oracle with the same compression start (its seeded draw replaced by V0)
    U = [u.copy() for u in U0]
    V, cho = None, []
    for it in range(3):
        prob = onl.coefficient_problem(c, dims, V)
        for _ in range(2):
            from oracle import als
            als.sweep(prob, U)
            als.balance(U)
        Vn = onl.compress(c, dims, U, 2, V if V is not None else V0, 3)
        if V is not None:
            nn = onl.td_inner(dims, Vn, Vn)
            cho.append(math.sqrt(max(nn + onl.td_inner(dims, V, V) - 2 * onl.td_inner(dims, Vn, V), 0.0) / nn))
        V = Vn
    # bars: the oracle's own response to 1e-14 perturbations of every dim solve
    with pu.perturbed(1e-14, seed=2):
        Up = [u.copy() for u in U0]
        Vp = None
        for it in range(3):
            prob = onl.coefficient_problem(c, dims, Vp)
            for _ in range(2):
                als.sweep(prob, Up)
                als.balance(Up)
            Vp = onl.compress(c, dims, Up, 2, Vp if Vp is not None else V0, 3)
    fu, fv = fulltensor.td_tensor(U), fulltensor.td_tensor(V)
    bar_u = max(pu.TOL, 10 * pu.maxrel(fulltensor.td_tensor(Up), fu))
    bar_v = max(pu.TOL, 10 * pu.maxrel(fulltensor.td_tensor(Vp), fv))
    ru = pu.check(fulltensor.td_tensor([u.cpu().numpy() for u in Ug]), fu, bar_u, "field")
    rv = pu.check(fulltensor.td_tensor([v.cpu().numpy() for v in Vg]), fv, bar_v, "compressed field")
    _say(f"  field {ru[0]:.1e}/{ru[1]:.1e} (bar {bar_u:.0e}), compressed {rv[0]:.1e}/{rv[1]:.1e} (bar {bar_v:.0e}); "
         f"changes gpu {[f'{x:.6e}' for x in chg[1:]]} oracle {[f'{x:.6e}' for x in cho]}")
    for a, b in zip(chg[1:], cho):
        assert abs(a - b) <= max(1e-7, 100 * bar_v) * max(b, 1e-300)


def test_manufactured_field_on_gpu(env):
    torch, capi, nonlinear, h = env
    c = W.nonlinear_heat(9, 6, 6, 7, M=1, Lx=1.0, Ly=1.0, H=0.5, T=1.0, source="poly", amp=20.0, m_k=1e-3,
                         n_k=1e-2, m_c=1e-3, n_c=2e-2)
    dims = problems.dims_of(c)
    rng = np.random.Generator(np.random.PCG64(7))
    V0 = [rng.standard_normal((D.n, 1)) for D in dims]
    for v, D in zip(V0, dims):
        v[list(D.fixed)] = 0.0
    U, V, ch = nonlinear.global_local(h, c, W.initial_factors(c.axes, 1, 3), Rc=1, outer=25, sweeps=3,
                                      comp_sweeps=3, V_init=V0)
    u = fulltensor.td_tensor([x.cpu().numpy() for x in U])
    x, t = dims[0].nodes, dims[3].nodes
    ref = np.einsum("i,j,k,l->ijkl", 20 * x * (1 - x), np.ones(6), np.ones(6), t)
    _say(f"manufactured field: max error {np.abs(u - ref).max() / 5.0:.2e}, changes {[f'{v:.1e}' for v in ch]}")
    assert np.abs(u - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.timeout(900)
def test_paper_setup_global_local(env):
    torch, capi, nonlinear, h = env
    c = W.nonlinear_heat(M=10)
    n = [a.n for a in c.axes]
    rng = np.random.Generator(np.random.PCG64(8))
    V0 = []
    for a in c.axes:
        v = rng.standard_normal((a.n, 3))
        if a.fixed:
            v[list(a.fixed)] = 0.0
        V0.append(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, V, ch = nonlinear.global_local(h, c, W.initial_factors(c.axes, 10, 9), Rc=3, outer=8, sweeps=3,
                                      comp_sweeps=4, tol=1e-4, V_init=V0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    _say(f"paper set-up {n} (x, y, z, t), M=10, R_c=3: {len(ch)} global stages in {el:.2f} s; "
         f"coefficient change per stage {[f'{x:.2e}' for x in ch]}")
    # the nonlinear field against the linear one (constant n_k, n_c): the
    # temperature rise lowers k and raises rho c_p, so the peak moves
    lin = nonlinear.coefficient_problem(h, c, None)
    Ul = lin.factors(W.initial_factors(c.axes, 10, 9))
    capi.taps_als(h, lin.struct, Ul, 0.0, 3 * len(ch))
    mid = [a.n // 2 for a in c.axes[:3]]
    peak = lambda F: float(np.max(np.einsum("m,m,m,tm->t", *[f.cpu().numpy()[i] for f, i in zip(F[:3], mid)],
                                            F[3].cpu().numpy())))
    _say(f"  peak temperature rise on the centre line: nonlinear {peak(U):.1f}, linear {peak(Ul):.1f}")
    assert ch[-1] < ch[1]
