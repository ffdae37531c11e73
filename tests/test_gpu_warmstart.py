"""What the learned warm start gains: a network trained on the GPU (own
forward/backward/Adam kernels) on factors that Algorithm 1 produced for
two-slab chains (parameter draws plus a carried initial condition), then used
to initialise held-out slabs; residuals after each sweep compared with the
plain random initialisation, with the fallback rule applied."""
import numpy as np
import pytest

import taps_workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[warm]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, chain, warmstart
    h = capi.Handle()
    yield torch, capi, chain, warmstart, h
    h.close()


def draws(n, seed, **grid):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        P, r, k = rng.uniform(100, 300), rng.uniform(0.03, 0.08), rng.uniform(0.01, 0.03)
        out.append(W.heat_slab(seed=seed * 7919 + i, power=float(P), radius=float(r), k=float(k), **grid))
    return out


def test_trained_network_beats_plain_initialisation(env):
    torch, capi, chain, ws, h = env
    grid = dict(nx=48, ny=48, nz=16, nt=33, M=8)
    n_chain, M, Kc, sweeps = 160, 8, 4, 6
    cases_a = draws(n_chain, 5, **grid)
    cases_b = [W.replace(c, x_start=0.9) for c in draws(n_chain, 6, **grid)]
    layout = ws.Layout(h, cases_a[0], M)
    _say(f"data: {n_chain} two-slab chains 48x48x16x33 M={M} Kc={Kc}, {sweeps} sweeps each")
    data = ws.make_chains(h, cases_a, cases_b, M, Kc, sweeps, 4, 100, layout)
    X, T, hist = data["X"], data["T"], data["hist"]
    n = X.shape[0]
    perm = np.random.Generator(np.random.PCG64(4)).permutation(n)
    tr, te = perm[: n - 48], perm[n - 48:]
    med1 = float(np.nanmedian(hist[0, tr]))
    _say(f"plain init: median rho after sweep 1 = {med1:.3e}, after {sweeps} = {np.nanmedian(hist[-1, tr]):.3e}")
    widths = [X.shape[1], 256, 256, 256, T.shape[1]]
    net = ws.Net(h, widths, *W.mlp_init(widths, 0))
    tri = torch.tensor(tr, device="cuda")
    losses = ws.train(h, net, X[tri].contiguous(), T[tri].contiguous(), steps=1500, lr=1e-3, batch=64, seed=1)
    _say(f"training loss {losses[:10].mean():.3e} -> {losses[-100:].mean():.3e}")
    assert losses[-100:].mean() < losses[:10].mean() / 5
    # held-out slabs, warm-started
    Y = net.forward(X[torch.tensor(te, device="cuda")].contiguous())
    probs, U0 = [], []
    for j, i in enumerate(te):
        c = data["cases"][i]
        V = None if i < n_chain else data["V"][i - n_chain]
        p = chain.slab_problem(h, c, V)
        probs.append(p)
        U0.append(layout.initial(Y[j], [ax.fixed for ax in c.axes]))
    # the batched prolongation gives every slab exactly its single-slab start
    fixed0 = [ax.fixed for ax in data["cases"][te[0]].axes]
    Ub = layout.initial_batch(Y, fixed0)
    for j in range(len(te)):
        for u, v in zip(Ub[j], layout.initial(Y[j], fixed0)):
            assert u.is_contiguous() and torch.equal(u, v)
    warm = ws.sweep_history(h, probs, U0, sweeps)
    plain = hist[:, te]
    for s in range(sweeps):
        _say(f"  sweep {s + 1}: median rho warm {np.nanmedian(warm[s]):.3e}  plain {np.nanmedian(plain[s]):.3e}")
    # fallback rule: keep the warm start unless it loses to the plain median at sweep 1 or grows
    keep = np.array([not ws.restart_plain(warm[0, j], warm[1, j], med1) for j in range(len(te))])
    # what the network gains: sweeps to reach the plain start's median residual
    # after 3 sweeps (the target the benchmark uses), a slab that falls back
    # paying its two warm sweeps plus the plain start's count; never reached
    # within the sweeps run counts as sweeps + 1
    target = float(np.nanmedian(hist[2, tr]))

    def to_target(h_col):
        hit = np.nonzero(h_col <= target)[0]
        return int(hit[0]) + 1 if hit.size else sweeps + 1

    n_plain = np.array([to_target(plain[:, j]) for j in range(len(te))])
    n_warm = np.array([to_target(warm[:, j]) if keep[j] else 2 + n_plain[j] for j in range(len(te))])
    _say(f"warm start kept for {keep.sum()}/{len(te)} slabs; sweeps to the plain 3-sweep median {target:.3e}: "
         f"warm {n_warm.mean():.2f} (with fallbacks) vs plain {n_plain.mean():.2f}")
    assert np.nanmedian(warm[0]) < np.nanmedian(plain[0])
    assert np.nanmedian(warm[1]) < np.nanmedian(plain[1])
    assert n_warm.mean() < n_plain.mean()
