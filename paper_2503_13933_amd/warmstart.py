"""Learned warm start of a slab's factors (driver above the C ABI).

A network maps slab features -- (P, r, k, y0) scaled to [-1, 1] and the carried
initial condition sampled on a 4 x 4 x 4 coarse grid -- to the canonical
factors of the converged slab solution in y, z and t, sampled at coarse nodes.
Its prediction, prolongated to the fine grid by C-HiDeNN interpolation of the
coarse nodal values, initialises Algorithm 1 (the x factor needs none: the
first dim solve uses only the other factors).  Training and inference run in
the library's kernels: taps_mlp_forward / taps_mlp_backward / taps_mlp_mse /
taps_adam_step for the network, taps_canonicalize, taps_shape1d and
taps_interp1d for the factor data, taps_reconstruct for the initial-condition
features, taps_als / taps_als_batched for the slab solves.

Fallback: the warm start is dropped for the plain initialisation when its
projected residual after sweep 1 exceeds the median sweep-1 residual of the
plain initialisation (measured on the training slabs), or when the residual
grows from sweep 1 to sweep 2.
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi

F32, F64 = torch.float32, torch.float64
PARAM_RANGES = {"power": (100.0, 300.0), "radius": (0.030, 0.080), "k": (0.010, 0.030), "y0": (0.3, 0.7)}


class FactorBatch:
    """Factors of N slabs on one grid: one contiguous (N, n_d, M) FP64 tensor
    per dim.  Slab b's factor of dim d starts at a computed address, so a
    round of the batched driver needs no per-slab tensor objects; ``fb[b]``
    gives tensor views when they are wanted."""

    def __init__(self, dims):
        self.dims = [t.contiguous() for t in dims]
        self.N, self.M = self.dims[0].shape[0], self.dims[0].shape[2]
        self.n = [int(t.shape[1]) for t in self.dims]
        self.base = [t.data_ptr() for t in self.dims]
        self.stride = [int(t.shape[1] * t.shape[2]) * 8 for t in self.dims]

    def __len__(self):
        return self.N

    def __getitem__(self, b):
        return [t[b] for t in self.dims]

    def ptr(self, b, d, row=0):
        """Address of row ``row`` of slab b's factor of dim d."""
        return self.base[d] + b * self.stride[d] + row * self.M * 8

    def addrs(self, idx, d, row=0):
        """Addresses of row ``row`` of the factors of dim d of the slabs idx
        (a uint64 array)."""
        b = np.asarray(idx, dtype=np.uint64)
        return np.uint64(self.base[d] + row * self.M * 8) + b * np.uint64(self.stride[d])

    def ptrs(self, idx):
        """Factor pointers of the slabs idx, problem-major (driver order)."""
        import ctypes as C
        D = len(self.dims)
        b = np.asarray(idx, dtype=np.uint64)[:, None]
        a = np.asarray(self.base, dtype=np.uint64)[None, :] + b * np.asarray(self.stride, dtype=np.uint64)[None, :]
        return (C.c_void_p * (len(idx) * D)).from_buffer_copy(np.ascontiguousarray(a).tobytes())

    def clone(self):
        return FactorBatch([t.clone() for t in self.dims])


def ldw(w: int) -> int:
    return (w + 31) // 32 * 32


class Net:
    """Device weights (FP32 masters + BF16 copies), Adam state and buffers."""

    def __init__(self, h, widths, Ws, bs, device="cuda"):
        self.h = h
        self.widths = list(widths)
        self.L = len(widths) - 1
        self.master, self.bias, self.w16 = [], [], []
        for l, (W, b) in enumerate(zip(Ws, bs)):
            out, inp = W.shape
            P = torch.zeros((out, ldw(inp)), dtype=F32, device=device)
            P[:, :inp] = torch.tensor(np.asarray(W, dtype=np.float32), device=device)
            self.master.append(P)
            self.bias.append(torch.tensor(np.asarray(b, dtype=np.float32), device=device))
            self.w16.append(torch.zeros((out, ldw(inp)), dtype=torch.int16, device=device))
        self.params = self.master + self.bias
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.grads = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        # BF16 copies of the masters through the Adam kernel with a zero step
        for P, Q, m, v, g in zip(self.master, self.w16, self.m, self.v, self.grads):
            capi.taps_adam_step(h, P, g, m, v, 0.0, 1, p16=Q)
        self.struct = capi.mlp_struct(self.widths, self.w16, self.bias)
        self._cache = {}

    def cache(self, B):
        if B not in self._cache:
            nbytes = capi.taps_mlp_cache_bytes(self.struct, B)
            self._cache[B] = torch.empty(nbytes, dtype=torch.uint8, device=self.master[0].device)
        return self._cache[B]

    def forward(self, X):
        B = X.shape[0]
        Y = torch.empty((B, self.widths[-1]), dtype=F32, device=X.device)
        capi.taps_mlp_forward(self.h, self.struct, X, self.cache(B), Y)
        return Y

    def backward(self, B, dY):
        capi.taps_mlp_backward(self.h, self.struct, B, self.cache(B), dY, self.grads[: self.L],
                               self.grads[self.L:])

    def step(self, lr):
        self.t += 1
        for i, (p, g, m, v) in enumerate(zip(self.params, self.grads, self.m, self.v)):
            capi.taps_adam_step(self.h, p, g, m, v, lr, self.t, p16=self.w16[i] if i < self.L else None)


def param_features(case):
    return [2.0 * (getattr(case, n) - lo) / (hi - lo) - 1.0 for n, (lo, hi) in PARAM_RANGES.items()]


class Coarse:
    """Sampling at coarse nodes and prolongation back, for one axis."""

    def __init__(self, h, ax, nc, device="cuda"):
        self.h, self.ax, self.nc = h, ax, nc
        x = torch.tensor(ax.nodes(), dtype=F64, device=device)
        xc = torch.tensor(np.linspace(ax.lo, ax.hi, nc), dtype=F64, device=device)
        self.keep = [x, xc]
        fine = capi.Basis1D(ax.n, x.data_ptr(), ax.s, float(ax.a), ax.p, ax.n_gauss)
        L = 2 * ax.s + 2
        self.Ns = torch.empty((nc, L), dtype=F64, device=device)          # fine basis at coarse nodes
        self.fs = torch.empty(nc, dtype=torch.int32, device=device)
        capi.taps_shape1d(h, fine, xc, self.Ns, None, self.fs)
        s_c = min(2, (nc - 2) // 2)
        coarse = capi.Basis1D(nc, xc.data_ptr(), s_c, 20.0, min(2, s_c), 5)
        Lc = 2 * s_c + 2
        self.Np = torch.empty((ax.n, Lc), dtype=F64, device=device)       # coarse basis at fine nodes
        self.fp = torch.empty(ax.n, dtype=torch.int32, device=device)
        capi.taps_shape1d(h, coarse, x, self.Np, None, self.fp)

    def sample(self, U, out=None):
        out = torch.empty((self.nc, U.shape[1]), dtype=F64, device=U.device) if out is None else out
        capi.taps_interp1d(self.h, self.Ns, self.fs, self.ax.n, U, out)
        return out

    def prolong(self, Uc):
        out = torch.empty((self.ax.n, Uc.shape[1]), dtype=F64, device=Uc.device)
        capi.taps_interp1d(self.h, self.Np, self.fp, self.nc, Uc, out)
        return out


def ic_features(h, coarse4, V):
    """Carried field sampled on the 4 x 4 x 4 coarse grid (64 values)."""
    dev = coarse4[0].keep[0].device
    if V is None:
        return torch.zeros(64, dtype=F64, device=dev)
    Phis = [c.sample(v) for c, v in zip(coarse4, V)]
    out = torch.empty((4, 4, 4), dtype=F64, device=dev)
    capi.taps_reconstruct(h, Phis, V[0].shape[1], out, prec=capi.FP64, mode=capi.STORE)
    return out.permute(1, 2, 0).reshape(-1)      # plane-major k, i, j -> (i, j, k)


# ------------------------------------------------------------------ data


class Layout:
    """Target layout: canonical y, z, t factors at (ny_c, nz_c, nt_c) coarse
    nodes x M modes, each scaled by sqrt(n_d) so entries are O(1)."""

    def __init__(self, h, case, M, coarse=(32, 16, 32), device="cuda"):
        self.M = M
        self.axes = case.axes
        self.coarse = [Coarse(h, ax, nc, device) for ax, nc in zip(case.axes[1:], coarse)]
        self.ic4 = [Coarse(h, ax, 4, device) for ax in case.axes[:3]]
        self.scale = [float(np.sqrt(ax.n)) for ax in case.axes[1:]]
        self.sizes = [nc * M for nc in coarse]
        self.n_out = sum(self.sizes)
        self.h = h

    def target(self, U):
        """Canonical factors of one solved slab -> (n_out,) FP32 target."""
        can = [torch.empty_like(u) for u in U]
        capi.taps_canonicalize(self.h, U, can)
        parts = [c.sample(can[d + 1]) * s for d, (c, s) in enumerate(zip(self.coarse, self.scale))]
        return torch.cat([p.reshape(-1) for p in parts]).to(F32)

    def initial(self, y, fixed):
        """Network output (n_out,) -> fine initial factors [0, U_y, U_z, U_t];
        rows of fixed nodes set to zero."""
        return self.initial_batch(y.unsqueeze(0), fixed)[0]

    def initial_batch(self, Y, fixed):
        """Network outputs (N, n_out) -> FactorBatch of [0, U_y, U_z, U_t]
        per slab: one prolongation call per dim for the whole batch (the N
        coarse factors side by side as N*M columns)."""
        N, M = Y.shape[0], self.M
        dims, off = [], 0
        for d, (c, s, size) in enumerate(zip(self.coarse, self.scale, self.sizes)):
            Uc = (Y[:, off: off + size].to(F64) / s).reshape(N, c.nc, M).permute(1, 0, 2).reshape(c.nc, N * M)
            off += size
            Uf = c.prolong(Uc.contiguous()).reshape(c.ax.n, N, M).permute(1, 0, 2).contiguous()
            if fixed[d + 1]:
                Uf[:, torch.tensor(sorted(fixed[d + 1]), device=Y.device)] = 0.0
            dims.append(Uf)
        U0 = torch.zeros((N, self.axes[0].n, M), dtype=F64, device=Y.device)
        return FactorBatch([U0] + dims)

    def features(self, case, V):
        f = torch.tensor(param_features(case), dtype=F64, device=self.coarse[0].keep[0].device)
        return torch.cat([f, ic_features(self.h, self.ic4, V)]).to(F32)


def sweep_history(h, probs, Us, sweeps):
    """Algorithm 1 on a batch, one sweep per call: rho after every sweep
    (sweeps x B array; NaN marks a breakdown)."""
    hist = []
    for _ in range(sweeps):
        _, rho = capi.taps_als_batched(h, [p.struct for p in probs], Us, 0.0, 1)
        hist.append(rho)
    return np.array(hist)


def make_chains(h, cases_a, cases_b, M, Kc, sweeps, comp_sweeps, seed, layout):
    """Two-slab chains: slab A from zero initial condition, slab B carrying
    A's compressed end state.  Returns features, targets and the plain
    initialisation's residual history of every slab."""
    from . import chain
    import taps_workloads as W
    B = len(cases_a)
    probs_a = [chain.slab_problem(h, c) for c in cases_a]
    Ua = [p.factors(W.initial_factors(c.axes, M, seed + i)) for i, (p, c) in enumerate(zip(probs_a, cases_a))]
    hist_a = sweep_history(h, probs_a, Ua, sweeps)
    comp = [chain.compression_problem(h, p, None, U, Kc) for p, U in zip(probs_a, Ua)]
    Vs = [cp.factors(W.initial_factors(c.axes[:3], Kc, seed + 10_000 + i)) for i, (cp, c) in enumerate(zip(comp, cases_a))]
    capi.taps_als_batched(h, [cp.struct for cp in comp], Vs, 0.0, comp_sweeps)
    probs_b = [chain.slab_problem(h, c, V) for c, V in zip(cases_b, Vs)]
    Ub = [p.factors(W.initial_factors(c.axes, M, seed + 20_000 + i)) for i, (p, c) in enumerate(zip(probs_b, cases_b))]
    hist_b = sweep_history(h, probs_b, Ub, sweeps)
    X = torch.stack([layout.features(c, None) for c in cases_a] + [layout.features(c, V) for c, V in zip(cases_b, Vs)])
    T = torch.stack([layout.target(U) for U in Ua + Ub])
    return {"X": X, "T": T, "hist": np.concatenate([hist_a, hist_b], axis=1), "V": Vs,
            "cases": list(cases_a) + list(cases_b)}


def train(h, net, X, T, steps, lr, batch, seed):
    """Adam on the squared error over mini-batches (seeded order); returns the
    loss of every step."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = X.shape[0]
    losses = []
    loss = torch.empty(1, dtype=F64, device=X.device)
    for it in range(steps):
        idx = torch.tensor(rng.choice(n, size=min(batch, n), replace=False), device=X.device)
        xb, tb = X[idx].contiguous(), T[idx].contiguous()
        y = net.forward(xb)
        dY = torch.empty_like(y)
        capi.taps_mlp_mse(h, y, tb, dY, loss)
        net.backward(xb.shape[0], dY)
        net.step(lr)
        losses.append(loss)
        loss = torch.empty(1, dtype=F64, device=X.device)
    return torch.cat(losses).cpu().numpy()


def restart_plain(rho1, rho2, plain_median_rho1):
    """True when the warm start lost: its sweep-1 residual is above the plain
    start's median, it grew from sweep 1 to 2, or either residual is not a
    number (a breakdown counts as a loss)."""
    return not (rho1 <= plain_median_rho1) or not (rho2 <= rho1)


# ------------------------------------------------------------- streaming


def pack_problems(probs):
    """The problem records of probs (objects with .struct) as one ctypes
    array, in order."""
    return (capi.Problem * len(probs))(*[p.struct for p in probs])


def solve_stream(h, probs, U, tol, cap, slots, U_plain=None, median_rho1=None, on_done=None, on_done_batch=None,
                 first_sweep_all=False):
    """Continuous batching of Algorithm 1: up to ``slots`` slabs in flight,
    one batched sweep (taps_als_batched) per round; a slab leaves as soon as
    its projected residual reaches tol, it has run ``cap`` sweeps, or its
    solve broke down (NaN residual), and the next waiting slab takes its
    place, so the kernels stay busy while slabs converge at different speeds.

    first_sweep_all: every slab runs its first sweep before any runs its
    second (rounds of ``slots`` slabs in input order), and the slabs still
    unsolved then wait in order of decreasing residual (a restarted slab
    first), so the slabs that need the most sweeps start early and the last
    rounds, which run part-empty at nearly a full round's cost, are few.
    For slabs of one grid and load structure (the launch parameters then do
    not depend on which slabs share a round) a slab's sweeps and residuals
    do not depend on the schedule: the batched kernels treat every problem
    of a launch alone.

    With U_plain and median_rho1 given, U holds warm starts and the fallback
    rule is applied: a slab whose warm start lost (sweep-1 residual above
    median_rho1, or growing from sweep 1 to 2, or a breakdown in either
    sweep) restarts from its U_plain factors with a fresh sweep count.
    on_done(i) is called for every slab as it leaves; on_done_batch(list)
    once per round with all slabs that left in it.
    U (and U_plain) may be FactorBatch objects (addresses computed per
    round) or lists of per-slab factor lists.  probs is a list of problem
    objects (with .struct) or their records packed once by pack_problems
    (the objects must then outlive the call: the records point into their
    device buffers).
    Returns (sweeps run per slab, final residual per slab, number of
    restarts, outcome per slab: 0 reached tol, 1 stopped at the cap,
    2 broke down)."""
    import ctypes as C
    n = len(probs)
    allp = probs if isinstance(probs, C.Array) else pack_problems(probs)
    psize = C.sizeof(capi.Problem)
    # a view of the records as rows of 8-byte words (the struct holds
    # pointers and doubles, so its size is a multiple of 8); allp outlives
    # the rounds
    allp_words = np.frombuffer(allp, dtype=np.uint64).reshape(n, psize // 8)

    def prob_array(idx):
        if len(idx) == n and np.array_equal(idx, np.arange(n)):
            return allp
        # one gather; the ctypes array keeps the gathered rows alive
        return (capi.Problem * len(idx)).from_buffer(allp_words[idx])

    # the waiting slabs in order (wait[w0:] still waits) and the slabs in
    # flight, as integer arrays
    wait, w0 = np.arange(n, dtype=np.intp), 0
    active = np.zeros(0, dtype=np.intp)
    # per-slab state as arrays: a round's bookkeeping is a few vector
    # operations, not a Python loop over the slabs in flight (the GPU waits
    # for it between rounds)
    count = np.zeros(n, dtype=np.int64)       # sweeps since the (re)start
    total = np.zeros(n, dtype=np.int64)       # sweeps run
    rho = np.full(n, np.nan)
    rho1 = np.full(n, np.nan)
    outcome = np.ones(n, dtype=np.int64)
    restarted = np.zeros(n, dtype=bool)

    def one_round(act):
        Ua = U.ptrs(act) if isinstance(U, FactorBatch) else [U[i] for i in act.tolist()]
        _, r = capi.taps_als_batched(h, prob_array(act), Ua, 0.0, 1, arrays=True)
        count[act] += 1
        total[act] += 1
        rho[act] = r
        lost = np.zeros(len(act), dtype=bool)
        if U_plain is not None:
            fresh = ~restarted[act]
            c = count[act]
            first = fresh & (c == 1)
            rho1[act[first]] = r[first]
            # the fallback rule (restart_plain) on every slab of the round;
            # a comparison with NaN is false, so a breakdown is a loss
            r1 = rho1[act]
            lost = (first & np.isnan(r)) | (fresh & (c == 2) & (~(r1 <= median_rho1) | ~(r <= r1)))
            for i in act[lost].tolist():
                for u, u0 in zip(U[i], U_plain[i]):
                    u.copy_(u0)
            restarted[act[lost]] = True
            count[act[lost]] = 0
        fin = ~lost & ((r <= tol) | np.isnan(r) | (count[act] >= cap))
        fa, fr = act[fin], r[fin]
        outcome[fa] = np.where(fr <= tol, 0, np.where(np.isnan(fr), 2, 1))
        done = fa.tolist()
        if on_done is not None:
            for i in done:
                on_done(i)
        if done and on_done_batch is not None:
            on_done_batch(done)
        return act[~fin]

    if first_sweep_all:
        rest = []
        while w0 < n:
            k = min(slots, n - w0)
            rest.append(one_round(wait[w0:w0 + k]))
            w0 += k
        # hardest first: restarted slabs (count 0), then by decreasing residual
        # (a stable sort, as the slabs' input order breaks ties)
        ra = np.concatenate(rest)
        wait, w0 = ra[np.lexsort((-rho[ra], count[ra] != 0))], 0
    while w0 < len(wait) or len(active):
        k = min(slots - len(active), len(wait) - w0)
        if k > 0:
            active = np.concatenate([active, wait[w0:w0 + k]])
            w0 += k
        active = one_round(active)
    return total.tolist(), rho.tolist(), int(restarted.sum()), outcome.tolist()
