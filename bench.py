#!/usr/bin/env python
"""Benchmark: TAPS slab solves/s on one MI355X, warm-started and batched
against the plain form, at the same residual.

Workload: --slabs independent space-time heat slabs on one grid, 512 x 512 x
128 nodes x 257 time nodes, M = 40 modes, moving Gaussian source with per-slab
power, radius, conductivity and scan line.  Every kernel of the path runs on
the GPU through the C ABI, with inputs resident in HBM before timing starts.

A step solves all slabs: the learned warm start (network forward and
prolongation of its coarse factors), then Algorithm 1 in batched form (Grams,
couplings, dim solves by fast diagonalisation -- the complex Schur route the
paper names -- balancing with the relative change, projected residual) with
continuous batching: --batch slabs in flight, one workgroup each per kernel;
a slab leaves when its residual reaches the target, at the sweep cap, or on a
breakdown, and the next takes its slot, so with more slabs than slots (by
default 4096 through 2048) only the last rounds of a step run part-empty.
The fallback rule runs after sweeps 1 and 2, and a BF16 reconstruction of
the end-time field of every slab that leaves (per-plane max, sum of squares
and hot-point count), one batched call per round, is part of the step.

Target residual: Algorithm 1 on these slabs stalls far above 1e-8 (the
projected residual of a rank-M space-time field on 257 time nodes wanders at
about 1e-2; the set-up measures that floor on --floor-slabs slabs over
--floor-sweeps sweeps and reports it), so every variant runs to a common
stated tolerance: the residual that the plain initialisation reaches, on the
network's training slabs, after --sweeps sweeps (their median; the default 3
is the sweep count the paper reports as enough), capped at 2 x --sweeps.
`value` counts only slabs that reached it; slabs stopped at the cap and
breakdowns are reported beside it.  The network is trained before timing,
on two-slab chains drawn separately from the benchmark slabs.  The plain
form (one slab at a time, random start, same solver) is timed per slab on
--plain-slabs slabs after an untimed warm-up solve, median taken; the batched
form with random starts is timed like the warm-started one.  Kernel times
come from a separate profiled step (HIP events on the launch stream), never
from the timed steps.

Roofline: the dominant kernel is the one of the two largest kernels of the
fast diagonalisation with more kernel time in the profiled step, the banded
stage k_fd_solve or the real Schur kernel k_fd_schur; each is reported with
the method's own work (flops of the eliminations and transforms, or of the
Hessenberg reduction and Francis QR; the kernel's scratch traffic is not
work) against the FP64 peak, as both sit above the FP64 ridge.  The
contractions (Grams, load Grams, force) are reported against HBM with the
method's bytes, the BF16 reconstruction against the BF16 matrix-core peak
with the method's 2 M flops per point.  The CPU baseline is the oracle on
a bounded sample: one sweep of --cpu-slabs slabs in parallel processes, one
per host core.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 (vector and matrix)
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
# Memory traffic per launch over the method's bytes per launch, from two
# rocprofv3 counter runs of this script (FETCH_SIZE, then WRITE_SIZE, each
# scaled by the same counter on a plain device copy of known size), valid
# for the kernel sources with these SHA-256 prefixes only (None: not measured
# for the current sources).
TRAFFIC = {"k_fd_solve": 10.228, "k_fd_schur": 1.019, "contract": 2.976, "contract_spt": 1.821,
           "sources": "13d91a1be39c9708"}
TRAFFIC_SOURCES = ("taps_solve.hip", "taps_device.hpp", "taps_batch.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def family(n, seed, **grid):
    import taps_workloads as W
    return W.heat_slab_family(n, seed=seed, **grid)


def _oracle_sweep_worker(job):
    """One oracle sweep of one slab (a CPU worker process, one thread)."""
    import taps_workloads as W
    from oracle import als, problems, separated
    case = job
    prob = problems.heat_slab(case)
    U = W.initial_factors(case.axes, case.M, case.seed)
    t0 = time.perf_counter()
    als.sweep(prob, U)
    als.balance(U)
    rho = separated.residual_norm(prob, U)
    return time.perf_counter() - t0, rho


def cpu_baseline(cases, sweeps_per_solve):
    """The oracle, as it stands, on a bounded sample: one sweep of each of
    len(cases) slabs, one worker process per host core (single-threaded BLAS),
    scaled to slab solves/s."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16, len(cases))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_sweep_worker, list(cases))
    wall = time.perf_counter() - t0
    per = [r[0] for r in res]
    log(f"cpu oracle: {len(cases)} slabs x 1 sweep on {cores} processes in {wall:.1f} s "
        f"(per slab {np.median(per):.1f} s, rho {np.median([r[1] for r in res]):.3e})")
    sweeps_per_s = len(cases) / wall
    return {
        "value": sweeps_per_s / sweeps_per_solve,
        "unit": "slab solves/s",
        "cores": int(cores),
        "kind": "oracle",
        "cpu": model,
        "sample": f"1 sweep of each of {len(cases)} benchmark slabs on {cores} single-threaded processes "
                  f"({wall:.1f} s wall, median {np.median(per):.1f} s per slab-sweep, process start-up included), "
                  f"scaled to {sweeps_per_solve:.2f} sweeps per solve",
    }


def sources_digest():
    import hashlib
    hs = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        hs.update(open(os.path.join(ROOT, "paper_2503_13933_amd", "csrc", name), "rb").read())
    return hs.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--nt", type=int, default=257)
    ap.add_argument("--M", type=int, default=40)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=3, help="plain sweep budget that sets the target residual")
    ap.add_argument("--target-sweeps", type=int, default=3,
                    help="plain sweeps behind the warm-start network's training targets (at least --sweeps)")
    ap.add_argument("--batch", type=int, default=2048, help="slabs in flight, one workgroup each")
    ap.add_argument("--stream-order", choices=["hardest-first", "input"], default="hardest-first",
                    help="continuous batching: first sweep of every slab, then the unsolved ones by decreasing "
                         "residual (hardest-first), or slabs strictly in input order")
    ap.add_argument("--slabs", type=int, default=4096,
                    help="slabs solved per step (streamed through --batch slots)")
    ap.add_argument("--train-chains", type=int, default=4096)
    ap.add_argument("--train-steps", type=int, default=12000)
    ap.add_argument("--Kc", type=int, default=8, help="modes of the carried initial condition")
    ap.add_argument("--coarse", default="32,16,32", help="coarse nodes of the predicted y, z, t factors")
    ap.add_argument("--solver", choices=["fastdiag", "blocklu"], default="fastdiag",
                    help="dim solver: fast diagonalisation (complex Schur) or block LU")
    ap.add_argument("--floor-slabs", type=int, default=64)
    ap.add_argument("--floor-sweeps", type=int, default=50)
    ap.add_argument("--plain-slabs", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-random", action="store_true", help="skip the random-start batched variant")
    ap.add_argument("--cpu-slabs", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the space-parameter-time batch")
    ap.add_argument("--no-autotune", action="store_true",
                    help="no tuner and no captured graphs (host launches; rocprofv3 counter runs abort on graph "
                         "launches); --lgram-rows sets the row split instead")
    ap.add_argument("--lgram-rows", type=int, default=0, help="load-Gram row split without the tuner (0: default)")
    ap.add_argument("--c3-only", action="store_true", help="run only the space-parameter-time batch")
    ap.add_argument("--c3-sweeps", type=int, default=3)
    ap.add_argument("--no-large", action="store_true", help="skip the large single slab (15000^2 x 15 x 513, M=60)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="end with a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by slab, "
              "one batch per GPU, with no communication inside a solve", file=sys.stderr)
        sys.exit(2)

    import torch
    import taps_workloads as W
    from paper_2503_13933_amd import capi, chain, warmstart as ws

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.c3_only:
        # the space-parameter-time batch alone (for kernel traces of it)
        res = c3_batch(capi, torch, args)
        calibration_copy(args, torch)
        print(json.dumps({"spt_batch": res}), flush=True)
        return
    grid = dict(nx=args.nx, ny=args.nx, nz=args.nz, nt=args.nt, M=args.M)
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG if args.solver == "fastdiag" else capi.SOLVER_BLOCK_LU)
    M, B, N, cap = args.M, args.batch, args.slabs, 2 * args.sweeps

    # ---- set-up (untimed): benchmark slabs, training chains, network
    t0 = time.perf_counter()
    cases = family(N, args.seed, **grid)
    probs = [chain.slab_problem(h, c) for c in cases]
    packed = ws.pack_problems(probs)     # the records of all slabs (probs keeps their buffers)
    # random starts of all slabs, one (N, n_d, M) tensor per dim (a slab's factors are slices)
    U0_host = [W.initial_factors(c.axes, M, c.seed) for c in cases]
    U_plain_big = [torch.tensor(np.stack([u[d] for u in U0_host]), dtype=torch.float64, device="cuda")
                   for d in range(4)]
    del U0_host
    U_plain = ws.FactorBatch(U_plain_big)
    layout = ws.Layout(h, cases[0], M, coarse=tuple(int(v) for v in args.coarse.split(",")))
    n_tr = args.train_chains
    tr_a = family(n_tr, args.seed + 101, **grid)
    tr_b = [W.replace(c, x_start=0.9) for c in family(n_tr, args.seed + 202, **grid)]
    data = ws.make_chains(h, tr_a, tr_b, M, args.Kc, max(args.sweeps, args.target_sweeps), 4, 1000 + args.seed,
                          layout)
    hist = data["hist"][:, :n_tr]          # first slabs of the chains: zero initial condition, like the batch
    rho_star = float(np.nanmedian(hist[args.sweeps - 1]))
    med1 = float(np.nanmedian(hist[0]))
    widths = [data["X"].shape[1], 256, 256, 256, data["T"].shape[1]]
    net = ws.Net(h, widths, *W.mlp_init(widths, args.seed))
    losses = ws.train(h, net, data["X"], data["T"], args.train_steps, 1e-3, 64, args.seed)
    X_bench = torch.stack([layout.features(c, None) for c in cases])
    fixed = [ax.fixed for ax in cases[0].axes]
    del data
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.1f}s: {N} slabs {[a.n for a in cases[0].axes]} M={M}; target rho {rho_star:.3e} "
        f"(plain median after {args.sweeps} sweeps on {n_tr} training slabs); network loss "
        f"{losses[:10].mean():.3e} -> {losses[-50:].mean():.3e}")

    # ---- floor of Algorithm 1 on these slabs (untimed): rho and the paper's
    # relative change over many sweeps from the plain start
    nf = min(args.floor_slabs, N)
    floor = None
    if nf and args.floor_sweeps:
        Uf = ws.FactorBatch([t[:nf].clone() for t in U_plain_big])
        pf = [p.struct for p in probs[:nf]]
        rh, ch = [], []
        for _ in range(args.floor_sweeps):
            c = []
            _, r = capi.taps_als_batched(h, pf, Uf.ptrs(list(range(nf))), 0.0, 1, change=c)
            rh.append(r)
            ch.append(c)
        rh, ch = np.array(rh), np.array(ch)
        med_r, med_c = np.nanmedian(rh, axis=1), np.nanmedian(ch, axis=1)
        floor = {"slabs": nf, "sweeps": args.floor_sweeps,
                 "median_rho_by_sweep": [float(v) for v in med_r],
                 "median_change_by_sweep": [float(v) for v in med_c],
                 "rho_floor": float(np.nanmin(med_r)), "rho_floor_sweep": int(np.nanargmin(med_r)) + 1,
                 "change_floor": float(np.nanmin(med_c)),
                 "breakdowns": int(np.sum(np.isnan(rh[-1])))}
        del Uf
        log(f"floor: median rho over {args.floor_sweeps} sweeps of {nf} slabs: min {floor['rho_floor']:.3e} "
            f"at sweep {floor['rho_floor_sweep']}, last {med_r[-1]:.3e}; median relative change min "
            f"{floor['change_floor']:.3e}, last {med_c[-1]:.3e}")

    # ---- tuning of the batched driver on the first round's slabs (untimed):
    # load-Gram row split and graph length, applied to the stream's handle
    tune = None
    if args.no_autotune:
        capi.taps_set_tuning(h, lgram_rows=args.lgram_rows)
    else:
        nb = min(B, N)
        Ut = ws.FactorBatch([t[:nb].clone() for t in U_plain_big])
        tb = (capi.Problem * nb)(*[p.struct for p in probs[:nb]])
        tn, tms = capi.taps_autotune(h, tb, Ut.ptrs(list(range(nb))))
        tune = {"lgram_rows": tn.lgram_rows, "graph_sweeps": tn.graph_sweeps, "candidates_ms": tms}
        del Ut
        log(f"autotune on {nb} slabs: lgram_rows {tn.lgram_rows}, graph_sweeps {tn.graph_sweeps} "
            f"(ms per sweep {[round(m, 2) for m in tms]})")

    stats = torch.empty((N, args.nz, 4), dtype=torch.float64, device="cuda")

    n_pts, nt, s_row = [ax.n for ax in cases[0].axes[:3]], cases[0].axes[3].n, args.nz * 4 * 8

    def reconstruct(U, done):
        # end-time fields (time factor's last row as mode weights) of the
        # slabs that left this round, in one call, by address (address
        # arrays, no per-slab Python work)
        idx = np.asarray(done, dtype=np.uint64)
        phis = np.stack([U.addrs(idx, 0), U.addrs(idx, 1), U.addrs(idx, 2)], axis=1)
        outs = np.uint64(stats.data_ptr()) + idx * np.uint64(s_row)
        capi.taps_reconstruct_batched(h, phis, M, outs, prec=capi.BF16, mode=capi.REDUCE,
                                      mode_ws=U.addrs(idx, 3, nt - 1), thr=1000.0, n_pts=n_pts)

    hardest = args.stream_order == "hardest-first"

    def step_warm():
        Y = net.forward(X_bench)
        U = layout.initial_batch(Y, fixed)
        return ws.solve_stream(h, packed, U, rho_star, cap, B, U_plain=U_plain, median_rho1=med1,
                               on_done_batch=lambda done: reconstruct(U, done), first_sweep_all=hardest)

    def step_random_batched():
        U = U_plain.clone()
        return ws.solve_stream(h, packed, U, rho_star, cap, B, on_done_batch=lambda done: reconstruct(U, done),
                               first_sweep_all=hardest)

    def timed(fn, label):
        for w in range(args.warmup):
            fn()
            torch.cuda.synchronize()
        torch.cuda.synchronize()
        t = time.perf_counter()
        tot_sw, solved, capped, broke, fb = 0, 0, 0, 0, 0
        for k in range(args.steps):
            sw, rho, restarts, outcome = fn()
            oc = np.array(outcome)
            tot_sw += sum(sw)
            solved += int(np.sum(oc == 0))
            capped += int(np.sum(oc == 1))
            broke += int(np.sum(oc == 2))
            fb += restarts
            log(f"{label} step {k + 1}/{args.steps}: sweeps {min(sw)}..{max(sw)}, reached target "
                f"{np.mean(oc == 0):.4f}, capped {np.sum(oc == 1)}, breakdowns {np.sum(oc == 2)}, fallbacks {restarts}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        tot = N * args.steps
        return {"elapsed_s": el, "solved_per_s": solved / el, "slabs_per_s": tot / el,
                "sweeps_per_slab": tot_sw / tot, "reached_target": solved / tot, "capped": capped / tot,
                "breakdowns": broke / tot, "fallbacks": fb / tot}

    warm = timed(step_warm, "warm+batched")
    rand = None if args.no_random else timed(step_random_batched, "random+batched")

    # ---- kernel times: one profiled warm step, apart from the timed ones
    capi.taps_profile_enable(h, True)
    step_warm()
    torch.cuda.synchronize()
    capi.taps_profile_enable(h, False)
    prof = {name: capi.taps_profile_read(h, fam) for name, fam in (
        ("solve", capi.PROF_SOLVE), ("eig", capi.PROF_EIG), ("schur", capi.PROF_SCHUR),
        ("contract", capi.PROF_CONTRACT), ("recon", capi.PROF_RECON))}

    # ---- plain form: one slab at a time from its random start, same solver
    plain = None
    if not args.no_plain and N > args.plain_slabs:
        def plain_solve(b):
            U = [u.clone() for u in U_plain[b]]
            sw, rho, _ = capi.taps_als(h, probs[b].struct, U, rho_star, cap)
            capi.taps_reconstruct(h, U[:3], M, stats[b], prec=capi.BF16, mode=capi.REDUCE, mode_w=U[3][-1],
                                  thr=1000.0)
            return sw, rho
        plain_solve(N - 1)                              # untimed: first-call buffers and launches
        torch.cuda.synchronize()
        times, sws, reached = [], [], []
        for b in range(args.plain_slabs):
            tp = time.perf_counter()
            sw, rho = plain_solve(b)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - tp)
            sws.append(sw)
            reached.append(rho <= rho_star)
        med = float(np.median(times))
        plain = {"value": float(np.mean(reached)) / med, "median_s_per_slab": med, "slabs": args.plain_slabs,
                 "sweeps_per_slab": float(np.mean(sws)), "reached_target": float(np.mean(reached))}
        log(f"plain form: median {med:.3f} s per slab over {args.plain_slabs} slabs, "
            f"{np.mean(sws):.2f} sweeps, reached {np.mean(reached):.2f}")

    # ---- reduced-precision reconstruction of the large-slab subvolume shape:
    # 2048 x 2048 planes, M = 60 (256 planes of the 2048^3 subvolume)
    rec = recon_large(h, capi, torch)

    # ---- the large single slab: sweeps and its 2048^3 subvolume
    large = None if args.no_large else large_slab(capi, torch)

    # ---- the uneven space-parameter-time batch: autotuned, graph-replayed
    c3 = None if args.no_c3 else c3_batch(capi, torch, args)

    digest = sources_digest()
    measured = TRAFFIC["sources"] == digest

    def roof_alu(name, what, fam):
        n_l, ms_l, fl_l, by_l = prof[fam]
        sec = ms_l * 1e-3
        ach = fl_l / sec / 1e12 if n_l else 0.0
        ratio = TRAFFIC.get(name) if measured else None
        return {"bound": "alu", "kernel": f"{name} ({what})", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                "traffic": ratio * by_l / n_l if (ratio and n_l) else None,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "launches": n_l, "avg_launch_ms": ms_l / max(1, n_l), "flops_per_launch": fl_l / max(1, n_l),
                "method_bytes_per_launch": by_l / max(1, n_l),
                "method_hbm_frac": (by_l / sec / 1e9) / HBM_PEAK_GBS if n_l else 0.0}

    fd = args.solver == "fastdiag"
    if fd:
        r_solve = roof_alu("k_fd_solve", "banded stage of the fast diagonalisation: two complex transforms and M "
                           "banded complex eliminations per system, one 64-lane wave each", "solve")
        r_schur = roof_alu("k_fd_schur", "real Schur form: Hessenberg reduction and Francis QR with Schur vectors, "
                           "one 64-lane wave per system", "schur")
        roof, other = (r_solve, r_schur) if prof["solve"][1] >= prof["schur"][1] else (r_schur, r_solve)
    else:
        roof, other = roof_alu("k_block_lu_mfma_batched", "block-banded FP64 dim solve", "solve"), None
    n_c, ms_c, fl_c, by_c = prof["contract"]
    ratio_c = TRAFFIC.get("contract") if measured else None
    contract = {"bound": "hbm", "kernels": "kb_gram_partial/sum, kb_lgram_partial/sum, kb_couple, kb_load_terms, "
                                            "kb_load_weights(_fused)/kb_wsum, kb_force(/sum)",
                "achieved": by_c / (ms_c * 1e-3) / 1e9 if n_c else 0.0, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "launch_groups": n_c, "ms_per_step": ms_c, "method_bytes_per_step": by_c,
                "fp64_tflops": fl_c / (ms_c * 1e-3) / 1e12 if n_c else 0.0,
                "traffic_per_step": ratio_c * by_c if ratio_c else None}
    contract["frac"] = contract["achieved"] / HBM_PEAK_GBS
    n_e, ms_e, fl_e, _ = prof["eig"]
    eig_tf = fl_e / (ms_e * 1e-3) / 1e12 if n_e else 0.0
    n_r, ms_r, fl_r, _ = prof["recon"]
    rec_tf = fl_r / (ms_r * 1e-3) / 1e12 if n_r else 0.0
    value = warm["solved_per_s"]
    out = {
        "metric": "TAPS slab solves/s at rel. residual 1e-8; warm-start+batched vs plain",
        "value": value,
        "unit": "slab solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * warm["elapsed_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{N} x heat_slab {args.nx}x{args.nx}x{args.nz}x{args.nt} M={M}, learned warm start, "
                         f"{B} in flight (continuous batching, {args.stream_order}), to the plain {args.sweeps}-sweep "
                         f"median projected "
                         f"residual {rho_star:.3e} (cap {cap} sweeps), BF16 end-time reconstruction"),
            "variant": "warm-start+batched",
            "solver": args.solver,
            "batch": B,
            "stream_order": args.stream_order,
            "slabs_per_step": N,
            "target_rho": rho_star,
            "target_note": "Algorithm 1 stalls far above 1e-8 on these slabs (see floor); value counts only "
                           "slabs whose projected residual reached target_rho",
            "floor": floor,
            "tuning": tune,
            "warm_batched": warm,
            "random_start_batched": rand,
            "plain": plain,
            "warm_batched_over_plain": (value / plain["value"]) if plain and plain["value"] > 0 else None,
            "warm_over_random_batched": (value / rand["solved_per_s"]) if rand and rand["solved_per_s"] > 0
            else None,
            "setup_s": setup_s,
            "profiled_step_ms": {k: v[1] for k, v in prof.items()},
            "eig_stage": {"kernels": "k_fd_inverse + k_fd_schur + k_fd_vectors", "launch_groups": n_e,
                          "ms_per_step": ms_e, "fp64_tflops": eig_tf, "fp64_frac": eig_tf / FP64_PEAK_TFLOPS}
            if fd else None,
            "second_kernel_roofline": other,
            "contract_roofline": contract,
            "recon_in_step": {"launches": n_r, "ms_per_step": ms_r, "bf16_tflops_at_M": rec_tf,
                              "bf16_frac": rec_tf / BF16_PEAK_TFLOPS},
            "recon_2048_planes_M60": rec,
            "large_slab": large,
            "spt_batch": c3,
            "traffic_sources_sha256": digest,
        },
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        spb = rand["sweeps_per_slab"] if rand else warm["sweeps_per_slab"]
        out["cpu_baseline"] = cpu_baseline(cases[:args.cpu_slabs], spb)
    calibration_copy(args, torch)
    h.close()
    print(json.dumps(out), flush=True)


def calibration_copy(args, torch):
    """A plain device copy of --calibration-copy-mib MiB (its source filled
    first): the known byte counts that scale the memory counters."""
    if not args.calibration_copy_mib:
        return
    n = args.calibration_copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    log(f"calibration copy: {args.calibration_copy_mib} MiB")
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def c3_batch(capi, torch, args):
    """64 space-parameter-time slabs (x, y, z, P, r, k, t; n_x..n_t drawn from
    64..1024, 32 nodes for P, r, k; M = 30; R = 32 n_t load terms): the
    autotuner picks the load-Gram row split (and reports its graph-length
    choice) on the batch, then --c3-sweeps sweeps of Algorithm 1 run through
    the batched driver as one captured HIP graph, timed; a second, profiled
    run (host launches) gives the contraction kernels' time against their
    bytes."""
    import taps_workloads as W
    from paper_2503_13933_amd import problem
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    t0 = time.perf_counter()
    cases = W.spt_batch(64, 64, 1024, 32, M=30, seed=3)
    probs = [problem.spt_slab(h, c) for c in cases]
    U0 = [p.factors(W.initial_factors(c.axes, c.M, c.seed)) for p, c in zip(probs, cases)]
    structs = [p.struct for p in probs]
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    f_bytes = sum(8.0 * p.axes[d].F.numel() for p in probs for d in range(7))
    if args.no_autotune:
        capi.taps_set_tuning(h, lgram_rows=args.lgram_rows)
        tune, tms = capi.taps_get_tuning(h), []
        graph = 0
    else:
        tune, tms = capi.taps_autotune(h, structs, U0)
        graph = args.c3_sweeps
    torch.cuda.synchronize()
    log(f"c3: 64 space-parameter-time slabs set up in {setup:.1f} s ({f_bytes / 1e9:.2f} GB of load columns); "
        f"lgram_rows {tune.lgram_rows}, tuner's graph_sweeps {tune.graph_sweeps} "
        f"(ms per sweep {[round(m, 2) for m in tms]})")
    # the timed sweeps replay one captured graph holding all of them (the
    # tuner's row split kept); host launches without the tuner
    capi.taps_set_tuning(h, graph_sweeps=graph)
    U = [[u.clone() for u in Ub] for Ub in U0]
    capi.taps_als_batched(h, structs, U, 0.0, args.c3_sweeps)   # warm-up and graph capture
    U = [[u.clone() for u in Ub] for Ub in U0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    chg = []
    sw, rho = capi.taps_als_batched(h, structs, U, 0.0, args.c3_sweeps, change=chg)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    U = [[u.clone() for u in Ub] for Ub in U0]
    capi.taps_profile_enable(h, True)
    capi.taps_als_batched(h, structs, U, 0.0, args.c3_sweeps)
    torch.cuda.synchronize()
    capi.taps_profile_enable(h, False)
    n_c, ms_c, fl_c, by_c = capi.taps_profile_read(h, capi.PROF_CONTRACT)
    n_s, ms_s, _, _ = capi.taps_profile_read(h, capi.PROF_SOLVE)
    n_e, ms_e, _, _ = capi.taps_profile_read(h, capi.PROF_EIG)
    h.close()
    gbs = by_c / (ms_c * 1e-3) / 1e9 if n_c else 0.0
    log(f"c3: {args.c3_sweeps} sweeps in {el * 1e3:.1f} ms ({el / args.c3_sweeps * 1e3:.1f} ms per sweep); "
        f"median rho {np.nanmedian(rho):.3e}; contractions {ms_c / args.c3_sweeps:.2f} ms per sweep at "
        f"{gbs:.0f} GB/s of method bytes")
    return {"workload": "64 x spt_slab (x,y,z,P,r,k,t), n_x..n_t ~ U{64..1024}, 32 nodes for P, r, k, M=30, "
                        "R = 32 n_t load terms, fast diagonalisation (block LU for P and r)",
            "setup_s": setup, "load_column_gb": f_bytes / 1e9,
            "tuning": {"lgram_rows": tune.lgram_rows, "graph_sweeps": tune.graph_sweeps, "candidates_ms": tms},
            "graph_sweeps_timed": graph,
            "sweeps": args.c3_sweeps, "ms_per_sweep": el / args.c3_sweeps * 1e3,
            "problem_sweeps_per_s": 64 * args.c3_sweeps / el, "median_rho": float(np.nanmedian(rho)),
            "median_change": float(np.nanmedian(chg)),
            "contract_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": gbs / HBM_PEAK_GBS, "ms_per_sweep": ms_c / args.c3_sweeps,
                                  "method_bytes_per_sweep": by_c / args.c3_sweeps,
                                  "traffic_per_sweep": (TRAFFIC["contract_spt"] * by_c / args.c3_sweeps
                                                        if TRAFFIC["sources"] == sources_digest() else None),
                                  "fp64_tflops": fl_c / (ms_c * 1e-3) / 1e12 if n_c else 0.0},
            "profiled_ms_per_sweep": {"contract": ms_c / args.c3_sweeps, "solve": ms_s / args.c3_sweeps,
                                      "eig": ms_e / args.c3_sweeps}}


def large_slab(capi, torch, sweeps=3):
    """The large single slab (x, y: 15000 nodes over 15 mm, z: 15, t: 513,
    M = 60): Algorithm 1 sweeps from the random start with the fast
    diagonalisation, timed (wall clock and the library's kernel events), and
    the BF16 / FP32 / FP64 reductions of the 2048^3 subvolume around the melt
    pool at the slab's end time, timed by the library's kernel events."""
    import taps_workloads as W
    from paper_2503_13933_amd import problem
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    case = W.large_slab()
    t0 = time.perf_counter()
    dev = problem.heat_slab(h, case)
    U0 = W.initial_factors(case.axes, case.M, case.seed)
    U = dev.factors(U0)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    capi.taps_als(h, dev.struct, [u.clone() for u in U], 0.0, 1)      # workspace growth, untimed
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, rho, hist = capi.taps_als(h, dev.struct, U, 0.0, sweeps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    U = dev.factors(U0)
    capi.taps_profile_enable(h, True)
    capi.taps_als(h, dev.struct, U, 0.0, sweeps)
    torch.cuda.synchronize()
    capi.taps_profile_enable(h, False)
    fam = {nm: capi.taps_profile_read(h, f) for nm, f in (("solve", capi.PROF_SOLVE), ("eig", capi.PROF_EIG),
                                                         ("contract", capi.PROF_CONTRACT))}
    # 2048^3 points about the beam's last position (x, y 2.048 mm wide, all of z)
    n, M = 2048, case.M
    xe = case.x_start + case.speed * case.axes[3].hi
    spans = [(xe - 1.024, xe + 1.024), (case.y0 - 1.024, case.y0 + 1.024), (0.0, case.axes[2].hi)]
    Phis = []
    for d, (lo, hi) in enumerate(spans):
        pts = torch.tensor(lo + (hi - lo) * (np.arange(n) + 0.5) / n, device="cuda")
        N = torch.empty((n, 2 * case.axes[d].s + 2), dtype=torch.float64, device="cuda")
        first = torch.empty(n, dtype=torch.int32, device="cuda")
        capi.taps_shape1d(h, dev.axes[d].basis, pts, N, None, first)
        P = torch.empty((n, M), dtype=torch.float64, device="cuda")
        capi.taps_interp1d(h, N, first, case.axes[d].n, U[d], P)
        Phis.append(P)
    w = U[3][-1].contiguous()
    rec = {}
    for prec, pn, peak in ((capi.BF16, "bf16", BF16_PEAK_TFLOPS), (capi.FP32, "fp32", 157.3),
                           (capi.FP64, "fp64", FP64_PEAK_TFLOPS)):
        out = torch.empty((n, 4), dtype=torch.float64, device="cuda")
        capi.taps_reconstruct(h, Phis, M, out, prec=prec, mode=capi.REDUCE, mode_w=w, thr=100.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        capi.taps_reconstruct(h, Phis, M, out, prec=prec, mode=capi.REDUCE, mode_w=w, thr=100.0)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3
        rec[pn] = {"ms": ms, "points": n ** 3, "tflops_at_M": 2.0 * M * n ** 3 / (ms * 1e-3) / 1e12,
                   "frac_of_peak": 2.0 * M * n ** 3 / (ms * 1e-3) / 1e12 / peak,
                   "hottest_plane_max": float(out[:, 0].max().item())}
    h.close()
    log(f"large slab: {sweeps} sweeps in {el * 1e3:.1f} ms, rho {hist}; 2048^3 reductions "
        f"{[(k, round(v['ms'], 2)) for k, v in rec.items()]} ms")
    return {"workload": "heat slab x, y 15000 nodes over 15 mm, z 15 nodes over 0.2 mm, t 513 nodes over 1 ms, "
                        "M=60, fast diagonalisation, random start",
            "setup_s": setup, "sweeps": sweeps, "ms_per_sweep": el / sweeps * 1e3, "rho_by_sweep": hist,
            "profiled_ms_per_sweep": {k: v[1] / sweeps for k, v in fam.items()},
            "subvolume_2048_cubed_reduce": rec}


def recon_large(h, capi, torch, n=2048, M=60, planes=256):
    """BF16 and FP32 REDUCE reconstruction of 2048 x 2048 planes with M = 60
    (the large-slab subvolume's plane shape), timed by the library's kernel
    events, and BF16 STORE; flops counted at M."""
    g = torch.Generator(device="cuda").manual_seed(0)
    P = [torch.randn((m, M), dtype=torch.float64, device="cuda", generator=g) for m in (n, n, planes)]
    res = {}
    for prec, pn in ((capi.BF16, "bf16"), (capi.FP32, "fp32")):
        for mode, mn in ((capi.REDUCE, "reduce"), (capi.STORE, "store")):
            shape, dt = ((planes, 4), torch.float64) if mode == capi.REDUCE else ((planes, n, n), torch.float32)
            out = torch.empty(shape, dtype=dt, device="cuda")
            capi.taps_reconstruct(h, P, M, out, prec=prec, mode=mode, thr=0.5)
            torch.cuda.synchronize()
            capi.taps_profile_enable(h, True)
            for _ in range(3):
                capi.taps_reconstruct(h, P, M, out, prec=prec, mode=mode, thr=0.5)
            torch.cuda.synchronize()
            capi.taps_profile_enable(h, False)
            k, ms, fl, by = capi.taps_profile_read(h, capi.PROF_RECON)
            t = ms / k * 1e-3
            peak = BF16_PEAK_TFLOPS if prec == capi.BF16 else 157.3
            res[f"{pn}_{mn}"] = {"ms_per_launch": ms / k, "tflops_at_M": fl / k / t / 1e12,
                                 "frac_of_peak": fl / k / t / 1e12 / peak, "written_gbs": by / k / t / 1e9}
            del out
    return res


if __name__ == "__main__":
    main()
