#!/usr/bin/env python
"""Benchmark: TAPS slab solves/s on one MI355X.

A step is one batch of slab solves: Algorithm 1 (subspace iteration) from the
seeded initial factors until the projected residual reaches --tol or --sweeps
sweeps have run, every kernel of the path (contractions, block-banded dim
solves, balancing, residual) on the GPU through the C ABI.  Inputs are
resident in HBM before timing starts.  The default workload is a batch of
--batch independent space-time heat slabs on one grid, 512 x 512 x 128 nodes
x 257 time nodes, M = 40 modes, moving Gaussian source with per-slab power,
radius, conductivity and track offset; --batch 1 runs the plain
one-slab-at-a-time form.  The plain form is also timed on one slab and
reported beside the batched value.

The JSON line carries the roofline of the dominant kernel (the block-banded
dim solve, FP64 ALU-bound: algorithmic flops / event-timed kernel time over
the timed region) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_case(args):
    import taps_workloads as W
    if args.workload == "heat_slab":
        return W.heat_slab(args.nx, args.nx, args.nz, args.nt, M=args.M, seed=args.seed)
    if args.workload == "poisson2d":
        return W.poisson2d(64, M=min(args.M, 10), seed=args.seed)
    raise SystemExit(f"unknown workload {args.workload}")


def cpu_baseline(case, sweeps_per_solve, n_sweeps):
    """The oracle, as it stands, on a bounded sample: n_sweeps sweeps of the
    same slab (setup excluded), scaled to slab solves/s."""
    import numpy as np
    import taps_workloads as W
    from oracle import als, problems, separated
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = 1
    prob = problems.heat_slab(case) if case.kind == "heat_slab" else problems.poisson2d(case)
    U = W.initial_factors(case.axes, case.M, case.seed)
    t0 = time.perf_counter()
    for it in range(n_sweeps):
        als.sweep(prob, U)
        als.balance(U)
        rho = separated.residual_norm(prob, U)
        log(f"cpu oracle sweep {it + 1}/{n_sweeps} rho={rho:.3e}")
    dt = time.perf_counter() - t0
    per_sweep = dt / n_sweeps
    return {
        "value": 1.0 / (per_sweep * sweeps_per_solve),
        "unit": "slab solves/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"{n_sweeps} sweep(s) of the same slab ({dt:.1f} s, {per_sweep:.2f} s/sweep), "
                  f"scaled to {sweeps_per_solve} sweeps per solve",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat_slab")
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--nt", type=int, default=257)
    ap.add_argument("--M", type=int, default=40)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=10, help="sweep budget per slab solve")
    ap.add_argument("--batch", type=int, default=256, help="slabs solved together, one workgroup each (1 = plain form)")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain form beside the batch")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-sweeps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by problem, "
              "see the multi-GPU paragraph of the design notes", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_13933_amd import capi, problem
    import taps_workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    case = make_case(args)
    h = capi.Handle()
    t0 = time.perf_counter()
    if case.kind == "heat_slab" and args.batch > 1:
        cases = W.heat_slab_family(args.batch, seed=args.seed, nx=args.nx, ny=args.nx, nz=args.nz,
                                   nt=args.nt, M=args.M)
    else:
        cases = [case]
    dps = [problem.build(h, c) for c in cases]
    U0 = [dp.factors(W.initial_factors(c.axes, c.M, c.seed)) for dp, c in zip(dps, cases)]
    U = [[u.clone() for u in us] for us in U0]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    B = len(cases)
    log(f"setup {setup_s:.2f}s: {B} x {case.kind} n={[a.n for a in case.axes]} M={case.M}")

    def reset(i=None):
        for k in (range(B) if i is None else [i]):
            for u, u0 in zip(U[k], U0[k]):
                u.copy_(u0)

    def solve_batch():
        reset()
        if B == 1:
            sw, rho, _ = capi.taps_als(h, dps[0].struct, U[0], args.tol, args.sweeps)
            return [sw], [rho]
        return capi.taps_als_batched(h, [dp.struct for dp in dps], U, args.tol, args.sweeps)

    for w in range(args.warmup):
        sw, rho = solve_batch()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup}: sweeps {min(sw)}..{max(sw)}, rho {min(rho):.3e}..{max(rho):.3e}")

    capi.taps_profile_enable(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps_total, rhos = 0, []
    for k in range(args.steps):
        sw, rhos = solve_batch()
        sweeps_total += sum(sw)
        log(f"step {k + 1}/{args.steps}: sweeps {min(sw)}..{max(sw)}, rho {min(rhos):.3e}..{max(rhos):.3e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    capi.taps_profile_enable(h, False)
    n_solve, ms_solve, fl_solve, _ = capi.taps_profile_read(h, capi.PROF_SOLVE)
    n_con, ms_con, fl_con, by_con = capi.taps_profile_read(h, capi.PROF_CONTRACT)

    plain = None
    if B > 1 and not args.no_plain:
        reset(0)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        sw, rho, _ = capi.taps_als(h, dps[0].struct, U[0], args.tol, args.sweeps)
        torch.cuda.synchronize()
        plain = {"value": 1.0 / (time.perf_counter() - tp), "sweeps": sw, "rho": rho}
        log(f"plain form: one slab {1.0 / plain['value']:.3f} s, {sw} sweeps")

    value = B * args.steps / elapsed
    achieved = (fl_solve / n_solve) / (ms_solve / n_solve * 1e-3) / 1e12 if n_solve else 0.0
    sweeps_per_solve = sweeps_total / (B * args.steps)
    rho = float(np.nanmax(rhos)) if rhos else float("nan")
    out = {
        "metric": "TAPS slab solves/s at rel. residual 1e-8; warm-start+batched vs plain",
        "value": value,
        "unit": "slab solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{B} x {case.kind} {'x'.join(str(a.n) for a in case.axes)} M={case.M} "
                         f"random init, sweep budget {args.sweeps}, tol {args.tol:g}"),
            "variant": "batched" if B > 1 else "plain",
            "batch": B,
            "sweeps_per_solve": sweeps_per_solve,
            "rho_final_max": rho,
            "tol_reached": bool(rho <= args.tol),
            "setup_s": setup_s,
            "solve_kernel_ms_per_step": ms_solve / args.steps,
            "contract_kernel_ms_per_step": ms_con / args.steps,
            "plain": plain,
            "batched_over_plain": (value / plain["value"]) if plain else None,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_block_lu_mfma(_batched) (block-banded FP64 dim solve)",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": None,
            "launches": n_solve,
            "avg_launch_ms": ms_solve / max(1, n_solve),
            "flops_per_launch": fl_solve / max(1, n_solve),
        },
    }
    if not args.no_cpu_baseline and case.kind in ("heat_slab", "poisson2d"):
        log("cpu baseline: oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cases[0], sweeps_per_solve, args.cpu_sweeps)
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
