"""Profiling driver for the dim solve: one batched sweep of Algorithm 1 over
--slabs heat slabs (512 x 512 x 128 x 257, M = 40 by default) with the fast
diagonalisation (--solver fastdiag, the default) or the block LU, followed by
a plain device copy of --copy-mib MiB (torch's copy kernel) whose known size
calibrates the memory counters.  Prints the launches, event-timed kernel time
and algorithmic flops and bytes of the solve, eigen, real Schur and
contraction kernel families over the sweep.  Meant to run under rocprofv3:

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- \\
        python3 paper_2503_13933_amd/prof_solve.py
"""
import argparse
import os
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--slabs", type=int, default=1024)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--nt", type=int, default=257)
    ap.add_argument("--M", type=int, default=40)
    ap.add_argument("--sweeps", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--solver", choices=["fastdiag", "blocklu"], default="fastdiag")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import taps_workloads as W
    from paper_2503_13933_amd import capi, chain
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG if args.solver == "fastdiag" else capi.SOLVER_BLOCK_LU)
    cases = W.heat_slab_family(args.slabs, seed=2, nx=args.nx, ny=args.nx, nz=args.nz, nt=args.nt, M=args.M)
    probs = [chain.slab_problem(h, c) for c in cases]
    U = [p.factors(W.initial_factors(c.axes, args.M, c.seed)) for p, c in zip(probs, cases)]
    torch.cuda.synchronize()
    print(f"batched sweep ({args.solver}): {args.slabs} slabs {[a.n for a in cases[0].axes]} M={args.M}", flush=True)
    capi.taps_profile_enable(h, True)
    sw, rho = capi.taps_als_batched(h, [p.struct for p in probs], U, 0.0, args.sweeps)
    torch.cuda.synchronize()
    capi.taps_profile_enable(h, False)
    for name, fam in (("solve", capi.PROF_SOLVE), ("eig", capi.PROF_EIG), ("schur", capi.PROF_SCHUR),
                      ("contract", capi.PROF_CONTRACT)):
        n_l, ms, fl, by = capi.taps_profile_read(h, fam)
        print(f"family {name}: launches {n_l} kernel ms {ms:.3f} algorithmic flops {fl:.6e} bytes {by:.6e}",
              flush=True)
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    print(f"copy: {args.copy_mib} MiB", flush=True)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"done: rho {min(rho):.3e}..{max(rho):.3e}", flush=True)
    h.close()


if __name__ == "__main__":
    main()
