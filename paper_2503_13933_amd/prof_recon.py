"""Timing of the reduced-precision reconstruction kernels on 2048 x 2048
planes (the large-slab subvolume shape): REDUCE over --planes-reduce planes
and STORE over --planes-store planes, BF16 and FP32, factors N(0,1) with
--M modes.  Kernel time from the library's HIP-event profiling
(TAPS_PROF_RECON), reported as achieved TFLOP/s and written GB/s:

    python3 paper_2503_13933_amd/prof_recon.py
"""
import argparse
import os
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--M", type=int, default=60)
    ap.add_argument("--planes-reduce", type=int, default=2048)
    ap.add_argument("--planes-store", type=int, default=256)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    from paper_2503_13933_amd import capi
    h = capi.Handle()
    n, M = args.n, args.M
    for prec, pn in ((capi.BF16, "bf16"), (capi.FP32, "fp32")):
        for mode, mn, n2 in ((capi.REDUCE, "reduce", args.planes_reduce), (capi.STORE, "store", args.planes_store)):
            g = torch.Generator(device="cuda").manual_seed(0)
            P = [torch.randn((m, M), dtype=torch.float64, device="cuda", generator=g) for m in (n, n, n2)]
            shape, dt = ((n2, 4), torch.float64) if mode == capi.REDUCE else ((n2, n, n), torch.float32)
            out = torch.empty(shape, dtype=dt, device="cuda")
            capi.taps_reconstruct(h, P, M, out, prec=prec, mode=mode, thr=0.5)
            torch.cuda.synchronize()
            capi.taps_profile_enable(h, True)
            for _ in range(args.reps):
                capi.taps_reconstruct(h, P, M, out, prec=prec, mode=mode, thr=0.5)
            torch.cuda.synchronize()
            capi.taps_profile_enable(h, False)
            k, ms, fl, by = capi.taps_profile_read(h, capi.PROF_RECON)
            t = ms / k * 1e-3
            print(f"{pn} {mn} {n}x{n}x{n2} M={M}: {ms / k:.3f} ms/launch, {fl / k / t / 1e12:.1f} TFLOP/s, "
                  f"{by / k / t / 1e9:.0f} GB/s", flush=True)
            del out
    h.close()


if __name__ == "__main__":
    main()
