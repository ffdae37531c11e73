"""The allocation-free reconstruction entry point (taps_reconstruct_noalloc)
against taps_reconstruct on the same inputs: the same kernels with their
scratch in the library's static device array, so every output is
bit-identical -- every precision and mode, two calls in a row with the second
one smaller (the array keeps the first call's contents), no workspace grown
on the handle, and sizes beyond the array refused before anything runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[noalloc]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi
    return torch, capi


def _fields(torch, shape, M, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    Phis = [torch.randn((n, M), dtype=torch.float64, device="cuda", generator=g) for n in shape]
    w = torch.randn(M, dtype=torch.float64, device="cuda", generator=g)
    return Phis, w


@pytest.mark.parametrize("prec,mode", [("BF16", "REDUCE"), ("BF16", "STORE"), ("FP32", "REDUCE"),
                                       ("FP32", "STORE"), ("FP64", "REDUCE"), ("FP64", "STORE")])
def test_noalloc_equals_reconstruct(env, prec, mode):
    torch, capi = env
    p, md = getattr(capi, prec), getattr(capi, mode)
    h_ref, h = capi.Handle(), capi.Handle()
    try:
        for shape, M, seed in (((300, 260, 9), 40, 1), ((70, 33, 5), 17, 2)):   # the second call smaller
            _say(f"{prec} {mode} {shape} M={M}")
            Phis, w = _fields(torch, shape, M, seed)
            n0, n1, n2 = shape
            if md == capi.REDUCE:
                ref = torch.full((n2, 4), -7.0, dtype=torch.float64, device="cuda")
                out = torch.full((n2, 4), 5.0, dtype=torch.float64, device="cuda")
            else:
                dt = torch.float64 if p == capi.FP64 else torch.float32
                ref = torch.full((n2, n0, n1), -7.0, dtype=dt, device="cuda")
                out = torch.full((n2, n0, n1), 5.0, dtype=dt, device="cuda")
            capi.taps_reconstruct(h_ref, Phis, M, ref, prec=p, mode=md, mode_w=w, thr=0.25)
            capi.taps_reconstruct_noalloc(h, Phis, M, out, prec=p, mode=md, mode_w=w, thr=0.25)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (prec, mode, shape)
            assert capi.lib().taps_workspace_bytes(h.h) == 0
    finally:
        h_ref.close()
        h.close()


def test_noalloc_refuses_sizes_beyond_its_scratch(env):
    torch, capi = env
    h = capi.Handle()
    try:
        Phis, _ = _fields(torch, (40000, 8, 2), 64, 3)     # 40000 x 64 staged floats alone exceed 8 MiB
        out = torch.full((2, 4), 5.0, dtype=torch.float64, device="cuda")
        with pytest.raises(capi.TapsError, match="scratch"):
            capi.taps_reconstruct_noalloc(h, Phis, 64, out, prec=capi.BF16, mode=capi.REDUCE)
        torch.cuda.synchronize()
        assert torch.all(out == 5.0)
        assert capi.lib().taps_workspace_bytes(h.h) == 0
    finally:
        h.close()
