"""ctypes binding of libtaps.so (the C ABI declared in include/taps.h).

Argument marshalling only: every computation runs in the HIP library.  Torch
tensors provide device memory and the current stream.  Functions keep the C
names; they raise TapsError on a non-OK status with the library's message.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtaps.so")

MAX_DIMS, MAX_TERMS, MAX_KINDS, MAX_M, MAX_S, MAX_GAUSS = 8, 32, 8, 64, 3, 8

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_ALLOC, ERR_HIP = 0, -1, -2, -3, -4
MASS, STIFF, DDT, WMASS, BMASS, WSTIFF, WDDT = 0, 1, 2, 3, 4, 5, 6
SRC_GAUSS, SRC_TOPLAYER, SRC_POLY, SRC_SIN, SRC_NODAL, SRC_EXPQUAD = 0, 1, 2, 3, 4, 5
FP64, FP32, BF16 = 0, 1, 2
STORE, REDUCE = 0, 1

FUNCTIONS = (
    "taps_create", "taps_destroy", "taps_last_error", "taps_reserve", "taps_workspace_bytes",
    "taps_gauss_points", "taps_shape1d", "taps_source1d", "taps_assemble1d", "taps_contract",
    "taps_solve_dim", "taps_residual", "taps_balance", "taps_sweep", "taps_als", "taps_interp1d",
    "taps_reconstruct", "taps_reconstruct_batched", "taps_profile_enable", "taps_profile_read", "taps_als_batched", "taps_band_apply",
    "taps_canonicalize", "taps_mlp_cache_bytes", "taps_mlp_forward", "taps_mlp_backward", "taps_mlp_mse",
    "taps_adam_step", "taps_set_tuning", "taps_get_tuning", "taps_autotune", "taps_reconstruct_noalloc",
    "taps_td_inner", "taps_load1d",
)
MLP_MAX_LAYERS = 8
PROF_SOLVE, PROF_CONTRACT, PROF_RECON, PROF_EIG, PROF_SCHUR = 0, 1, 2, 3, 4


class TapsError(RuntimeError):
    pass


class Basis1D(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("d_x", C.c_void_p), ("s", C.c_int32), ("a", C.c_double),
                ("p", C.c_int32), ("n_gauss", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [
        ("D", C.c_int32), ("M", C.c_int32), ("T", C.c_int32), ("R", C.c_int32),
        ("n", C.c_int32 * MAX_DIMS), ("s", C.c_int32 * MAX_DIMS), ("n_kinds", C.c_int32 * MAX_DIMS),
        ("term_kind", (C.c_int32 * MAX_DIMS) * MAX_TERMS), ("gamma", C.c_double * MAX_TERMS),
        ("d_band", C.c_void_p * MAX_DIMS), ("R_cols", C.c_int32 * MAX_DIMS),
        ("d_F", C.c_void_p * MAX_DIMS), ("d_load_col", C.c_void_p * MAX_DIMS),
        ("d_load_ptr", C.c_void_p * MAX_DIMS), ("d_load_idx", C.c_void_p * MAX_DIMS),
        ("d_fixed", C.c_void_p * MAX_DIMS),
    ]


class Tuning(C.Structure):
    _fields_ = [("graph_sweeps", C.c_int32), ("solver", C.c_int32), ("lgram_rows", C.c_int32)]


class MLP(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("width", C.c_int32 * (MLP_MAX_LAYERS + 1)),
                ("d_W", C.c_void_p * MLP_MAX_LAYERS), ("d_b", C.c_void_p * MLP_MAX_LAYERS)]


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TapsError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, dbl, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_double, C.c_size_t
        P = C.POINTER
        sig = {
            "taps_create": (i32, [P(vp)]),
            "taps_destroy": (i32, [vp]),
            "taps_last_error": (C.c_char_p, [vp]),
            "taps_reserve": (i32, [vp, sz]),
            "taps_workspace_bytes": (sz, [vp]),
            "taps_gauss_points": (i32, [vp, P(Basis1D), vp, vp, vp]),
            "taps_shape1d": (i32, [vp, P(Basis1D), i32, vp, vp, vp, vp, vp]),
            "taps_source1d": (i32, [vp, i32, i32, vp, i32, i32, P(dbl), vp, P(Basis1D), vp, vp]),
            "taps_assemble1d": (i32, [vp, P(Basis1D), i32, P(i32), vp, P(i32), vp, i32, vp, vp, vp]),
            "taps_contract": (i32, [vp, P(Problem), i32, u32, P(vp), vp, vp, vp]),
            "taps_solve_dim": (i32, [vp, P(Problem), i32, vp, vp, vp, vp, vp, vp]),
            "taps_residual": (i32, [vp, P(Problem), P(vp), vp, vp]),
            "taps_balance": (i32, [vp, P(Problem), P(vp), vp]),
            "taps_sweep": (i32, [vp, P(Problem), P(vp), vp, vp, vp]),
            "taps_als": (i32, [vp, P(Problem), P(vp), dbl, dbl, i32, P(i32), P(dbl), P(dbl), P(dbl), P(dbl), vp]),
            "taps_interp1d": (i32, [vp, i32, i32, vp, vp, i32, i32, vp, vp, vp]),
            "taps_reconstruct": (i32, [vp, P(i32), P(vp), i32, vp, i32, i32, vp, dbl, vp]),
            "taps_reconstruct_batched": (i32, [vp, i32, P(i32), P(vp), i32, P(vp), i32, i32, P(vp), dbl, vp]),
            "taps_profile_enable": (i32, [vp, i32]),
            "taps_als_batched": (i32, [vp, i32, P(Problem), P(vp), dbl, dbl, i32, P(i32), P(dbl), P(dbl), vp]),
            "taps_profile_read": (i32, [vp, i32, P(i32), P(dbl), P(dbl), P(dbl)]),
            "taps_band_apply": (i32, [vp, i32, i32, vp, i32, vp, i32, vp, dbl, vp, i32, vp]),
            "taps_canonicalize": (i32, [vp, i32, P(i32), i32, P(vp), P(vp), vp]),
            "taps_mlp_cache_bytes": (sz, [P(MLP), i32]),
            "taps_mlp_forward": (i32, [vp, P(MLP), i32, vp, vp, vp, vp]),
            "taps_mlp_backward": (i32, [vp, P(MLP), i32, vp, vp, P(vp), P(vp), vp]),
            "taps_mlp_mse": (i32, [vp, C.c_int64, vp, vp, vp, vp, vp]),
            "taps_adam_step": (i32, [vp, C.c_int64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, i32, vp, vp]),
            "taps_set_tuning": (i32, [vp, P(Tuning)]),
            "taps_get_tuning": (i32, [vp, P(Tuning)]),
            "taps_autotune": (i32, [vp, i32, P(Problem), P(vp), C.c_char_p, P(Tuning), P(dbl), vp]),
            "taps_reconstruct_noalloc": (i32, [vp, P(i32), P(vp), i32, vp, i32, i32, vp, dbl, vp]),
            "taps_td_inner": (i32, [vp, i32, P(i32), P(i32), P(vp), i32, P(vp), i32, P(vp), vp, vp]),
            "taps_load1d": (i32, [vp, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp]),
        }
        missing = set(FUNCTIONS) - set(sig)
        if missing:
            raise TapsError(f"no ctypes signature for {sorted(missing)}")
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers


def _ptr(t):
    """Device (or host) address of a tensor (or a raw address given as an
    int), None for None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise TapsError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


class Handle:
    """Owning wrapper of a taps_handle_t."""

    def __init__(self):
        h = C.c_void_p()
        st = lib().taps_create(C.byref(h))
        if st != OK:
            raise TapsError(f"taps_create failed ({st})")
        self.h = h

    def close(self):
        self.__dict__.pop("_grids", None)      # device data cached per grid (problem.py)
        if self.h:
            lib().taps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st, what):
        if st != OK:
            msg = lib().taps_last_error(self.h).decode()
            raise TapsError(f"{what} -> {st}: {msg}")


def _ptr_array(tensors):
    """C array of addresses from a list of tensors / ints / None, or from an
    integer numpy array of addresses (copied in one step)."""
    if isinstance(tensors, np.ndarray):
        a = np.ascontiguousarray(tensors, dtype=np.uint64).ravel()
        return (C.c_void_p * len(a)).from_buffer_copy(a.tobytes())
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = _ptr(t)
    return arr


# ---------------------------------------------------------------- C names


def taps_gauss_points(h: Handle, basis: Basis1D, xg, wg, stream=None):
    h.check(lib().taps_gauss_points(h.h, C.byref(basis), _ptr(xg), _ptr(wg), _stream(stream)), "taps_gauss_points")


def taps_shape1d(h: Handle, basis: Basis1D, pts, N, dN, first, stream=None):
    h.check(lib().taps_shape1d(h.h, C.byref(basis), pts.numel(), _ptr(pts), _ptr(N), _ptr(dN), _ptr(first),
                               _stream(stream)), "taps_shape1d")


def taps_source1d(h: Handle, kind: int, pts, n_cols: int, params, out, centers=None, basis=None, stream=None):
    prm = (C.c_double * max(1, len(params)))(*params)
    bref = C.byref(basis) if basis is not None else None
    h.check(lib().taps_source1d(h.h, kind, pts.numel(), _ptr(pts), n_cols, len(params), prm, _ptr(centers), bref,
                                _ptr(out), _stream(stream)), "taps_source1d")


def taps_assemble1d(h: Handle, basis: Basis1D, kinds, band, coef_g=None, bnode=None, f_g=None, F=None,
                    n_loads: int = 0, stream=None):
    k = (C.c_int32 * max(1, len(kinds)))(*kinds)
    bn = (C.c_int32 * max(1, len(kinds)))(*(bnode or [-1] * len(kinds)))
    h.check(lib().taps_assemble1d(h.h, C.byref(basis), len(kinds), k, _ptr(coef_g), bn, _ptr(band), n_loads,
                                  _ptr(f_g), _ptr(F), _stream(stream)), "taps_assemble1d")


def taps_load1d(h: Handle, n_nodes: int, s: int, n_gauss: int, Ng, first, wg, f_g, F, stream=None):
    """Loads of f_g ((R, n_gpts) at the Gauss points) from shape values at
    the Gauss points (Ng, first from taps_shape1d; wg the Gauss weights)."""
    h.check(lib().taps_load1d(h.h, n_nodes, s, n_gauss, _ptr(Ng), _ptr(first), _ptr(wg), int(f_g.shape[0]),
                              _ptr(f_g), _ptr(F), _stream(stream)), "taps_load1d")


def taps_contract(h: Handle, prob: Problem, d: int, stale_mask: int, U, Cout, Q, stream=None):
    h.check(lib().taps_contract(h.h, C.byref(prob), d, stale_mask & 0xFFFFFFFF, _ptr_array(U), _ptr(Cout), _ptr(Q),
                                _stream(stream)), "taps_contract")


def taps_solve_dim(h: Handle, prob: Problem, d: int, Cin, Q, X, info, berr=None, stream=None):
    h.check(lib().taps_solve_dim(h.h, C.byref(prob), d, _ptr(Cin), _ptr(Q), _ptr(X), _ptr(info), _ptr(berr),
                                 _stream(stream)), "taps_solve_dim")


def taps_residual(h: Handle, prob: Problem, U, out, stream=None):
    h.check(lib().taps_residual(h.h, C.byref(prob), _ptr_array(U), _ptr(out), _stream(stream)), "taps_residual")


def taps_balance(h: Handle, prob: Problem, U, stream=None):
    h.check(lib().taps_balance(h.h, C.byref(prob), _ptr_array(U), _stream(stream)), "taps_balance")


def taps_sweep(h: Handle, prob: Problem, U, info=None, berr=None, stream=None):
    h.check(lib().taps_sweep(h.h, C.byref(prob), _ptr_array(U), _ptr(info), _ptr(berr), _stream(stream)),
            "taps_sweep")


def taps_als(h: Handle, prob: Problem, U, tol: float, iter_max: int, change_tol: float = 0.0, stream=None,
             change_hist=None):
    """Returns (sweeps, rho, history list); rho is NaN after a breakdown
    (the reason is in last_error(h)).  change_hist, a list, receives the
    relative change of the factors after every sweep."""
    sweeps = C.c_int32()
    rho = C.c_double()
    hist = (C.c_double * iter_max)()
    chist = (C.c_double * iter_max)() if change_hist is not None else None   # measured only when asked for
    h.check(lib().taps_als(h.h, C.byref(prob), _ptr_array(U), tol, change_tol, iter_max, C.byref(sweeps),
                           C.byref(rho), None, hist, chist, _stream(stream)), "taps_als")
    if change_hist is not None:
        change_hist.extend(chist[: sweeps.value])
    return sweeps.value, rho.value, list(hist[: sweeps.value])


SOLVER_BLOCK_LU, SOLVER_FAST_DIAG = 0, 1


def taps_get_tuning(h: Handle) -> Tuning:
    t = Tuning()
    h.check(lib().taps_get_tuning(h.h, C.byref(t)), "taps_get_tuning")
    return t


def taps_set_tuning(h: Handle, graph_sweeps: int = None, solver: int = None, lgram_rows: int = None):
    """Fields left as None keep the handle's current value."""
    t = taps_get_tuning(h)
    if graph_sweeps is not None:
        t.graph_sweeps = graph_sweeps
    if solver is not None:
        t.solver = solver
    if lgram_rows is not None:
        t.lgram_rows = lgram_rows
    h.check(lib().taps_set_tuning(h.h, C.byref(t)), "taps_set_tuning")


def taps_autotune(h: Handle, probs, Us, cache_path=None, stream=None):
    """Returns (chosen Tuning, ms per sweep of the 8 candidates: row splits
    128, 256, 512, 1024 with host launches, then graph lengths 0, 1, 2, 4)."""
    B = len(probs)
    arr = probs if isinstance(probs, C.Array) else (Problem * B)(*probs)
    ptrs = Us if isinstance(Us, C.Array) else _ptr_array([u for U in Us for u in U])
    t = Tuning()
    ms = (C.c_double * 8)()
    path = cache_path.encode() if cache_path else None
    h.check(lib().taps_autotune(h.h, B, arr, ptrs, path, C.byref(t), ms, _stream(stream)), "taps_autotune")
    return t, list(ms)


def taps_band_apply(h: Handle, s: int, band, X, Y, alpha: float = 1.0, scale=None, stream=None):
    """Y = alpha * (A X) * scale (per column), A = band (n x (4s+3)).  X and Y
    may be column slices of wider row-major tensors (their row strides are
    passed as leading dimensions)."""
    n, ncols = X.shape
    if X.stride(1) != 1 or Y.stride(1) != 1 or not band.is_contiguous():
        raise TapsError("rows must be contiguous")
    if Y.shape != X.shape:
        raise TapsError("X and Y shapes differ")
    h.check(lib().taps_band_apply(h.h, n, s, band.data_ptr(), ncols, X.data_ptr(), X.stride(0), _ptr(scale),
                                  alpha, Y.data_ptr(), Y.stride(0), _stream(stream)), "taps_band_apply")


def taps_canonicalize(h: Handle, Us, outs, stream=None):
    n = (C.c_int32 * len(Us))(*[int(u.shape[0]) for u in Us])
    h.check(lib().taps_canonicalize(h.h, len(Us), n, int(Us[0].shape[1]), _ptr_array(Us), _ptr_array(outs),
                                    _stream(stream)), "taps_canonicalize")


def mlp_struct(widths, Ws, bs):
    """taps_mlp_t over device tensors (Ws: uint16/bfloat16 width[l+1] x ldw, bs: float32)."""
    m = MLP()
    m.n_layers = len(widths) - 1
    for l, w in enumerate(widths):
        m.width[l] = int(w)
    for l, (W, b) in enumerate(zip(Ws, bs)):
        m.d_W[l] = _ptr(W)
        m.d_b[l] = _ptr(b)
    return m


def taps_mlp_cache_bytes(net: MLP, B: int) -> int:
    return int(lib().taps_mlp_cache_bytes(C.byref(net), B))


def taps_mlp_forward(h: Handle, net: MLP, X, cache, Y, stream=None):
    h.check(lib().taps_mlp_forward(h.h, C.byref(net), int(X.shape[0]), _ptr(X), _ptr(cache), _ptr(Y),
                                   _stream(stream)), "taps_mlp_forward")


def taps_mlp_backward(h: Handle, net: MLP, B: int, cache, dY, gWs, gbs, stream=None):
    h.check(lib().taps_mlp_backward(h.h, C.byref(net), B, _ptr(cache), _ptr(dY), _ptr_array(gWs), _ptr_array(gbs),
                                    _stream(stream)), "taps_mlp_backward")


def taps_mlp_mse(h: Handle, Y, T, dY, loss, stream=None):
    h.check(lib().taps_mlp_mse(h.h, int(Y.numel()), _ptr(Y), _ptr(T), _ptr(dY), _ptr(loss), _stream(stream)),
            "taps_mlp_mse")


def taps_adam_step(h: Handle, p, g, m, v, lr, t, p16=None, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    h.check(lib().taps_adam_step(h.h, int(p.numel()), _ptr(p), _ptr(g), _ptr(m), _ptr(v), lr, b1, b2, eps, t,
                                 _ptr(p16), _stream(stream)), "taps_adam_step")


def taps_interp1d(h: Handle, N, first, n_nodes: int, U, Phi, stream=None):
    npts, L = N.shape
    h.check(lib().taps_interp1d(h.h, npts, L, _ptr(N), _ptr(first), n_nodes, U.shape[1], _ptr(U), _ptr(Phi),
                                _stream(stream)), "taps_interp1d")


def taps_reconstruct(h: Handle, Phis, M: int, out, prec: int = FP64, mode: int = STORE, mode_w=None,
                     thr: float = 0.0, stream=None):
    n = (C.c_int32 * 3)(*[int(P.shape[0]) for P in Phis])
    h.check(lib().taps_reconstruct(h.h, n, _ptr_array(Phis), M, _ptr(mode_w), prec, mode, _ptr(out), thr,
                                   _stream(stream)), "taps_reconstruct")


def taps_td_inner(h: Handle, s, bands, A, B, out, stream=None):
    """out (Ma*Mb + 1 doubles): entrywise prod_d A_d^T S_d B_d, then the sum
    (the inner product of the two TD fields in the metric of the bands)."""
    D = len(A)
    n = (C.c_int32 * D)(*[int(a.shape[0]) for a in A])
    ss = (C.c_int32 * D)(*s)
    h.check(lib().taps_td_inner(h.h, D, n, ss, _ptr_array(bands), int(A[0].shape[1]), _ptr_array(A),
                                int(B[0].shape[1]), _ptr_array(B), _ptr(out), _stream(stream)), "taps_td_inner")


def taps_reconstruct_noalloc(h: Handle, Phis, M: int, out, prec: int = FP64, mode: int = STORE, mode_w=None,
                             thr: float = 0.0, stream=None):
    n = (C.c_int32 * 3)(*[int(P.shape[0]) for P in Phis])
    h.check(lib().taps_reconstruct_noalloc(h.h, n, _ptr_array(Phis), M, _ptr(mode_w), prec, mode, _ptr(out), thr,
                                           _stream(stream)), "taps_reconstruct_noalloc")


def taps_reconstruct_batched(h: Handle, Phis, M: int, outs, prec: int = BF16, mode: int = REDUCE, mode_ws=None,
                             thr: float = 0.0, stream=None, n_pts=None):
    """Phis: B lists of 3 factor tensors (one grid shape) or raw addresses
    (then n_pts gives the three lengths), or a (B, 3) integer array of
    addresses; outs: B outputs; mode_ws: B weight tensors or addresses
    (entries may be None) or None; outs and mode_ws may be integer arrays of
    addresses too."""
    B = len(Phis)
    n = (C.c_int32 * 3)(*(n_pts if n_pts is not None else [int(P.shape[0]) for P in Phis[0]]))
    mw = _ptr_array(mode_ws) if mode_ws is not None else None
    phis = Phis if isinstance(Phis, np.ndarray) else [P for F in Phis for P in F]
    h.check(lib().taps_reconstruct_batched(h.h, B, n, _ptr_array(phis), M, mw, prec, mode,
                                           _ptr_array(outs), thr, _stream(stream)), "taps_reconstruct_batched")


def taps_profile_enable(h: Handle, enable: bool):
    h.check(lib().taps_profile_enable(h.h, 1 if enable else 0), "taps_profile_enable")


def taps_profile_read(h: Handle, family: int):
    """(launches, total_ms, flops, bytes) of one kernel family since enable."""
    n, ms, fl, by = C.c_int32(), C.c_double(), C.c_double(), C.c_double()
    h.check(lib().taps_profile_read(h.h, family, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)),
            "taps_profile_read")
    return n.value, ms.value, fl.value, by.value


def last_error(h: Handle) -> str:
    return lib().taps_last_error(h.h).decode()


def taps_als_batched(h: Handle, probs, Us, tol: float, iter_max: int, change_tol: float = 0.0, stream=None,
                     change=None, arrays: bool = False):
    """Algorithm 1 over a batch.  probs: list of Problem; Us: list (per problem)
    of factor tensor lists, or a ctypes array of factor pointers.  Returns
    (sweeps list, rho list), or with arrays=True (sweeps, rho) as numpy
    arrays over the call's own output buffers; change, a list, receives
    every problem's relative change of the factors over its last sweep
    (measured only when change is given or change_tol > 0)."""
    B = len(probs)
    arr = probs if isinstance(probs, C.Array) else (Problem * B)(*probs)
    ptrs = Us if isinstance(Us, C.Array) else _ptr_array([u for U in Us for u in U])
    sw = (C.c_int32 * B)()
    rh = (C.c_double * B)()
    ch = (C.c_double * B)() if change is not None else None   # measured only when asked for
    h.check(lib().taps_als_batched(h.h, B, arr, ptrs, tol, change_tol, iter_max, sw, rh, ch, _stream(stream)),
            "taps_als_batched")
    if change is not None:
        change.extend(ch)
    if arrays:
        return np.frombuffer(sw, dtype=np.int32), np.frombuffer(rh, dtype=np.float64)
    return list(sw), list(rh)
