"""Host logic of the stream driver: the factor pointers a round hands to the
batched call (problem-major, one per dim) are the slabs' addresses in the
contiguous per-dim factor tensors, for any order and repetition of slabs;
with the batched call replaced by a script of residuals, every round hands
over the active slabs' own records and pointers (from the problem list or
the records packed once), slabs leave at the tolerance, the cap or a
breakdown with the right sweep counts and outcomes under both schedules,
and the fallback rule restarts exactly the slabs whose warm start lost
(sweep-1 residual above the median, growth from sweep 1 to 2, or a
breakdown) from their plain factors."""
import ctypes as C

import numpy as np
import torch

from paper_2503_13933_amd import warmstart as ws


def test_factor_pointers_follow_the_slab_layout():
    dims = [torch.zeros(7, n, 3, dtype=torch.float64) for n in (5, 4, 6, 2)]
    fb = ws.FactorBatch(dims)
    idx = [6, 0, 3, 3, 1]
    arr = fb.ptrs(idx)
    assert isinstance(arr, C.Array) and len(arr) == len(idx) * 4
    want = [dims[d][b].data_ptr() for b in idx for d in range(4)]
    assert list(arr) == want
    # a row address inside a slab's factor
    assert fb.ptr(2, 1, row=3) == dims[1][2, 3].data_ptr()


def test_factor_pointers_of_a_full_batch_in_order():
    dims = [torch.zeros(33, n, 5, dtype=torch.float64) for n in (9, 8)]
    fb = ws.FactorBatch(dims)
    arr = np.array(list(fb.ptrs(list(range(33)))), dtype=np.uint64).reshape(33, 2)
    for d in range(2):
        assert np.all(np.diff(arr[:, d]) == dims[d].shape[1] * dims[d].shape[2] * 8)
        assert arr[0, d] == dims[d].data_ptr()


# ---- the stream driver's schedule with the batched call replaced by a script

from paper_2503_13933_amd import capi  # noqa: E402


class _Slab:
    """A problem record whose R field names the slab (and gamma[0] checks
    the whole record travelled)."""

    def __init__(self, i):
        self.struct = capi.Problem()
        self.struct.R = i
        self.struct.gamma[0] = 0.5 + i


def _script_call(monkeypatch, script, fb, seen):
    """The batched call as a script: slab i's residual after its j-th sweep
    of the run is script[i][j].  Checks that every round hands over the
    active slabs' own records and factor pointers, in the same order."""
    def fake(h, probs, Us, tol, iter_max, change_tol=0.0, stream=None, change=None, arrays=False):
        assert iter_max == 1
        idx = [probs[k].R for k in range(len(probs))]
        assert len(set(idx)) == len(idx)
        assert all(probs[k].gamma[0] == 0.5 + idx[k] for k in range(len(idx)))
        assert list(Us) == list(fb.ptrs(idx))
        r = []
        for i in idx:
            r.append(script[i][seen[i]])
            seen[i] += 1
        if arrays:
            return np.ones(len(idx), dtype=np.int32), np.asarray(r, dtype=np.float64)
        return [1] * len(idx), r
    monkeypatch.setattr(capi, "taps_als_batched", fake)


def _factors(n):
    return ws.FactorBatch([torch.ones(n, 3, 2, dtype=torch.float64) for _ in range(2)])


def test_stream_schedule_outcomes_and_records(monkeypatch):
    nan = float("nan")
    tol, cap = 0.1, 4
    # slab i needs (i % 4) + 1 sweeps; slab 5 breaks down at its second
    # sweep, slab 7 never reaches tol (stopped at the cap)
    script = [[0.5] * (i % 4) + [0.05] for i in range(11)]
    script[5] = [0.4, nan]
    script[7] = [0.6, 0.5, 0.4, 0.3]
    want_sweeps = [(i % 4) + 1 for i in range(11)]
    want_sweeps[5], want_sweeps[7] = 2, 4
    want_outcome = [0] * 11
    want_outcome[5], want_outcome[7] = 2, 1
    slabs = [_Slab(i) for i in range(11)]
    for first in (False, True):
        for probs in (slabs, ws.pack_problems(slabs)):
            fb = _factors(11)
            seen = [0] * 11
            _script_call(monkeypatch, script, fb, seen)
            left = []
            total, rho, restarts, outcome = ws.solve_stream(None, probs, fb, tol, cap, 4, first_sweep_all=first,
                                                            on_done_batch=left.extend)
            assert total == want_sweeps and outcome == want_outcome and restarts == 0
            assert seen == want_sweeps
            assert sorted(left) == list(range(11))
            for i in range(11):
                r = script[i][want_sweeps[i] - 1]
                assert (np.isnan(rho[i]) and np.isnan(r)) or rho[i] == r


def test_stream_fallback_restarts_from_the_plain_factors(monkeypatch):
    nan = float("nan")
    tol, cap, med1 = 0.1, 3, 0.5
    script = [
        [0.3, 0.05],          # 0: keeps its warm start
        [0.9, 0.3, 0.05],     # 1: sweep-1 residual above the median -> restart
        [0.2, 0.25, 0.05],    # 2: grows from sweep 1 to 2 -> restart
        [nan, 0.05],          # 3: breaks down in sweep 1 -> restart
        [0.4, 0.2, 0.15, 0.12],  # 4: keeps its warm start, stopped at the cap
    ]
    slabs = [_Slab(i) for i in range(5)]
    fb = _factors(5)
    plain = ws.FactorBatch([torch.full((5, 3, 2), 2.0, dtype=torch.float64) + torch.arange(5.0)[:, None, None]
                            for _ in range(2)])
    seen = [0] * 5
    _script_call(monkeypatch, script, fb, seen)
    total, rho, restarts, outcome = ws.solve_stream(None, slabs, fb, tol, cap, 2, U_plain=plain, median_rho1=med1)
    assert restarts == 3
    assert total == [2, 3, 3, 2, 3]
    assert outcome == [0, 0, 0, 0, 1]
    assert rho == [0.05, 0.05, 0.05, 0.05, 0.15]
    for i in range(5):
        for u, u0 in zip(fb[i], plain[i]):
            assert torch.equal(u, u0) == (i in (1, 2, 3))
