"""Host logic of the stream driver: the factor pointers a round hands to the
batched call (problem-major, one per dim) are the slabs' addresses in the
contiguous per-dim factor tensors, for any order and repetition of slabs."""
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
