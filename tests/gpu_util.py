"""Helpers shared by the GPU tests (parity against the oracle)."""

import numpy as np

import oracle
from paper_1911_00093_amd import hmat


def need_gpu():
    import pytest
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def blockset(h) -> hmat.BlockSet:
    """The oracle's FP64 H-matrix in the ABI's block format."""
    return hmat.BlockSet.from_arrays(h.n, h.row0, h.nrows, h.col0, h.ncols, h.kind, h.rank, h.offset, h.data,
                                     h.perm)


def abs_scale(h, x):
    """|A~| |x| computed with the magnitudes of the stored FP64 factors: an
    upper bound of every partial sum's size, used to normalise errors."""
    ha = oracle.HMatrix.from_blocks(h.n, h.row0, h.nrows, h.col0, h.ncols, h.kind, h.rank, h.offset, np.abs(h.data))
    return oracle.Converted(ha, oracle.M1_DOUBLE).matvec(np.abs(x))


def tolerance(variant):
    """GPU vs oracle on the same blocks and the same rounded values.  Where z
    is FP64 only the summation order differs: 1e-13 of |A~||x|.  Where
    Table 1 keeps z in FP32 (M1-Single/Mixed), an FP64 sum that lands on the
    other side of an FP32 rounding boundary moves z by one FP32 ulp: 2^-23."""
    return 2.0 ** -23 if variant in (oracle.M1_SINGLE, oracle.M1_MIXED) else 1e-13


def to_dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()
