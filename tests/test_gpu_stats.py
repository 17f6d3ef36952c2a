"""hmat_get_stats' introspection: stored bytes per storage class and block
counts per size class, against the block description and the conversion's
choices (Method 3's split puts some low-rank terms in each class)."""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import blockset, need_gpu

pytestmark = pytest.mark.gpu


def size_class(side):
    k = 0
    while k < 7 and side > (16 << k):
        k += 1
    return k


@pytest.mark.parametrize("variant,c", [(oracle.M1_DOUBLE, -1), (oracle.M2_MIXED, -1), (oracle.M3, 1),
                                       (oracle.BF16_SCALED, -1)])
def test_stats_by_class_and_size(variant, c):
    need_gpu()
    _, h = oracle_hmatrix("spheres-mixed")
    st = hmat.HMatrix(blockset(h), variant, c=c).stats()
    cls = list(st.bytes_class)
    assert sum(cls) == st.bytes_dense + st.bytes_v + st.bytes_w
    side = np.maximum(h.nrows, h.ncols)
    for kind, got in ((0, st.blocks_dense_by_size), (1, st.blocks_lowrank_by_size)):
        want = np.bincount([size_class(s) for s in side[h.kind == kind]], minlength=8)
        assert list(got) == want.tolist(), kind
    assert sum(st.blocks_dense_by_size) == st.nblocks_dense and sum(st.blocks_lowrank_by_size) == st.nblocks_lowrank
    if variant == oracle.M1_DOUBLE:
        assert cls[1] == cls[2] == 0
    elif variant == oracle.M2_MIXED:
        assert cls[0] == cls[2] == 0
    elif variant == oracle.BF16_SCALED:
        assert cls[0] == 0 and cls[2] == st.bytes_v + st.bytes_w and cls[1] == st.bytes_dense
    else:
        assert cls[0] > 0 and cls[1] > 0 and cls[2] == 0
