"""The autotuner's persistent cache (paper_1911_00093_amd.tuning): the first
handle is tuned and its configuration stored under the handle's key; a
second handle of the same blocks gets the stored configuration without
timing, and both compute the same product bit for bit."""

import json

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat, tuning
from tests.conftest import oracle_hmatrix
from tests.gpu_util import blockset, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant,nrhs_max", [(oracle.M2_MIXED, 1), (oracle.BF16_SCALED, 1), (oracle.M2_MIXED, 16)])
def test_cache_roundtrip(variant, nrhs_max, tmp_path, monkeypatch):
    need_gpu()
    import torch

    path = tmp_path / "tune.json"
    monkeypatch.setenv(tuning.ENV, str(path))
    _, h = oracle_hmatrix("plates-32")
    bs = blockset(h)
    A = hmat.HMatrix(bs, variant, nrhs_max=nrhs_max)
    first = tuning.autotune(A, reps=3)
    assert first["cached"] is False and path.exists()
    stored = json.loads(path.read_text())
    assert list(stored) == [tuning.handle_key(A)]
    B = hmat.HMatrix(bs, variant, nrhs_max=nrhs_max)
    assert tuning.handle_key(B) == tuning.handle_key(A)
    second = tuning.autotune(B, reps=3)
    assert second["cached"] is True and "ms_tuned" not in second
    for k in ("stage1_grid", "stage2_grid", "stage2_tile", "stage1_batch", "stage2_batch"):
        assert second[k] == first[k], k
    cols = 3 if nrhs_max > 1 else 1
    X = torch.as_tensor(np.random.default_rng(2).standard_normal((cols, h.n))).cuda()
    x = X.T if cols > 1 else X[0]
    assert torch.equal(A.matvec(x), B.matvec(x))
    # another precision is another key
    C = hmat.HMatrix(bs, oracle.M1_DOUBLE, nrhs_max=nrhs_max)
    assert tuning.handle_key(C) != tuning.handle_key(A)
    assert tuning.autotune(C, reps=3)["cached"] is False
    assert len(json.loads(path.read_text())) == 2


def test_unreadable_cache_is_retuned(tmp_path):
    need_gpu()
    path = tmp_path / "tune.json"
    path.write_text("not json")
    _, h = oracle_hmatrix("plates-16")
    H = hmat.HMatrix(blockset(h), oracle.M2_MIXED)
    assert tuning.autotune(H, reps=2, cache=str(path))["cached"] is False
    assert tuning.handle_key(H) in json.loads(path.read_text())
