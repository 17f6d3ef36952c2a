"""bench.py's host side (no GPU): the one-GPU contract, the CPU refusal, and
the helpers that label the JSON line."""

import os
import subprocess
import sys

import pytest

from tests.conftest import ROOT


def run_bench(*args):
    env = dict(os.environ, HIP_VISIBLE_DEVICES="")
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=env, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    p = run_bench("--gpus", "2")
    assert p.returncode == 2 and "exactly one GPU" in p.stderr


def test_no_gpu_is_refused_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    for extra in ((), ("--sweep-variants", "--workload", "plates-128"), ("--workload", "ellipsoids-64x16")):
        p = run_bench("--steps", "1", *extra)
        assert p.returncode == 1 and "needs a GPU" in p.stderr, (extra, p.stderr[-500:])


def test_labels():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1911_00093_amd import hmat

    assert "fp32 dense" in bench.storage_label(hmat.M2_MIXED)
    assert "bf16" in bench.storage_label(hmat.BF16_SCALED).lower()
    assert "fp64" in bench.storage_label(hmat.M1_DOUBLE).lower()
    assert len(bench.sources_hash()) == 16


def test_default_early_checks():
    """Early FP64 checks by default: BF16 always (1e-2), M2-Mixed only where
    restarts were measured to pay (plates-128 and the batch, 1e-4)."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1911_00093_amd import hmat

    assert bench.default_refine(hmat.M2_MIXED, "sphere-L7+8") == 0.0
    assert bench.default_refine(hmat.M2_MIXED, "plates-128") == 1e-4
    assert bench.default_refine(hmat.M2_MIXED, "ellipsoids-64x16") == 1e-4
    for w in ("sphere-L7+8", "plates-128"):
        assert bench.default_refine(hmat.BF16_SCALED, w) == 1e-2
