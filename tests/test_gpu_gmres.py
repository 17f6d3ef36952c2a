"""GPU restarted GMRES (hmat_gmres) against the oracle's GMRES
(oracle/gmres.py) on the same blocks and operator arithmetic."""

import numpy as np
import pytest

import oracle
from oracle import gmres as OG
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import blockset, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def setup(key, variant, nrhs_max=1):
    m, h = oracle_hmatrix(key)
    H = hmat.HMatrix(blockset(h), variant, c=1, nrhs_max=nrhs_max)
    H64 = hmat.HMatrix(blockset(h), oracle.M1_DOUBLE, nrhs_max=nrhs_max) if variant != oracle.M1_DOUBLE else H
    return m, h, H, H64


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.BF16_SCALED])
@pytest.mark.parametrize("restart", [8, 30])
def test_gmres_matches_oracle(variant, restart):
    """Same status, step counts within a few (the estimate crosses tol after
    summation-order differences), the first five estimates to 1e-8, the FP64
    true residual below tol and the solution as close to a tight FP64 solve
    as the oracle's.  The products differ from the oracle's by summation
    order only (1e-15 of |A~||x|), but this operator smooths (|A~x| is 1e-3 of
    |A~||x| on these vectors), so the Arnoldi vectors differ by ~1e-12 and the
    estimates by up to ~1e-11 after four steps (measured; the bound leaves
    room for the fifth)."""
    need_gpu()
    m, h, H, H64 = setup("sphere-L4", variant)
    b = m.rhs()[h.perm]
    x, info = hmat.hmat_gmres(H, to_dev(b), h_fp64=H64, tol=1e-8, restart=restart, maxiter=600, history=True)
    op, op64 = oracle.Converted(h, variant, 1), oracle.Converted(h, oracle.M1_DOUBLE)
    xo, io = OG.gmres(op.matvec, b, matvec64=op64.matvec, tol=1e-8, restart=restart, maxiter=600)
    print(f"{oracle.VARIANT_NAMES[variant]} m={restart}: gpu {info['iterations']} steps {info['restarts']} restarts, "
          f"oracle {io['iterations']} steps {io['cycles'] - 1} restarts")
    assert info["status"] == 0 and io["status"] == OG.OK
    assert abs(info["iterations"] - io["iterations"]) <= max(3, io["iterations"] // 10)
    # one product per step (x_0 = 0: r_0 = b needs none; the oracle forms it)
    assert info["true_rel_res"] < 1e-8 and info["matvecs"] == info["iterations"]
    k = min(5, io["iterations"])
    est = info["history"][1:k + 1]
    rel = np.abs(est - io["history"][:k]) / io["history"][:k]
    print("estimate relative differences", rel)
    assert rel.max() <= 1e-8
    xr, _ = oracle.bicgstab(op64, b, tol=1e-12)
    eg = np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr)
    eo = np.linalg.norm(xo - xr) / np.linalg.norm(xr)
    assert eg <= max(3 * eo, 1e-9), (eg, eo)


@pytest.mark.parametrize("k", [1, 4, 12])
def test_gmres_estimate_equals_true_residual(k):
    """Stopped after k steps (maxiter), the FP64 operator's true residual of
    the returned x equals the last estimate |g_k|/|b| (M1-Double: the
    iteration and the check use the same operator)."""
    need_gpu()
    m, h, H, _ = setup("plates-16", oracle.M1_DOUBLE)
    b = m.rhs()[h.perm]
    x, info = hmat.hmat_gmres(H, to_dev(b), tol=1e-30, restart=30, maxiter=k, history=True)
    assert info["status"] == hmat.HMAT_E_NOCONV and info["iterations"] == k
    assert abs(info["history"][k] - info["true_rel_res"]) <= 1e-10 * info["true_rel_res"]


def test_gmres_graph_poll_and_multirhs_handle():
    """Graph replay and the polling interval change nothing, bit for bit;
    a multi-RHS handle (matrix-core product) converges the same way."""
    need_gpu()
    m, h, H, H64 = setup("spheres-mixed", oracle.M2_MIXED)
    b = to_dev(m.rhs()[h.perm])
    runs = [hmat.hmat_gmres(H, b, h_fp64=H64, restart=12, use_graph=g, poll_every=p)
            for g, p in ((False, 1), (True, 5), (False, 7))]
    x0 = runs[0][0].cpu().numpy()
    for x, info in runs[1:]:
        assert np.array_equal(x.cpu().numpy(), x0)
        assert info["iterations"] == runs[0][1]["iterations"] and info["matvecs"] == runs[0][1]["matvecs"]
    _, _, Hm, Hm64 = setup("spheres-mixed", oracle.M2_MIXED, nrhs_max=16)
    xm, im = hmat.hmat_gmres(Hm, b, h_fp64=Hm64, restart=12)
    assert im["status"] == 0 and abs(im["iterations"] - runs[0][1]["iterations"]) <= 3
    assert np.linalg.norm(xm.cpu().numpy() - x0) / np.linalg.norm(x0) < 1e-6


def test_gmres_edges_and_preconditioner():
    need_gpu()
    import torch

    m, h, H, H64 = setup("sphere-L3", oracle.M1_DOUBLE)
    n = h.n
    x, info = hmat.hmat_gmres(H, torch.zeros(n, dtype=torch.float64, device="cuda"), x=to_dev(np.ones(n)))
    assert info["status"] == 0 and info["iterations"] == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(hmat.HmatError):
        hmat.hmat_gmres(H, to_dev(np.ones(n)), restart=0)
    with pytest.raises(hmat.HmatError):
        hmat.hmat_gmres(H, to_dev(np.ones(n)), restart=129)
    bh = m.rhs()[h.perm]
    b = to_dev(bh)
    x0, i0 = hmat.hmat_gmres(H, b, tol=1e-10, restart=30)
    P = hmat.Precond(blockset(h), hmat.PRECOND_JACOBI)
    x1, i1 = hmat.hmat_gmres(H, b, tol=1e-10, restart=30, precond=P)
    assert i0["status"] == 0 and i1["status"] == 0
    # right preconditioning as the oracle does it (x = K u), same steps
    op = oracle.Converted(h, oracle.M1_DOUBLE)
    xo, io = OG.gmres(op.matvec, bh, tol=1e-10, restart=30, precond=oracle.Jacobi(h).apply)
    assert abs(i1["iterations"] - io["iterations"]) <= 2
    a, c = x0.cpu().numpy(), x1.cpu().numpy()
    assert np.linalg.norm(a - c) / np.linalg.norm(a) < 1e-7 and np.linalg.norm(c - xo) / np.linalg.norm(xo) < 1e-8
    print(f"iterations: none {i0['iterations']}, block-Jacobi {i1['iterations']} (oracle {io['iterations']})")


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.BF16_SCALED])
@pytest.mark.parametrize("restart", [6, 20])
def test_gmres_one_cycle_matches_oracle(variant, restart):
    """Exactly one cycle of `restart` steps (tol unreachable): the solution
    after the cycle's update, x = x_0 + V y, equals the oracle's element by
    element.  The products differ from the oracle's by summation order only;
    the Arnoldi vectors carry that difference (about 1e-12 after a few steps
    on this smoothing operator) into y, so the bound is 1e-9."""
    need_gpu()
    m, h, H, H64 = setup("sphere-L4", variant)
    b = m.rhs()[h.perm] + 0.2 * np.random.default_rng(3).standard_normal(h.n)
    x, info = hmat.hmat_gmres(H, to_dev(b), h_fp64=H64, tol=1e-30, restart=restart, maxiter=restart, history=True)
    op, op64 = oracle.Converted(h, variant, 1), oracle.Converted(h, oracle.M1_DOUBLE)
    xo, io = OG.gmres(op.matvec, b, matvec64=op64.matvec, tol=1e-30, restart=restart, maxiter=restart)
    assert info["iterations"] == io["iterations"] == restart
    assert info["restarts"] == 0 and io["cycles"] == 1
    x = x.cpu().numpy()
    e = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"{oracle.VARIANT_NAMES[variant]} m={restart}: max |x - x_oracle| / max |x_oracle| = {e:.2e}")
    assert e <= 1e-9
    est = info["history"][1:restart + 1]
    assert np.allclose(est, io["history"][:restart], rtol=1e-7, atol=0)
