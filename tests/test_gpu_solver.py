"""GPU BiCGSTAB (Algorithm 1) against the oracle's BiCGSTAB, breakdown and
edge cases, and the block-Jacobi preconditioner."""

import numpy as np
import pytest

import oracle
from paper_1911_00093_amd import hmat
from tests.conftest import oracle_hmatrix
from tests.gpu_util import blockset, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _iterations_over_dot_orders(op, b, tol, maxiter):
    """Iterations Algorithm 1 takes with the oracle's operator when only the
    summation order of its inner products changes (sequential as in the
    oracle, numpy's pairwise sum, and sums of chunk sums as the GPU forms
    them).  The paper fixes no order, and near a residual plateau the step at
    which |r|/|b| crosses tol moves with it (plates-32 at 1e-10: 42 to 46)."""
    def seq(a, c):
        t = 0.0
        for u in (a * c).tolist():
            t += u
        return t

    def chunked(k):
        return lambda a, c: seq(np.add.reduceat(a * c, np.arange(0, a.size, k)), np.ones((a.size + k - 1) // k))

    counts = []
    for dot in (seq, np.dot, chunked(64), chunked(256)):
        x = np.zeros_like(b)
        r = b - op(x)
        rt = r.copy()
        bn = np.sqrt(dot(b, b))
        rho_prev = alpha = omega = 1.0
        p = v = None
        it_done = maxiter
        for it in range(1, maxiter + 1):
            rho = dot(rt, r)
            p = r.copy() if it == 1 else r + (rho / rho_prev) * (alpha / omega) * (p - omega * v)
            v = op(p)
            alpha = rho / dot(rt, v)
            s_ = r - alpha * v
            if np.sqrt(dot(s_, s_)) / bn < tol:
                it_done = it
                break
            t = op(s_)
            omega = dot(t, s_) / dot(t, t)
            x += alpha * p + omega * s_
            r = s_ - omega * t
            rho_prev = rho
            if np.sqrt(dot(r, r)) / bn < tol:
                it_done = it
                break
        counts.append(it_done)
    return counts


@pytest.mark.parametrize("key", ["sphere-L4", "plates-32"])
def test_bicgstab_fp64_matches_oracle(key):
    need_gpu()
    m, h = oracle_hmatrix(key)
    b = m.rhs()[h.perm]
    bs = blockset(h)
    H = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    x, info = hmat.hmat_bicgstab(H, to_dev(b), tol=1e-10, maxiter=300, history=True)
    op = oracle.Converted(h, oracle.M1_DOUBLE)
    xo, io = oracle.bicgstab(op, b, tol=1e-10, maxiter=300)
    assert info["status"] == 0 and io["status"] == 0
    # the iteration count is fixed only up to the inner products' summation
    # order: the GPU's lies within the range those orders give (+-1)
    counts = _iterations_over_dot_orders(op.matvec, b, 1e-10, 300)
    print(f"{key}: iterations gpu {info['iterations']}, oracle {io['iterations']}, over dot orders {counts}")
    assert io["iterations"] == counts[0]
    assert min(counts) - 1 <= info["iterations"] <= max(counts) + 1
    x = x.cpu().numpy()
    # both solves stop at |r|/|b| < 1e-10, so each is off the exact solution
    # by up to kappa * 1e-10; compare each with a tight solve instead
    xt, _ = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), b, tol=1e-14, maxiter=500)
    e_gpu = np.linalg.norm(x - xt) / np.linalg.norm(xt)
    e_ora = np.linalg.norm(xo - xt) / np.linalg.norm(xt)
    print(f"{key}: iters gpu {info['iterations']} oracle {io['iterations']}, x err gpu {e_gpu:.2e} oracle {e_ora:.2e}")
    assert e_gpu <= 10 * e_ora + 1e-12
    assert info["true_rel_res"] < 1e-10
    # the recurrence history follows the oracle's over the first iterations.
    # BiCGSTAB amplifies rounding quickly: the same operator with pairwise
    # instead of sequential dot products already moves |r_1|/|b| by ~2e-11
    # and |r_2|/|b| by ~6e-10 on this mesh, so compare at 1e-8 there
    hg, ho = info["history"][:3], io["history"][:3]
    assert np.allclose(hg, ho, rtol=1e-8, atol=0)


@pytest.mark.parametrize("variant", [oracle.M1_SINGLE, oracle.M1_MIXED, oracle.M2_SINGLE, oracle.M2_MIXED, oracle.M3,
                                     oracle.BF16_SCALED])
def test_bicgstab_mixed_true_residual(variant):
    """Mixed operators: convergence is confirmed with the FP64 true residual
    (Sec. 4.1.3); the solution error against the FP64 solve is reported."""
    need_gpu()
    m, h = oracle_hmatrix("sphere-L4")
    b = m.rhs()[h.perm]
    bs = blockset(h)
    H64 = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    Hm = hmat.HMatrix(bs, variant, c=-1)
    x, info = hmat.hmat_bicgstab(Hm, to_dev(b), h_fp64=H64, tol=1e-8, maxiter=500)
    assert info["status"] == 0, info
    assert info["true_rel_res"] < 1e-8
    op64 = oracle.Converted(h, oracle.M1_DOUBLE)
    x = x.cpu().numpy()
    assert np.linalg.norm(b - op64.matvec(x)) / np.linalg.norm(b) < 1e-8
    xo, io = oracle.bicgstab(op64, b, tol=1e-12, maxiter=500)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    # a residual of 1e-8 leaves an error of up to kappa * 1e-8 in x for any
    # operator; the FP64 oracle stopped at the same tolerance shows how much
    x8, _ = oracle.bicgstab(op64, b, tol=1e-8, maxiter=500)
    err64 = np.linalg.norm(x8 - xo) / np.linalg.norm(xo)
    print(f"{oracle.VARIANT_NAMES[variant]}: iters {info['iterations']} restarts {info['restarts']} "
          f"x err vs FP64 {err:.2e} (FP64 at the same tol: {err64:.2e})")
    assert err < 10 * err64 + 1e-9
    # the oracle running the same operator converges too
    xm, im = oracle.bicgstab(oracle.Converted(h, variant, -1), b, op64=op64, tol=1e-8, maxiter=500)
    assert im["status"] == 0


def _dense(A):
    n = A.shape[0]
    h = oracle.HMatrix.from_blocks(n, [0], [n], [0], [n], [0], [0], [0], np.asfortranarray(A).ravel(order="F"))
    return h, hmat.HMatrix(blockset(h), oracle.M1_DOUBLE)


def test_bicgstab_breakdowns_and_edges():
    need_gpu()
    # omega = 0 (exact): A = [[-2,-2],[-2,0]], b = (1,2)
    h, H = _dense(np.array([[-2.0, -2.0], [-2.0, 0.0]]))
    x, info = hmat.hmat_bicgstab(H, to_dev([1.0, 2.0]))
    assert info["status"] == hmat.HMAT_E_BREAKDOWN
    # r~^T v = 0: A = diag(1, -1), b = (1, 1)
    h, H = _dense(np.diag([1.0, -1.0]))
    x, info = hmat.hmat_bicgstab(H, to_dev([1.0, 1.0]))
    assert info["status"] == hmat.HMAT_E_BREAKDOWN
    # identity: one iteration
    h, H = _dense(np.eye(70))
    b = np.arange(1.0, 71.0)
    x, info = hmat.hmat_bicgstab(H, to_dev(b), tol=1e-10)
    assert info["status"] == 0 and info["iterations"] == 1
    assert np.array_equal(x.cpu().numpy(), b)
    # b = 0: x = 0 without iterating
    x0 = to_dev(np.ones(70))
    x, info = hmat.hmat_bicgstab(H, to_dev(np.zeros(70)), x=x0)
    assert info["status"] == 0 and info["iterations"] == 0 and np.all(x.cpu().numpy() == 0)
    # maxiter reached
    rng = np.random.default_rng(8)
    A = np.eye(40) + rng.standard_normal((40, 40))
    h, H = _dense(A)
    x, info = hmat.hmat_bicgstab(H, to_dev(rng.standard_normal(40)), tol=1e-14, maxiter=2)
    assert info["status"] == hmat.HMAT_E_NOCONV and info["iterations"] == 2
    with pytest.raises(hmat.HmatError):
        hmat.hmat_bicgstab(H, to_dev(rng.standard_normal(40)), tol=1e-14, maxiter=2, raise_on_error=True)


def test_bicgstab_nonfinite():
    need_gpu()
    m, h = oracle_hmatrix("plates-32")
    H = hmat.HMatrix(blockset(h), oracle.M1_DOUBLE)
    b = m.rhs()[h.perm].copy()
    b[3] = np.inf
    x, info = hmat.hmat_bicgstab(H, to_dev(b), maxiter=20)
    assert info["status"] in (hmat.HMAT_E_NONFINITE, hmat.HMAT_E_BREAKDOWN)


@pytest.mark.parametrize("nrhs_max", [1, 16])
def test_bicgstab_poll_every_same_result(nrhs_max):
    """Iterations queued past convergence (the rest of a poll window) are
    no-ops on the device, products included: the same x bit for bit and the
    same product count whatever the window; a multi-RHS handle (matrix-core
    product) serves the single solver too."""
    need_gpu()
    m, h = oracle_hmatrix("sphere-L4")
    b = to_dev(m.rhs()[h.perm])
    H = hmat.HMatrix(blockset(h), oracle.M2_MIXED, nrhs_max=nrhs_max)
    H64 = hmat.HMatrix(blockset(h), oracle.M1_DOUBLE, nrhs_max=nrhs_max)
    x1, i1 = hmat.hmat_bicgstab(H, b, h_fp64=H64, poll_every=1)
    x5, i5 = hmat.hmat_bicgstab(H, b, h_fp64=H64, poll_every=5)
    x7, i7 = hmat.hmat_bicgstab(H, b, h_fp64=H64, poll_every=7, use_graph=True)
    print(i1, i5, i7)
    assert i1["status"] == 0 and i1["iterations"] == i5["iterations"] == i7["iterations"]
    # x_0 = 0: r_0 = b without a product, then two products per iteration
    assert i1["matvecs"] == i5["matvecs"] == i7["matvecs"] == 2 * i1["iterations"]
    assert i1["matvecs_fp64"] == i5["matvecs_fp64"] == i7["matvecs_fp64"]
    assert np.array_equal(x1.cpu().numpy(), x5.cpu().numpy())
    assert np.array_equal(x1.cpu().numpy(), x7.cpu().numpy())


def test_jacobi_apply_and_preconditioned_solve():
    need_gpu()
    m, h = oracle_hmatrix("sphere-L4")
    bs = blockset(h)
    P = hmat.Precond(bs)
    J = oracle.Jacobi(h)
    x = np.random.default_rng(4).standard_normal(h.n)
    y = P.apply(to_dev(x)).cpu().numpy()
    yo = J.apply(x)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    b = m.rhs()[h.perm]
    H = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    x0, i0 = hmat.hmat_bicgstab(H, to_dev(b), tol=1e-10)
    x1, i1 = hmat.hmat_bicgstab(H, to_dev(b), tol=1e-10, precond=P)
    assert i0["status"] == 0 and i1["status"] == 0
    xo, io = oracle.bicgstab(oracle.Converted(h, oracle.M1_DOUBLE), b, tol=1e-10, precond=J)
    assert abs(i1["iterations"] - io["iterations"]) <= 1
    a, c = x0.cpu().numpy(), x1.cpu().numpy()
    assert np.linalg.norm(a - c) / np.linalg.norm(a) < 1e-7
    print(f"iterations: none {i0['iterations']}, block-Jacobi {i1['iterations']}")


def test_bicgstab_refine_bf16_matches_oracle():
    """Early FP64 true-residual checks (refine) on the BF16 operator: the
    GPU solve converges with the oracle's policy in about as many
    iterations, and in fewer than without the checks."""
    need_gpu()
    m, h = oracle_hmatrix("plates-32")
    b = m.rhs()[h.perm]
    bs = blockset(h)
    H64 = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    Hb = hmat.HMatrix(bs, oracle.BF16_SCALED)
    x0, i0 = hmat.hmat_bicgstab(Hb, to_dev(b), h_fp64=H64, tol=1e-8, maxiter=500)
    x1, i1 = hmat.hmat_bicgstab(Hb, to_dev(b), h_fp64=H64, tol=1e-8, maxiter=500, refine=1e-2)
    op64 = oracle.Converted(h, oracle.M1_DOUBLE)
    xo, io = oracle.bicgstab(oracle.Converted(h, oracle.BF16_SCALED), b, op64=op64, tol=1e-8, maxiter=500,
                             refine=1e-2)
    assert i0["status"] == 0 and i1["status"] == 0 and io["status"] == 0
    x = x1.cpu().numpy()
    assert np.linalg.norm(b - op64.matvec(x)) / np.linalg.norm(b) < 1e-8
    assert abs(i1["iterations"] - io["iterations"]) <= max(6, io["iterations"] // 4)
    assert i1["iterations"] < i0["iterations"]
    print(f"BF16 iterations: plain {i0['iterations']} ({i0['restarts']} restarts), refine {i1['iterations']} "
          f"({i1['restarts']} restarts), oracle refine {io['iterations']}")
    with pytest.raises(hmat.HmatError):
        hmat.hmat_bicgstab(Hb, to_dev(b), h_fp64=H64, refine=1.5, raise_on_error=True)


@pytest.mark.parametrize("pre", [False, True])
def test_bicgstab_graph_replay_identical(pre):
    """use_graph replays one captured iteration: same iterations, same x bit
    for bit as direct launches, with and without a preconditioner; the FP64
    true-residual products are counted apart from the iteration's."""
    need_gpu()
    m, h = oracle_hmatrix("sphere-L4")
    bs = blockset(h)
    H = hmat.HMatrix(bs, oracle.M2_MIXED)
    H64 = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    P = hmat.Precond(bs) if pre else None
    b = to_dev(m.rhs()[h.perm])
    xa, ia = hmat.hmat_bicgstab(H, b, h_fp64=H64, precond=P, poll_every=3)
    xb, ib = hmat.hmat_bicgstab(H, b, h_fp64=H64, precond=P, poll_every=3, use_graph=True)
    assert ia["status"] == 0 and ib["status"] == 0
    assert ia["iterations"] == ib["iterations"] and np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())
    # two per launched iteration (launches past convergence inside a polling
    # window are no-ops but counted; x_0 = 0 needs no product for r_0), the
    # same with and without graph
    assert ib["matvecs"] == ia["matvecs"] and ia["matvecs"] >= 2 * ia["iterations"]
    assert ib["matvecs_fp64"] == ia["matvecs_fp64"] >= 1
    x64, i64 = hmat.hmat_bicgstab(H64, b, poll_every=3, use_graph=True)
    assert i64["status"] == 0 and i64["matvecs_fp64"] >= 1 and i64["matvecs"] >= 2 * i64["iterations"]


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED, oracle.BF16_SCALED])
@pytest.mark.parametrize("key", ["sphere-L4", "plates-32", "spheres-mixed"])
def test_bicgstab_first_iterations_match_oracle(variant, key):
    """Exactly three iterations of Algorithm 1 (tol unreachable): x_3 equals
    the oracle's x_3 element by element for the same operator arithmetic.
    The product and the solver differ from the oracle only in summation
    order (1e-15 of |A~||x| per product), which three iterations amplify
    about 1000-fold on these meshes (measured on the batched solver), so the
    bound is 1e-10; the recurrence residuals of the three iterations agree
    to 1e-9."""
    need_gpu()
    m, h = oracle_hmatrix(key)
    b = m.rhs()[h.perm]
    if key == "spheres-mixed":  # an unsmooth right-hand side as well
        b = b + 0.3 * np.random.default_rng(11).standard_normal(h.n)
    bs = blockset(h)
    H = hmat.HMatrix(bs, variant, c=-1)
    H64 = hmat.HMatrix(bs, oracle.M1_DOUBLE)
    x, info = hmat.hmat_bicgstab(H, to_dev(b), h_fp64=H64, tol=1e-30, maxiter=3, history=True)
    op, op64 = oracle.Converted(h, variant, -1), oracle.Converted(h, oracle.M1_DOUBLE)
    xo, io = oracle.bicgstab(op, b, op64=op64, tol=1e-30, maxiter=3)
    assert info["status"] == hmat.HMAT_E_NOCONV and io["status"] == hmat.HMAT_E_NOCONV
    assert info["iterations"] == 3 and io["iterations"] == 3
    # the oracle forms r_0 = b - A x_0 with a product; the library skips the
    # product of x_0 = 0 (it adds only zeros)
    assert io["matvecs"] == 7 and info["matvecs"] == 6
    x = x.cpu().numpy()
    e = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"{key} {oracle.VARIANT_NAMES[variant]}: max |x3 - x3_oracle| / max |x3_oracle| = {e:.2e}")
    assert e <= 1e-10
    assert np.allclose(info["history"], io["history"], rtol=1e-9, atol=0)
    # the true residual the GPU reports for x_3 is the oracle's for x_3
    tr = np.linalg.norm(b - op64.matvec(x)) / np.linalg.norm(b)
    assert abs(info["true_rel_res"] - tr) <= 1e-9 * tr


def test_zero_x0_skips_the_initial_product():
    """x_0 exactly zero: r_0 = b without a product (the device checks x_0 and
    the product returns at once); any nonzero x_0 takes the product.  With
    x_0 = 1e-300 in one entry neither r_0 nor the iterates change in FP64, so
    the two solves agree bit for bit and differ by that one product."""
    need_gpu()
    import torch

    m, h = oracle_hmatrix("sphere-L4")
    b = to_dev(m.rhs()[h.perm])
    bs = blockset(h)
    H, H64 = hmat.HMatrix(bs, oracle.M2_MIXED), hmat.HMatrix(bs, oracle.M1_DOUBLE)
    xa, ia = hmat.hmat_bicgstab(H, b, h_fp64=H64, tol=1e-10)
    x0 = torch.zeros(h.n, dtype=torch.float64, device="cuda")
    x0[5] = 1e-300
    xb, ib = hmat.hmat_bicgstab(H, b, x=x0, h_fp64=H64, tol=1e-10)
    assert ia["status"] == ib["status"] == 0 and ia["iterations"] == ib["iterations"]
    assert ia["matvecs"] == 2 * ia["iterations"] and ib["matvecs"] == ia["matvecs"] + 1
    assert torch.equal(xa, xb) and ia["rel_res"] == ib["rel_res"]

