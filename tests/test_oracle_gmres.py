"""Pins of the restarted GMRES oracle (oracle/gmres.py) against what the
mathematics fixes: direct solves, finite termination, the least-squares
residual estimate equal to the true residual, its monotone decrease within
a cycle, exact preconditioning, and the mixed-precision protocol on an
H-matrix (FP64 true residual confirms convergence)."""

import numpy as np
import pytest

import oracle
from oracle import gmres as G
from tests.conftest import oracle_hmatrix


def dense_system(n=40, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4.0 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    return A, b


def test_dense_vs_direct_solve():
    A, b = dense_system()
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-12, restart=40)
    xs = np.linalg.solve(A, b)
    assert info["status"] == G.OK
    assert np.linalg.norm(x - xs) <= np.linalg.cond(A) * 1e-12 * np.linalg.norm(xs) * 10


def test_finite_termination():
    """Without restarts GMRES finds the solution in at most n steps."""
    A, b = dense_system(n=20, seed=1)
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-13, restart=20)
    assert info["status"] == G.OK and info["iterations"] <= 20 and info["cycles"] == 1
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_estimate_equals_true_residual(k):
    """After k steps the rotated right-hand side's last entry |g_k| is the
    residual of the least-squares solution: stopping there (maxiter = k) and
    forming x gives |b - A x| = |g_k| to rounding."""
    A, b = dense_system(n=30, seed=2)
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-30, restart=30, maxiter=k)
    assert info["iterations"] == k and info["status"] == G.NOCONV
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(info["history"][-1] - true) <= 1e-12 * true + 1e-15
    assert abs(info["true_rel_res"] - true) <= 1e-14


def test_estimate_monotone_within_cycle():
    """Each step minimises the residual over a larger Krylov space."""
    A, b = dense_system(n=60, seed=3)
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-10, restart=60)
    h = info["history"]
    assert np.all(np.diff(h) <= 1e-15 * h[:-1])


def test_restart_converges_and_counts():
    A, b = dense_system(n=60, seed=4)
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-10, restart=5, maxiter=500)
    assert info["status"] == G.OK and info["cycles"] >= 2
    assert info["matvecs"] == 1 + info["iterations"] and info["matvecs_fp64"] == info["cycles"]
    assert np.linalg.norm(b - A @ x) < 1e-10 * np.linalg.norm(b)


def test_identity_one_step_and_zero_rhs():
    n = 25
    b = np.random.default_rng(5).standard_normal(n)
    x, info = G.gmres(lambda v: v.copy(), b, tol=1e-12)
    assert info["iterations"] == 1 and np.allclose(x, b, rtol=0, atol=1e-15)
    x0, i0 = G.gmres(lambda v: v.copy(), np.zeros(n))
    assert np.all(x0 == 0) and i0["iterations"] == 0 and i0["status"] == G.OK


def test_exact_right_preconditioner_one_step():
    A, b = dense_system(n=30, seed=6)
    Ainv = np.linalg.inv(A)
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-11, precond=lambda v: Ainv @ v)
    assert info["iterations"] == 1 and np.linalg.norm(x - Ainv @ b) <= 1e-12 * np.linalg.norm(Ainv @ b)


def test_nonfinite():
    A, b = dense_system(n=10, seed=7)
    A[3, 4] = np.nan
    x, info = G.gmres(lambda v: A @ v, b)
    assert info["status"] == G.NONFINITE


@pytest.mark.parametrize("variant", [oracle.M1_DOUBLE, oracle.M2_MIXED])
def test_mixed_precision_protocol_on_hmatrix(variant):
    """The iteration operator is the converted H-matrix, the FP64 true
    residual confirms 1e-8, and the solution agrees with an FP64 BiCGSTAB
    solve to 1e-12 within the conditioning bound."""
    m, h = oracle_hmatrix("sphere-L3")
    b = m.rhs()[h.perm]
    op = oracle.Converted(h, variant)
    op64 = oracle.Converted(h, oracle.M1_DOUBLE)
    x, info = G.gmres(op.matvec, b, matvec64=op64.matvec, tol=1e-8, restart=20)
    assert info["status"] == G.OK and info["true_rel_res"] < 1e-8
    xr, ir = oracle.bicgstab(op64, b, tol=1e-12)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-6
    print(f"{oracle.VARIANT_NAMES[variant]}: {info['iterations']} steps, {info['cycles']} cycles")


def test_orthogonality_kept_on_ill_conditioned_system():
    """Eigenvalues spread over eight decades: the basis stays orthogonal
    (Gram-Schmidt applied twice), so after 60 steps the residual estimate
    still equals the true residual to 1e-9 (one Gram-Schmidt pass drifts to
    ~1e-8 here)."""
    n = 80
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.logspace(0, 8, n)) @ Q.T + 1e-3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = G.gmres(lambda v: A @ v, b, tol=1e-30, restart=80, maxiter=60)
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(info["history"][-1] - true) <= 1e-9 * true
