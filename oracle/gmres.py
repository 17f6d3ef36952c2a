"""Restarted GMRES oracle -- TEST INFRASTRUCTURE (plain numpy, FP64).

The paper names GMRES as the next solver for its mixed-precision product
(Sec. 5) without defining one; this is the textbook method (Saad and Schultz,
1986): Arnoldi with classical Gram-Schmidt applied twice, Givens rotations on
the Hessenberg matrix, restart after m steps, right preconditioning x = K u.
Mixed precision follows the BiCGSTAB solver of Sec. 4.1.3: the iteration
uses the operator under test, convergence is confirmed with the FP64 true
residual, and a failed check restarts from the current x with that residual.

Only ``tests/`` may import this module.
"""

from __future__ import annotations

import numpy as np

OK, BREAKDOWN, NOCONV, NONFINITE = 0, 5, 6, 7  # the library's status codes


def gmres(matvec, b, matvec64=None, x0=None, tol=1e-8, restart=30, maxiter=1000, precond=None):
    """Solve A x = b.  matvec: the iteration operator (x -> A x); matvec64:
    the FP64 operator of the true residual (default: matvec); precond: a
    callable K (right preconditioner, default identity).  Returns (x, info):
    status, iterations (inner steps, one product each), matvecs (iteration
    operator), matvecs_fp64, cycles, history (residual estimate |g_{j+1}|/|b|
    after every inner step) and true_rel_res."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    A64 = matvec64 if matvec64 is not None else matvec
    K = precond if precond is not None else (lambda v: v)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = dict(status=OK, iterations=0, matvecs=0, matvecs_fp64=0, cycles=0, history=[], true_rel_res=0.0)
    if bnorm == 0.0:
        return np.zeros(n), info
    r = b - matvec(x)  # the first cycle starts from the iteration operator's residual
    info["matvecs"] += 1
    m = int(restart)
    while True:
        beta = np.linalg.norm(r)
        if not np.isfinite(beta):
            info["status"] = NONFINITE
            break
        info["cycles"] += 1
        V = np.zeros((m + 1, n))
        R = np.zeros((m + 1, m))  # rotated Hessenberg columns (upper triangle used)
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0  # columns of this cycle
        nonfinite = False
        if beta > 0.0:
            V[0] = r / beta
            for j in range(m):
                if info["iterations"] >= maxiter:
                    break
                w = matvec(K(V[j]))
                info["matvecs"] += 1
                info["iterations"] += 1
                # classical Gram-Schmidt, twice
                h = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h
                h2 = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h2
                h = h + h2
                hn = np.linalg.norm(w)
                col = np.zeros(j + 2)
                col[:j + 1] = h
                col[j + 1] = hn
                if not np.all(np.isfinite(col)):
                    nonfinite = True
                    break
                # earlier rotations, then the one that zeroes the subdiagonal
                for i in range(j):
                    a, c = col[i], col[i + 1]
                    col[i] = cs[i] * a + sn[i] * c
                    col[i + 1] = -sn[i] * a + cs[i] * c
                rho = np.hypot(col[j], col[j + 1])
                cs[j], sn[j] = (1.0, 0.0) if rho == 0.0 else (col[j] / rho, col[j + 1] / rho)
                col[j] = rho
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                R[:j + 1, j] = col[:j + 1]
                k = j + 1
                info["history"].append(abs(g[j + 1]) / bnorm)
                if hn == 0.0 or abs(g[j + 1]) / bnorm < tol:
                    break  # exact in the Krylov space, or the estimate reached tol
                V[j + 1] = w / hn
        if nonfinite:
            info["status"] = NONFINITE
            break
        if k > 0:
            # R y = g by back substitution, then x += K (V y)
            y = np.zeros(k)
            for i in range(k - 1, -1, -1):
                y[i] = (g[i] - R[i, i + 1:k] @ y[i + 1:k]) / R[i, i]
            x = x + K(V[:k].T @ y)
        r = b - A64(x)  # FP64 true residual (Sec. 4.1.3)
        info["matvecs_fp64"] += 1
        info["true_rel_res"] = np.linalg.norm(r) / bnorm
        if info["true_rel_res"] < tol:
            break
        if k == 0 and beta > 0.0:  # no step was possible
            info["status"] = NONFINITE if not np.isfinite(info["true_rel_res"]) else NOCONV
            break
        if info["iterations"] >= maxiter:
            info["status"] = NOCONV
            break
    info["history"] = np.array(info["history"])
    return x, info
