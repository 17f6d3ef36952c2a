"""Learned leaf-block preconditioner: plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg, never by the product path.

Not part of the paper (which uses no preconditioner).  A small MLP maps the
geometry of one leaf cluster tau (at most 64 panels, cluster order) to two
64 x 16 factors U, V; the right preconditioner restricted to tau is the
fixed linear map

    M_tau = diag(A_tau,tau)^-1 + (1 / s_tau) U V^T,

with s_tau the mean self term of tau (rows and columns beyond the leaf's m
panels are ignored).  It is trained to approximate the exact inverse of the
dense diagonal block:

    loss_tau = ||M_tau - A_tau,tau^-1||_F^2 / ||A_tau,tau^-1||_F^2,

averaged over a batch, with Adam (Kingma & Ba, 2015).  Everything here is
written from those definitions in FP64 with numpy; no blocking, fusion or
reordering beyond them.
"""

import numpy as np

LEAF = 64          # panels per leaf (at most)
RANK = 16          # columns of U and V
NFEAT = 7          # (c_p - c_mean) / diam (3), n_p (3), a_p / a_mean (1)
IN = LEAF * NFEAT + LEAF   # features + mask = 512
HID = 128
OUT = 2 * LEAF * RANK      # U then V, each row-major 64 x 16

SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, OUT)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat):
    """Flat parameter vector (W1 row-major, b1, W2, b2, W3, b3) -> dict of views."""
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = flat[o:o + k].reshape(shp)
        o += k
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def leaf_features(cent, normals, areas):
    """Input vector of one leaf: per panel p (cluster order) the offset of its
    centroid from the leaf's mean centroid divided by the diagonal of the
    leaf's centroid bounding box, its unit normal and its area over the mean
    area; zero for p >= m; then a mask of m ones and 64 - m zeros."""
    cent = np.asarray(cent, dtype=np.float64).reshape(-1, 3)
    normals = np.asarray(normals, dtype=np.float64).reshape(-1, 3)
    areas = np.asarray(areas, dtype=np.float64)
    m = areas.size
    assert 1 <= m <= LEAF
    mean = cent.sum(axis=0) / m
    diam = float(np.linalg.norm(cent.max(axis=0) - cent.min(axis=0)))
    if diam == 0.0:
        diam = 1.0
    x = np.zeros(IN)
    f = np.empty((m, NFEAT))
    f[:, 0:3] = (cent - mean) / diam
    f[:, 3:6] = normals
    f[:, 6] = areas / (areas.sum() / m)
    x[:m * NFEAT] = f.ravel()
    x[LEAF * NFEAT:LEAF * NFEAT + m] = 1.0
    return x


def forward(flat, X):
    """H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), O = H2 W3 + b3."""
    p = unflatten(flat)
    Z1 = X @ p["W1"] + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    O = H2 @ p["W3"] + p["b3"]
    return O, (X, Z1, H1, Z2, H2)


def factors(O):
    """U, V of every sample: (B, 64, 16) each."""
    B = O.shape[0]
    return O[:, :LEAF * RANK].reshape(B, LEAF, RANK), O[:, LEAF * RANK:].reshape(B, LEAF, RANK)


def precond_matrix(U, V, dinv, sinv, m):
    """M_tau on the leaf's m panels: diag(dinv) + sinv U V^T."""
    return np.diag(dinv[:m]) + sinv * (U[:m] @ V[:m].T)


def loss_and_grad(flat, X, ainv, dinv, sinv, m):
    """Batch mean of loss_tau and its gradient with respect to the flat
    parameters.  ainv: (B, 64, 64) with the exact inverse in the leading
    m x m corner; dinv: (B, 64) = 1 / A_ii; sinv: (B,) = 1 / s_tau."""
    O, (X, Z1, H1, Z2, H2) = forward(flat, X)
    B = O.shape[0]
    U, V = factors(O)
    dU = np.zeros_like(U)
    dV = np.zeros_like(V)
    loss = 0.0
    for b in range(B):
        k = int(m[b])
        T = ainv[b, :k, :k]
        R = precond_matrix(U[b], V[b], dinv[b], sinv[b], k) - T
        N = float((T * T).sum())
        loss += float((R * R).sum()) / N
        # d/dU of ||R||^2 / N with R = ... + sinv U V^T: (2 / N) sinv R V
        dU[b, :k] = (2.0 / N) * sinv[b] * (R @ V[b, :k])
        dV[b, :k] = (2.0 / N) * sinv[b] * (R.T @ U[b, :k])
    loss /= B
    dO = np.concatenate([dU.reshape(B, -1), dV.reshape(B, -1)], axis=1) / B
    p = unflatten(flat)
    g = {}
    g["W3"] = H2.T @ dO
    g["b3"] = dO.sum(axis=0)
    dZ2 = (dO @ p["W3"].T) * (Z2 > 0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"].T) * (Z1 > 0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return loss, flatten(g)


def adam_step(flat, m1, m2, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1), in place on flat, m1, m2."""
    m1 *= beta1
    m1 += (1.0 - beta1) * grad
    m2 *= beta2
    m2 += (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = m2 / (1.0 - beta2 ** t)
    flat -= lr * mhat / (np.sqrt(vhat) + eps)


def apply_leaf(x, U, V, dinv, sinv, m):
    """M_tau x for the leaf's m entries of x."""
    x = np.asarray(x, dtype=np.float64)[:m]
    return dinv[:m] * x + sinv * (U[:m] @ (V[:m].T @ x))
