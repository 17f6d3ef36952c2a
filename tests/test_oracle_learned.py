"""Pins of the learned-preconditioner oracle (oracle/learned.py) against
what mathematics fixes: central finite differences of the loss, the closed
form of Adam's first step, a loss of exactly zero when M_tau can equal the
inverse, invariances of the geometry features, and the apply equal to the
dense M_tau product."""

import numpy as np
import pytest

import oracle
from oracle import learned as L
from tests.conftest import oracle_hmatrix


def leaf_samples(key="sphere-L3", count=4, seed=0):
    """(X, ainv, dinv, sinv, m, blocks) for `count` diagonal leaves of a test mesh."""
    m_, h = oracle_hmatrix(key)
    cent, nrm, area = m_.centroids[h.perm], m_.normals[h.perm], m_.areas[h.perm]
    ids = [b for b in range(h.nblocks) if h.kind[b] == 0 and h.row0[b] == h.col0[b]]
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(ids), size=count, replace=False)
    B = len(pick)
    X = np.zeros((B, L.IN))
    ainv = np.zeros((B, L.LEAF, L.LEAF))
    dinv = np.zeros((B, L.LEAF))
    sinv = np.zeros(B)
    mm = np.zeros(B, dtype=np.int64)
    blocks = []
    for q, i in enumerate(pick):
        b = ids[i]
        r0, k = int(h.row0[b]), int(h.nrows[b])
        A = h.data[h.offset[b]:h.offset[b] + k * k].reshape(k, k, order="F")
        X[q] = L.leaf_features(cent[r0:r0 + k], nrm[r0:r0 + k], area[r0:r0 + k])
        ainv[q, :k, :k] = oracle.invert(A)
        dinv[q, :k] = 1.0 / np.diag(A)
        sinv[q] = 1.0 / np.diag(A).mean()
        mm[q] = k
        blocks.append(A)
    return X, ainv, dinv, sinv, mm, blocks


def random_params(seed=3, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in L.SHAPES:
        fan_in = shp[0] if len(shp) == 2 else 1
        p[name] = rng.standard_normal(shp) * (scale * np.sqrt(2.0 / fan_in) if len(shp) == 2 else 0.1)
    return L.flatten(p)


def test_loss_gradient_central_differences():
    """Backward pass vs central differences (h = 1e-6) on sampled entries of
    every parameter tensor: relative error <= 1e-6."""
    X, ainv, dinv, sinv, m, _ = leaf_samples(count=3)
    flat = random_params(scale=0.3)
    loss, g = L.loss_and_grad(flat, X, ainv, dinv, sinv, m)
    rng = np.random.default_rng(7)
    off = 0
    for name, shp in L.SHAPES:
        k = int(np.prod(shp))
        idx = off + rng.choice(k, size=min(25, k), replace=False)
        fd = np.empty(idx.size)
        for j, i in enumerate(idx):
            hstep = 1e-6 * max(1.0, abs(flat[i]))
            fp, fm = flat.copy(), flat.copy()
            fp[i] += hstep
            fm[i] -= hstep
            fd[j] = (L.loss_and_grad(fp, X, ainv, dinv, sinv, m)[0] - L.loss_and_grad(fm, X, ainv, dinv, sinv, m)[0]) / (2 * hstep)
        err = np.linalg.norm(fd - g[idx]) / max(np.linalg.norm(g[idx]), 1e-300)
        assert err <= 1e-6, (name, err)
        off += k


def test_adam_first_step_closed_form():
    """After one step from zero moments, the bias-corrected ratio is
    g / |g|, so every parameter moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.integers(-4, 3, 50)
    p, m1, m2 = p0.copy(), np.zeros(50), np.zeros(50)
    L.adam_step(p, m1, m2, g, 1, lr=1e-3)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps the step at lr * sign(g) (up to eps)
    for t in range(2, 6):
        L.adam_step(p, m1, m2, g, t, lr=1e-3)
    assert np.allclose(p, p0 - 5e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_loss_zero_when_form_is_exact():
    """With W3 = 0 the network outputs b3 = (U, V); taking the 'inverse' to be
    diag(dinv) + sinv U V^T gives loss 0 and zero gradient.  A transposed
    product (V U^T) or a missing 1/s factor would not."""
    rng = np.random.default_rng(5)
    flat = random_params()
    p = L.unflatten(flat)
    p["W3"][:] = 0.0
    p["b3"][:] = rng.standard_normal(L.OUT)
    X = rng.standard_normal((2, L.IN))
    O, _ = L.forward(flat, X)
    U, V = L.factors(O)
    m = np.array([64, 37])
    dinv = rng.uniform(0.5, 2.0, (2, L.LEAF))
    sinv = np.array([0.7, 1.9])
    ainv = np.zeros((2, L.LEAF, L.LEAF))
    for b in range(2):
        k = m[b]
        ainv[b, :k, :k] = np.diag(dinv[b, :k]) + sinv[b] * U[b, :k] @ V[b, :k].T
    loss, g = L.loss_and_grad(flat, X, ainv, dinv, sinv, m)
    assert loss < 1e-28 and np.abs(g).max() < 1e-12
    ainv_t = ainv.copy()
    for b in range(2):
        k = m[b]
        ainv_t[b, :k, :k] = np.diag(dinv[b, :k]) + sinv[b] * V[b, :k] @ U[b, :k].T
    assert L.loss_and_grad(flat, X, ainv_t, dinv, sinv, m)[0] > 1e-3


def test_features_invariances():
    """Translation and uniform scaling of a leaf leave its features unchanged
    (offsets are divided by the box diagonal, areas by their mean); the mask
    counts the panels; normals pass through."""
    X, _, _, _, m, _ = leaf_samples(count=1)
    m_, h = oracle_hmatrix("sphere-L3")
    k = int(m[0])
    cent, nrm, area = m_.centroids[h.perm][:k], m_.normals[h.perm][:k], m_.areas[h.perm][:k]
    f0 = L.leaf_features(cent, nrm, area)
    f1 = L.leaf_features(3.7 * cent + np.array([1.0, -2.0, 0.5]), nrm, 3.7 ** 2 * area)
    assert np.allclose(f0, f1, rtol=0, atol=1e-13)
    assert f0[L.LEAF * L.NFEAT:].sum() == k and np.all(f0[k * L.NFEAT:L.LEAF * L.NFEAT] == 0)
    F = f0[:k * L.NFEAT].reshape(k, L.NFEAT)
    assert np.allclose(F[:, 0:3].sum(axis=0), 0.0, atol=1e-13)   # offsets from the mean
    assert np.isclose(F[:, 6].mean(), 1.0)                       # areas over their mean
    assert np.allclose(np.linalg.norm(F[:, 3:6], axis=1), 1.0)
    # two panels on the x axis, 2 apart: offsets -+ 1/2 of the unit box diagonal direction
    f = L.leaf_features([[0, 0, 0], [2, 0, 0]], [[0, 0, 1], [0, 0, 1]], [1.0, 3.0])
    assert np.allclose(f[:14], [-0.5, 0, 0, 0, 0, 1, 0.5, 0.5, 0, 0, 0, 0, 1, 1.5])


def test_apply_is_the_dense_map():
    rng = np.random.default_rng(2)
    U, V = rng.standard_normal((64, 16)), rng.standard_normal((64, 16))
    dinv, x = rng.uniform(1, 2, 64), rng.standard_normal(64)
    for m in (64, 23, 1):
        M = L.precond_matrix(U, V, dinv, 0.3, m)
        assert np.allclose(L.apply_leaf(x, U, V, dinv, 0.3, m), M @ x[:m], rtol=1e-13, atol=1e-13)


def test_training_reduces_loss():
    """A few hundred Adam steps on a handful of real leaves cut the loss well
    below its start (the map can at least fit its training set)."""
    X, ainv, dinv, sinv, m, _ = leaf_samples(count=8, seed=4)
    flat = random_params(seed=9, scale=0.5)
    flat[-L.OUT - L.HID * L.OUT:] *= 0.01  # small last layer: M starts near diag^-1
    l0 = L.loss_and_grad(flat, X, ainv, dinv, sinv, m)[0]
    m1, m2 = np.zeros_like(flat), np.zeros_like(flat)
    for t in range(1, 301):
        loss, g = L.loss_and_grad(flat, X, ainv, dinv, sinv, m)
        L.adam_step(flat, m1, m2, g, t, lr=1e-3)
    assert loss < 0.5 * l0, (l0, loss)
