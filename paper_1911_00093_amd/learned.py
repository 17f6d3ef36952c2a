"""Learned leaf-block preconditioner (not in the paper): training set,
training loop and the factors of a mesh's leaves.

Host orchestration only.  The library computes everything: the H-matrix
assembly (cluster tree and dense diagonal leaves), the leaf features, the
exact FP64 leaf inverses, the MLP forward / backward / Adam steps on the GPU
and the preconditioner apply inside BiCGSTAB.  Seeded draws (initial
parameters, batch order) come from `seeded`.
"""

from __future__ import annotations

import numpy as np

from . import hmat, meshes, seeded

LEAF = hmat.MLP_LEAF


def leaf_inputs(mesh, bs: hmat.BlockSet, with_inverse: bool = False):
    """Per diagonal leaf of an assembled mesh, in the preconditioner's leaf
    order: features (k, 512) float32, 1 / A_ii (k, 64), 1 / s_tau (k,),
    panel count m (k,), and with_inverse the exact inverse (k, 64, 64),
    row-major with the leaf's inverse in the leading m x m corner (all
    leaves inverted in one batch on the GPU)."""
    blk, r0, m = hmat.precond_leaves(bs, hmat.PRECOND_LEARNED)
    k = blk.size
    cent, nrm, area = mesh.centroids[bs.perm], mesh.normals[bs.perm], mesh.areas[bs.perm]
    x = np.zeros((k, hmat.MLP_IN), np.float32)
    dinv = np.zeros((k, LEAF), np.float32)
    sinv = np.zeros(k, np.float32)
    ainv = np.zeros((k, LEAF, LEAF), np.float32) if with_inverse else None
    leaves = []
    for q in range(k):
        a, mm = int(r0[q]), int(m[q])
        x[q] = hmat.hmat_leaf_features(cent[a:a + mm], nrm[a:a + mm], area[a:a + mm])
        off = int(bs.offset[blk[q]])
        A = bs.data[off:off + mm * mm].reshape(mm, mm, order="F")
        dinv[q], sinv[q] = hmat.hmat_leaf_scales(A)
        leaves.append(A)
    if with_inverse:
        for q, Ai in enumerate(hmat.dense_inverses(leaves)):
            ainv[q, :Ai.shape[0], :Ai.shape[0]] = Ai
    return dict(x=x, dinv=dinv, sinv=sinv, m=m.astype(np.int32), ainv=ainv)


def training_set(target: int = 20000, seed: int = 1, leaf: int = 64, eta: float = 2.0, eps: float = 1e-3,
                 log=None):
    """At least `target` diagonal leaves (then cut to target) from random
    ellipsoids and plate pairs, with exact FP64 inverses as targets.  The
    ACA tolerance only affects the far field, which training does not use."""
    parts, have, nmesh = [], 0, 0
    for mesh in meshes.learned_training_meshes(seed):
        bs = hmat.hmat_assemble_bem(mesh.centroids, mesh.areas, leaf=leaf, eta=eta, eps=eps)
        d = leaf_inputs(mesh, bs, with_inverse=True)
        parts.append(d)
        have += d["m"].size
        nmesh += 1
        if log and nmesh % 10 == 0:
            log(f"[train-set] {nmesh} meshes, {have} leaves")
        if have >= target:
            break
    out = {key: np.concatenate([p[key] for p in parts])[:target] for key in ("x", "dinv", "sinv", "m", "ainv")}
    out["meshes"] = nmesh
    return out


def to_device(data, device="cuda"):
    import torch

    return {key: torch.as_tensor(np.ascontiguousarray(data[key])).to(device)
            for key in ("x", "dinv", "sinv", "m", "ainv")}


def train(data_dev, params0=None, epochs: int = 100, batch: int = 256, lr: float = 2e-3, lr_final: float = 2e-4,
          seed: int = 0, log=None):
    """Adam on the batch mean loss with a cosine decay of the rate from lr
    to lr_final; returns the trained hmat.MLP and the mean loss of every
    epoch (read once per epoch)."""
    import math

    import torch

    n = int(data_dev["m"].numel())
    net = hmat.MLP(seeded.init_params(seed) if params0 is None else params0, device=data_dev["x"].device)
    history = []
    steps_per_epoch = max(1, n // batch)
    total = steps_per_epoch * epochs
    acc = torch.zeros(1, dtype=torch.float32, device=data_dev["x"].device)
    # every step's sample indices go to the device at once: a copy per step
    # from pageable memory would wait for the previous step's kernels
    order = torch.as_tensor(np.stack(list(seeded.batch_order(n, batch, epochs, seed)))).to(data_dev["x"].device)
    step = 0
    for idx_d in order:
        net.loss_grad(data_dev, idx_d)
        acc += net.loss
        net.adam(lr_final + (lr - lr_final) * 0.5 * (1.0 + math.cos(math.pi * step / total)))
        step += 1
        if step % steps_per_epoch == 0:
            history.append(float(acc.item()) / steps_per_epoch)
            acc.zero_()
            if log:
                log(f"[train] epoch {len(history)}: loss {history[-1]:.4f}")
    return net, history


def mean_loss(net: hmat.MLP, data_dev, batch: int = 1024) -> float:
    """Mean loss of the network over every sample of a device data set."""
    import torch

    n = int(data_dev["m"].numel())
    tot = 0.0
    for s in range(0, n, batch):
        idx = torch.arange(s, min(n, s + batch), dtype=torch.int32, device=data_dev["x"].device)
        net.loss_grad(data_dev, idx)
        tot += float(net.loss.item()) * idx.numel()
    return tot / n


def factors(net: hmat.MLP, mesh, bs: hmat.BlockSet, chunk: int = 8192):
    """Device float32 (leaves, 2048): the predicted U, V of every diagonal
    leaf of an assembled mesh, in the preconditioner's leaf order."""
    import torch

    d = leaf_inputs(mesh, bs)
    x = torch.as_tensor(d["x"]).to(net.params.device)
    out = torch.empty((x.shape[0], hmat.MLP_OUT), dtype=torch.float32, device=x.device)
    for s in range(0, x.shape[0], chunk):
        net.forward(x[s:s + chunk], out=out[s:s + chunk])
    return out
