"""Seeded random inputs of the learned leaf map: initial parameters and the
order in which training samples are visited.  Random draws only (numpy
PCG64); no arithmetic of the method.  Shared by the library's training and
the oracle's tests so both start from the same numbers."""

import numpy as np

IN, HID, OUT = 512, 128, 2048
SHAPES = [(IN, HID), (HID,), (HID, HID), (HID,), (HID, OUT), (OUT,)]


def init_params(seed: int = 0, last_scale: float = 0.01) -> np.ndarray:
    """Flat float32 parameters (W1 row-major, b1, W2, b2, W3, b3): weights
    N(0, 2 / fan_in), the last layer's scaled by last_scale so that the
    initial map is close to diag(A)^-1; biases zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i, shp in enumerate(SHAPES):
        if len(shp) == 2:
            w = rng.standard_normal(shp) * np.sqrt(2.0 / shp[0])
            if i == 4:
                w *= last_scale
            parts.append(w.ravel())
        else:
            parts.append(np.zeros(shp[0]))
    return np.concatenate(parts).astype(np.float32)


def batch_order(nsamples: int, batch: int, epochs: int, seed: int = 0):
    """Sample indices per step: a fresh permutation every epoch, cut into
    full batches (the tail of a permutation is dropped)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(epochs):
        perm = rng.permutation(nsamples).astype(np.int32)
        for s in range(0, nsamples - batch + 1, batch):
            yield perm[s:s + batch]
