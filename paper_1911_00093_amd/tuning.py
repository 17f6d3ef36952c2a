"""Persistent cache of the autotuner's launch configurations.

`hmat_autotune` times the launch configurations of a handle on its own data
and keeps the fastest; `hmat_set_tuning` applies a configuration without
timing.  This module remembers the choice: the JSON file named by the
`cache` argument, else by the environment variable HMAT_TUNE_CACHE, maps a
handle's key to the configuration tuned for it.  The key covers what decides
the choice: the device, the library build, the precision options and the
handle's shape (order, block and chunk counts, bytes per stage).  A cached
configuration is applied with `hmat_set_tuning`; results are the same either
way, bit for bit (the tuner changes launch parameters only).
"""

from __future__ import annotations

import hashlib
import json
import os

from . import build, hmat

ENV = "HMAT_TUNE_CACHE"
_CFG = ("stage1_grid", "stage2_grid", "stage2_tile", "stage1_batch", "stage2_batch")


_LIB_ID = None


def _library_id() -> str:
    """sha256 of the loaded library file (first 16 hex digits), once per process."""
    global _LIB_ID
    if _LIB_ID is None:
        h = hashlib.sha256()
        with open(build.LIB, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 22), b""):
                h.update(chunk)
        _LIB_ID = h.hexdigest()[:16]
    return _LIB_ID


def handle_key(H: hmat.HMatrix) -> str:
    import torch

    st = H.stats()
    desc = {
        "device": torch.cuda.get_device_name(H.buf.device),
        "library": _library_id(),
        "options": [H.precision, H.c, H.nrhs_max, H.drop, int(H.dense_split)],
        "shape": [int(st.n), int(st.nblocks), int(st.row_chunks), int(st.column_groups), int(st.stage1_items),
                  int(st.z_len), int(st.stage1_algorithmic_bytes), int(st.stage2_algorithmic_bytes)],
    }
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:24]


def _read(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def autotune(H: hmat.HMatrix, reps: int = 10, cache: str | None = None) -> dict:
    """Tune H (hmat_autotune), or apply its cached configuration.  Returns
    the configuration with "cached": True/False; timings only when tuned."""
    path = cache or os.environ.get(ENV)
    key = handle_key(H) if path else None
    if path:
        hit = _read(path).get(key)
        if hit is not None:
            H.set_tuning(**{k: hit[k] for k in _CFG})
            return dict(hit, cached=True)
    info = H.autotune(reps=reps)
    cfg = {k: info[k] for k in _CFG}
    if path:
        data = _read(path)
        data[key] = cfg
        tmp = f"{path}.tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(info, cached=False)
