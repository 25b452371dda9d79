"""Checkpoints of the ordering network's training: the fp32 parameters, Adam's
moments and step count, and the hyper-parameters, in one .npz file (plain arrays,
no pickled objects).  The bfloat16 operands the intersection kernel uses are not
stored: ccs_scene_set_policy derives them from the fp32 parameters.
"""
from __future__ import annotations

import json
import os

import numpy as np

FORMAT = "ccs-policy-checkpoint-1"
N_PARAMS = 1732


def _host(x) -> np.ndarray:
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).reshape(-1)
    if a.size != N_PARAMS:
        raise ValueError(f"expected {N_PARAMS} values, got {a.size}")
    return a


def save(path: str, params, m=None, v=None, t: int = 0, hyper: dict | None = None) -> None:
    """Writes params (and Adam's m, v after t steps) to path, atomically (a
    temporary file in the same folder, then a rename)."""
    p = _host(params)
    m = np.zeros(N_PARAMS, np.float32) if m is None else _host(m)
    v = np.zeros(N_PARAMS, np.float32) if v is None else _host(v)
    if t < 0:
        raise ValueError("step count must be >= 0")
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "wb") as fh:
        np.savez(fh, format=np.array(FORMAT), params=p, adam_m=m, adam_v=v, adam_t=np.array(t, np.uint64),
                 hyper=np.array(json.dumps(hyper or {}, sort_keys=True)))
    os.replace(tmp, path)


def load(path: str) -> dict:
    """{params, adam_m, adam_v (float32 arrays), adam_t (int), hyper (dict)} from a file save() wrote."""
    with np.load(path, allow_pickle=False) as z:
        if str(z["format"]) != FORMAT:
            raise ValueError(f"{path}: not a {FORMAT} file")
        out = {k: np.array(z[k], dtype=np.float32) for k in ("params", "adam_m", "adam_v")}
        for k, a in out.items():
            if a.shape != (N_PARAMS,):
                raise ValueError(f"{path}: {k} has shape {a.shape}")
            if not np.isfinite(a).all():
                raise ValueError(f"{path}: {k} holds non-finite values")
        out["adam_t"] = int(z["adam_t"])
        out["hyper"] = json.loads(str(z["hyper"]))
    return out


def save_training(path: str, params, adam, hyper: dict | None = None) -> None:
    """save() of CUDA params and a ccs.Adam."""
    save(path, params, adam.m, adam.v, adam.t, hyper)


def load_training(path: str, device="cuda"):
    """(params, ccs.Adam, hyper) on device from a file save() wrote."""
    import torch

    from . import ccs
    c = load(path)
    params = torch.from_numpy(c["params"]).to(device)
    adam = ccs.Adam(device, torch.from_numpy(c["adam_m"]).to(device), torch.from_numpy(c["adam_v"]).to(device),
                    c["adam_t"])
    return params, adam, c["hyper"]
