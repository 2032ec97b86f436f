"""Weights of the learned preconditioner: layout, initialisation, storage.

The network (3-level 3-D U-Net, 16/32/64 channels, 3x3x3 bias-free
convolutions) runs in the HIP library; this module only handles the float32
weight blob that sim_net_set_weights / sim_net_train_step take: the 11
convolutions in order, each in PyTorch Conv3d layout [c_out][c_in][kz][ky][kx].
"""
from __future__ import annotations

import os

import numpy as np

CONVS = [(2, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
         (48, 16), (16, 16), (16, 1)]
NAMES = [f"c{q + 1}" for q in range(len(CONVS))]


def param_count() -> int:
    return sum(27 * a * b for a, b in CONVS)


def init_weights(seed: int = 0, out_scale: float = 0.1) -> np.ndarray:
    """He-normal initialisation (std sqrt(2 / (27 c_in))); the output layer
    is scaled by out_scale so the first corrections are small."""
    rng = np.random.default_rng([seed, 7])
    parts = []
    for q, (cin, cout) in enumerate(CONVS):
        std = np.sqrt(2.0 / (27 * cin)) * (out_scale if q == len(CONVS) - 1 else 1.0)
        parts.append(rng.standard_normal(27 * cin * cout) * std)
    return np.concatenate(parts).astype(np.float32)


def to_dict(blob: np.ndarray) -> dict:
    out, off = {}, 0
    for name, (cin, cout) in zip(NAMES, CONVS):
        m = 27 * cin * cout
        out[name] = np.ascontiguousarray(blob[off:off + m].reshape(cout, cin, 3, 3, 3))
        off += m
    return out


def from_dict(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float32).reshape(-1) for name in NAMES])


def save_weights(path: str, blob: np.ndarray, meta: dict | None = None) -> None:
    from safetensors.numpy import save_file
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    save_file(to_dict(np.asarray(blob, np.float32)), path,
              metadata={k: str(v) for k, v in (meta or {}).items()})


def load_weights(path: str, device=None):
    """Float32 blob from a safetensors file; a torch tensor on `device` when
    given, else a numpy array."""
    from safetensors.numpy import load_file
    blob = from_dict(load_file(path))
    if device is None:
        return blob
    import torch
    return torch.as_tensor(blob, device=device)
