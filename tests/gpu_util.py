"""Helpers for the GPU tests: device copies and the error metric."""
from __future__ import annotations

import numpy as np


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def normwise(x, ref):
    """max over components |x - ref| / max over components |ref|, per
    (save, trajectory); x and ref are [n_save][n][N]."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.max(np.abs(x - ref), axis=1) / np.max(np.abs(ref), axis=1)


def banner(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
