"""Helpers for the GPU parity tests (device transfer and error norms)."""
from __future__ import annotations

import numpy as np
import torch

DEV = torch.device("cuda:0")


def to_dev(fields, dtype=torch.float64):
    return [torch.from_numpy(np.ascontiguousarray(f)).to(device=DEV, dtype=dtype) for f in fields]


def to_host(tensors):
    torch.cuda.synchronize()
    return [t.detach().cpu().numpy().astype(np.float64) for t in tensors]


def rel_l2(got, exp):
    num = np.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in zip(got, exp)))
    den = np.sqrt(sum(float(np.sum(b ** 2)) for b in exp))
    return num / den


def max_rel(got, exp):
    scale = max(float(np.abs(b).max()) for b in exp)
    return max(float(np.abs(a - b).max()) for a, b in zip(got, exp)) / scale
