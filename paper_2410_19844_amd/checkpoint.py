"""Checkpoint and resume of a solve: the factor W, the optimiser state
(Adam moments and the best W the library keeps) and the step count, with the
problem's shape, in one ``.npz`` file.

The file holds plain arrays only (no pickled objects) and is read back with
``numpy.load(..., allow_pickle=False)``.  Device buffers are copied to the
host as raw bytes, so a resumed run continues from bitwise the same values:
on the grouped (serving) path, whose sums run in a fixed order, the next step
after a resume matches the uninterrupted run bit for bit.
"""
from __future__ import annotations

import numpy as np
import torch

from . import PRECISIONS, Plan

__all__ = ["save", "load"]

_FORMAT = 1


def save(path: str, plan: Plan, W: torch.Tensor, state: torch.Tensor, t: int) -> None:
    """Write W (plan.wdtype, N x rank), the state bytes and t (steps taken)."""
    plan._w(W)
    if state.dtype != torch.uint8 or state.numel() < plan.state_bytes:
        raise ValueError(f"state must be a uint8 tensor of at least {plan.state_bytes} bytes")
    prec = next(k for k, v in PRECISIONS.items() if v == plan.prec)
    np.savez(path, format=np.int64(_FORMAT),
             shape=np.array([plan.n, plan.d, plan.rank], dtype=np.int64),
             precision=np.array(prec), t=np.int64(t),
             W=W.detach().cpu().contiguous().view(torch.uint8).numpy(),
             state=state[: plan.state_bytes].detach().cpu().numpy())


def load(path: str, plan: Plan, device=None):
    """Read a checkpoint for ``plan``; returns (W, state, t) on the device.

    The file must have been written for the same (n, d, rank) and precision."""
    with np.load(path, allow_pickle=False) as f:
        if int(f["format"]) != _FORMAT:
            raise ValueError(f"{path}: unknown checkpoint format {int(f['format'])}")
        n, d, rank = (int(x) for x in f["shape"])
        prec = str(f["precision"])
        if (n, d, rank) != (plan.n, plan.d, plan.rank) or PRECISIONS.get(prec) != plan.prec:
            raise ValueError(f"{path}: checkpoint of ({n}, {d}, {rank}, {prec}) does not match the plan")
        dev = plan.device if device is None else device
        Wb = torch.from_numpy(f["W"].copy())
        W = Wb.view(plan.wdtype).reshape(plan.N, plan.rank).to(dev)
        state = torch.zeros(plan.state_bytes, dtype=torch.uint8, device=dev)
        state.copy_(torch.from_numpy(f["state"].copy()).to(dev))
        return W, state, int(f["t"])
