"""Gradients of the partition coefficient k = c_inf / c_max with respect to
theta = (A, M_phi, W), through the C ABI's adjoint step.

``PartitionCoefficient.apply(theta, workload)`` runs the explicit stepping for
``workload.nsteps`` steps from the workload's initial state (held fixed), saving
a checkpoint every ``workload.every`` steps, and returns k per run (k of
Sec. V.C: 1 / max c with c = p c_s + (1-p) c_l).  Its backward seeds the
adjoint at the final state with dL/dk (pf_kv_seed), then for each checkpoint
segment in reverse replays the segment's states (pf_step_traj) and takes the
adjoint steps backwards over them in one call (pf_adjoint_segment),
accumulating dL/dtheta on the device.  Torch supplies device memory and the
stream only.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import pf


@dataclass
class Workload:
    """Initial state and parameters of a run set (batched 1D runs or one 2D grid)."""
    params: dict
    fields0: tuple  # host float64 arrays (phi, c_s, c_l)
    nsteps: int
    every: int = 100
    runs: list | None = None
    offsets: np.ndarray | None = None
    handles: list = field(default_factory=list)

    @property
    def nrun(self) -> int:
        return len(self.runs) if self.runs is not None else 1


def _params_with(workload: Workload, theta) -> dict:
    p = dict(workload.params)
    p["A"], p["Mphi"], p["W"] = (float(v) for v in theta)
    return p


def _open(workload: Workload, theta):
    fields = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda() for a in workload.fields0]
    h = pf.pf_create(_params_with(workload, theta), *fields, runs=workload.runs, offsets=workload.offsets)
    return h, fields


def forward_k(workload: Workload, theta, checkpoints: bool = False):
    """k per run after nsteps; optionally the checkpoint list (device tensors)."""
    h, fields = _open(workload, theta)
    ck = []
    done = 0
    while done < workload.nsteps:
        if checkpoints:
            ck.append([f.clone() for f in fields])
        m = min(workload.every, workload.nsteps - done)
        pf.pf_step(h, m)
        done += m
    _, cmax, _ = pf.pf_solute(h)
    k = torch.from_numpy(1.0 / cmax)
    return k, h, fields, ck


class PartitionCoefficient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, workload: Workload):
        k, h, fields, ck = forward_k(workload, theta.detach().cpu().numpy(), checkpoints=True)
        ctx.workload = workload
        ctx.state = (h, fields, ck)
        return k

    @staticmethod
    def backward(ctx, grad_k):
        h, fields, ck = ctx.state
        wl = ctx.workload
        lam = [torch.empty_like(fields[0]) for _ in range(3)]
        pf.pf_kv_seed(h, grad_k.detach().cpu().numpy().astype(np.float64), lam)
        dtheta = _backward_segments(h, wl, fields, ck, lam)
        ctx.state = None
        return dtheta.cpu(), None


def _backward_segments(h, wl: Workload, fields, ck, lam):
    """Replay each checkpoint segment in reverse and take its adjoint steps;
    lam holds the cotangent of the final state on entry.  Returns dL/dtheta."""
    nfield = fields[0].numel()
    work = [torch.empty_like(fields[0]) for _ in range(3)]
    dtheta = torch.zeros(3, dtype=torch.float64, device=fields[0].device)
    K = wl.every
    traj = [torch.empty((K + 1, nfield), dtype=torch.float64, device=fields[0].device) for _ in range(3)]
    for s in reversed(range(len(ck))):
        n0 = s * K
        m = min(K, wl.nsteps - n0)
        for f, c in zip(fields, ck[s]):
            f.copy_(c)
        pf.pf_set_step(h, n0)
        pf.pf_step_traj(h, m, traj)
        pf.pf_adjoint_segment(h, n0, m, traj, lam, work, dtheta)
    return dtheta


def adjoint_only_seconds(workload: Workload, theta, nsteps: int | None = None) -> float:
    """Wall time of the backward pass alone (replay + adjoint) for timing."""
    import time
    k, h, fields, ck = forward_k(workload, theta, checkpoints=True)
    lam = [torch.zeros_like(fields[0]) for _ in range(3)]
    pf.pf_kv_seed(h, np.ones(workload.nrun), lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _backward_segments(h, workload, fields, ck, lam)
    torch.cuda.synchronize()
    return time.perf_counter() - t0
