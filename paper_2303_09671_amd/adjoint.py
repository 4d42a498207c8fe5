"""Gradients of the partition coefficient k = c_inf / c_max with respect to
theta = (A, M_phi, W) or (A, M_phi, W, b), through the C ABI's adjoint step
(b is the mobility-interpolation constant of Eq. interpolation1; A, b and W
are the fitting constants of Sec. V.D).

``PartitionCoefficient.apply(theta, workload)`` runs the explicit stepping for
``workload.nsteps`` steps from the workload's initial state (held fixed), saving
a checkpoint every ``workload.every`` steps, and returns k per run (k of
Sec. V.C: 1 / max c with c = p c_s + (1-p) c_l).  Its backward seeds the
adjoint at the final state with dL/dk (pf_kv_seed), then for each checkpoint
segment in reverse replays the segment's states (pf_step_traj) and takes the
adjoint steps backwards over them in one call (pf_adjoint_segment),
accumulating dL/dtheta on the device.  The replay of the next (earlier) segment
runs on a second stream, with its own handle and fields, while the adjoint of
the current one runs on the handle's stream (two trajectory buffers, ordered by
events).  Torch supplies device memory and the streams only.
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
    th = [float(v) for v in theta]
    p["A"], p["Mphi"], p["W"] = th[:3]
    if len(th) > 3:
        p["b"] = th[3]
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
        th = theta.detach().cpu().numpy()
        k, h, fields, ck = forward_k(workload, th, checkpoints=True)
        ctx.workload = workload
        ctx.state = (h, fields, ck, th)
        return k

    @staticmethod
    def backward(ctx, grad_k):
        h, fields, ck, th = ctx.state
        lam = [torch.empty_like(fields[0]) for _ in range(3)]
        pf.pf_kv_seed(h, grad_k.detach().cpu().numpy().astype(np.float64), lam)
        dtheta = _backward_segments(h, ctx.workload, th, fields, ck, lam)
        ctx.state = None
        return dtheta[:len(th)].cpu(), None


class FinalState(torch.autograd.Function):
    """The fields (phi, c_s, c_l) after ``workload.nsteps`` steps as a
    differentiable function of theta, for losses on the interface profile or
    the concentration fields: the backward receives dL/du at the final state
    (computed by torch from any loss on the returned tensors) and runs the same
    checkpointed adjoint as PartitionCoefficient."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, workload: Workload):
        th = theta.detach().cpu().numpy()
        _, h, fields, ck = forward_k(workload, th, checkpoints=True)
        ctx.workload = workload
        ctx.state = (h, fields, ck, th)
        return tuple(f.clone() for f in fields)

    @staticmethod
    def backward(ctx, g_phi, g_cs, g_cl):
        h, fields, ck, th = ctx.state
        lam = [torch.zeros_like(fields[0]) if g is None else g.detach().clone().contiguous()
               for g in (g_phi, g_cs, g_cl)]
        dtheta = _backward_segments(h, ctx.workload, th, fields, ck, lam)
        ctx.state = None
        return dtheta[:len(th)].cpu(), None


def _backward_segments(h, wl: Workload, theta, fields, ck, lam, overlap: bool = True):
    """Replay each checkpoint segment in reverse and take its adjoint steps;
    lam holds the cotangent of the final state on entry.  Returns dL/dtheta
    for theta = (A, M_phi, W, b).
    With ``overlap`` the replays run on a second stream one segment ahead."""
    main = h.stream
    side = torch.cuda.Stream(device=fields[0].device) if overlap else main
    nfield = fields[0].numel()
    K = wl.every
    nseg = len(ck)
    with torch.cuda.stream(main):
        work = [torch.empty_like(fields[0]) for _ in range(3)]
        dtheta = torch.zeros(4, dtype=torch.float64, device=fields[0].device)
        trajs = [[torch.empty((K + 1, nfield), dtype=torch.float64, device=fields[0].device) for _ in range(3)]
                 for _ in range(2)]
        rep_fields = [torch.empty_like(f) for f in fields]
    side.wait_stream(main)  # checkpoints, buffers and the seed are ready
    h_rep = pf.pf_create(_params_with(wl, theta), *rep_fields, stream=side, runs=wl.runs, offsets=wl.offsets)
    free = [None, None]  # per buffer: event after the adjoint that last read it

    def replay(s):
        n0 = s * K
        m = min(K, wl.nsteps - n0)
        buf = trajs[s % 2]
        with torch.cuda.stream(side):
            if free[s % 2] is not None:
                side.wait_event(free[s % 2])
            for f, c in zip(rep_fields, ck[s]):
                f.copy_(c)
            pf.pf_set_step(h_rep, n0)
            pf.pf_step_traj(h_rep, m, buf)
            ev = torch.cuda.Event()
            ev.record(side)
        return ev

    ready = replay(nseg - 1)
    for s in reversed(range(nseg)):
        n0 = s * K
        m = min(K, wl.nsteps - n0)
        main.wait_event(ready)
        if s > 0:
            ready = replay(s - 1)  # overlaps the adjoint of segment s
        pf.pf_adjoint_segment(h, n0, m, trajs[s % 2], lam, work, dtheta)
        ev = torch.cuda.Event()
        ev.record(main)
        free[s % 2] = ev
    main.wait_stream(side)
    main.synchronize()  # the buffers above are released on return
    pf.pf_destroy(h_rep)
    return dtheta


def adjoint_only_seconds(workload: Workload, theta, overlap: bool = True) -> float:
    """Wall time of the backward pass alone (replay + adjoint) for timing."""
    import time
    k, h, fields, ck = forward_k(workload, theta, checkpoints=True)
    lam = [torch.zeros_like(fields[0]) for _ in range(3)]
    pf.pf_kv_seed(h, np.ones(workload.nrun), lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _backward_segments(h, workload, theta, fields, ck, lam, overlap=overlap)
    torch.cuda.synchronize()
    return time.perf_counter() - t0
