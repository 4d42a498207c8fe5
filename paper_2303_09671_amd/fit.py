"""Fit of theta = (A, M_phi, W) to a target partition-coefficient curve k*(V).

Sec. V.C tunes the source strength A, the shape parameter b and the interface
width W so that the model's velocity-dependent partition coefficient follows a
measured or simulated curve, and notes that several combinations give the same
trapping.  The paper fits the asymptotic relation (Eq. partition1); here that
relation only gives the starting point (asymptotic_start), and the fit itself
is driven by exact gradients of the simulated k(V): each evaluation runs the checkpointed
forward over the workload's runs (PartitionCoefficient), the adjoint backward
gives dL/dtheta for L = sum_r (k_r - k*_r)^2, and a quasi-Newton step (BFGS
with a backtracking line search) moves theta.  Every step of the forward and
backward runs in the HIP library.

A trial theta whose runs leave the explicit scheme's stable range (a
non-finite k, or a time step pf_create rejects) counts as an infinite loss, so
the line search backs off from it.  theta also stays inside a box (A in [0, 3],
M_phi and W in [0.25, 4] in the units of the workload).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import asymptotics, pf
from .adjoint import PartitionCoefficient, Workload

THETA_LO = np.array([0.0, 0.25, 0.25])
THETA_HI = np.array([3.0, 4.0, 4.0])


@dataclass
class FitResult:
    theta: np.ndarray
    loss: float
    evaluations: int
    history: list = field(default_factory=list)  # (theta, loss) of every accepted iterate


def loss_and_grad(workload: Workload, k_target, theta):
    """L(theta) = sum_r (k_r - k*_r)^2, dL/dtheta (adjoint) and k.  A theta the
    library rejects, or whose runs become non-finite, gives (inf, None, None)."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
    kt = torch.as_tensor(np.asarray(k_target, dtype=np.float64))
    try:
        k = PartitionCoefficient.apply(th, workload)
    except pf.PFError:
        return np.inf, None, None
    if not torch.isfinite(k).all():
        return np.inf, None, None
    L = ((k - kt) ** 2).sum()
    L.backward()
    g = th.grad.numpy().copy()
    if not np.all(np.isfinite(g)):
        return np.inf, None, None
    return float(L.item()), g, k.detach().numpy()


def asymptotic_start(workload: Workload, k_target, chi: float = 1.0):
    """Starting theta for fit_theta from Eq. partition1 (asymptotics.start_theta):
    the workload's current (A, M_phi, W) with A, or W where A has no effect on
    the asymptotic curve, set to the value whose predicted k(V) best fits
    k_target over the runs' velocities.  The result is clipped to the box."""
    p = workload.params
    Vs = [r["V"] for r in workload.runs]
    theta, _ = asymptotics.start_theta(Vs, k_target, (p["A"], p["Mphi"], p["W"]), b=p["b"], Ds=p["Ds"],
                                       ke=p["ke"], chi=chi, ap=p.get("ap", 0.0),
                                       quintic=bool(p.get("quintic", 1)))
    return np.clip(theta, THETA_LO, THETA_HI)


def fit_theta(workload: Workload, k_target, theta0, iters: int = 20, max_step: float = 0.05,
              gtol: float = 1e-12, log=None) -> FitResult:
    """BFGS with Armijo backtracking; the first step of each line search is
    limited to max_step in the max norm.  log: optional callable receiving
    (iteration, theta, loss)."""
    th = np.clip(np.asarray(theta0, dtype=np.float64), THETA_LO, THETA_HI)
    L, g, _ = loss_and_grad(workload, k_target, th)
    if not np.isfinite(L):
        raise ValueError("the starting theta does not give a finite loss")
    nev = 1
    H = np.eye(3)
    hist = [(th.copy(), L)]
    if log is not None:
        log(0, th, L)
    for it in range(1, iters + 1):
        if np.linalg.norm(g) <= gtol:
            break
        d = -H @ g
        if g @ d >= 0:  # not a descent direction: restart from steepest descent
            H = np.eye(3)
            d = -g
        t = min(1.0, max_step / np.max(np.abs(d)))
        accepted = False
        for _ in range(12):
            tn = np.clip(th + t * d, THETA_LO, THETA_HI)
            Ln, gn, _ = loss_and_grad(workload, k_target, tn)
            nev += 1
            if np.isfinite(Ln) and Ln <= L + 1e-4 * (g @ (tn - th)):
                accepted = True
                break
            t *= 0.5
        if not accepted:
            break
        s, y = tn - th, gn - g
        sy = s @ y
        if sy > 1e-300:
            rho = 1.0 / sy
            V = np.eye(3) - rho * np.outer(s, y)
            H = V @ H @ V.T + rho * np.outer(s, s)
        th, L, g = tn, Ln, gn
        hist.append((th.copy(), L))
        if log is not None:
            log(it, th, L)
    return FitResult(theta=th, loss=L, evaluations=nev, history=hist)
