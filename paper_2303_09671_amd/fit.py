"""Fit of the model constants to a target partition-coefficient curve k*(V).

Sec. V.D selects the source strength A, the mobility-interpolation constant b
(Eq. interpolation1) and the interface width W so that the model's
velocity-dependent partition coefficient follows a measured curve, and notes
that several combinations give the same trapping.  The paper fits the
asymptotic relation (Eq. partition1); here that relation only gives the
starting point (asymptotic_start), and the fit itself is driven by exact
gradients of the simulated k(V): each evaluation runs the checkpointed forward
over the workload's runs (PartitionCoefficient), the adjoint backward gives
dL/dtheta for L = sum_r (k_r - k*_r)^2 with theta = (A, M_phi, W, b), and a
quasi-Newton step (BFGS with a backtracking line search) moves the free
components.  By default these are the paper's (A, b, W); b is optimised as
ln b, since it spans decades (the paper's values range from 1e-5 to 1).
Every step of the forward and backward runs in the HIP library.

A trial theta whose runs leave the explicit scheme's stable range (a
non-finite k, or a time step pf_create rejects) counts as an infinite loss, so
the line search backs off from it.  theta also stays inside a box (A in [0, 3],
M_phi and W in [0.25, 4] in the units of the workload, b in [1e-6, 1]).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import asymptotics, pf
from .adjoint import PartitionCoefficient, Workload

NAMES = ("A", "Mphi", "W", "b")
THETA_LO = np.array([0.0, 0.25, 0.25, 1e-6])
THETA_HI = np.array([3.0, 4.0, 4.0, 1.0])
LOG = np.array([False, False, False, True])  # optimised in log space


@dataclass
class FitResult:
    theta: np.ndarray  # (A, M_phi, W, b)
    loss: float
    evaluations: int
    history: list = field(default_factory=list)  # (theta, loss) of every accepted iterate


def full_theta(workload: Workload, theta) -> np.ndarray:
    """(A, M_phi, W, b): a 3-vector (A, M_phi, W) takes b from the workload."""
    th = np.asarray(theta, dtype=np.float64).ravel()
    if th.size == 3:
        th = np.append(th, workload.params["b"])
    return th


def loss_and_grad(workload: Workload, k_target, theta):
    """L(theta) = sum_r (k_r - k*_r)^2, dL/dtheta (adjoint, for theta =
    (A, M_phi, W, b)) and k.  A theta the library rejects, or whose runs
    become non-finite, gives (inf, None, None)."""
    th = torch.tensor(full_theta(workload, theta), requires_grad=True)
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
    """Starting theta = (A, M_phi, W, b) for fit_theta from Eq. partition1
    (asymptotics.start_theta): the workload's current values with A, or W where
    A has no effect on the asymptotic curve, set to the value whose predicted
    k(V) best fits k_target over the runs' velocities.  Clipped to the box."""
    p = workload.params
    Vs = [r["V"] for r in workload.runs]
    theta, _ = asymptotics.start_theta(Vs, k_target, (p["A"], p["Mphi"], p["W"]), b=p["b"], Ds=p["Ds"],
                                       ke=p["ke"], chi=chi, ap=p.get("ap", 0.0),
                                       quintic=bool(p.get("quintic", 1)))
    return np.clip(np.append(theta, p["b"]), THETA_LO, THETA_HI)


def fit_theta(workload: Workload, k_target, theta0, iters: int = 20, max_step: float = 0.05,
              gtol: float = 1e-12, free=("A", "b", "W"), log=None) -> FitResult:
    """BFGS with Armijo backtracking over the components ``free`` of theta =
    (A, M_phi, W, b) (the others stay at theta0); b moves as ln b.  The first
    step of each line search is limited to max_step in the max norm of the
    optimisation variables.  log: optional callable receiving (iteration,
    theta, loss)."""
    th = np.clip(full_theta(workload, theta0), THETA_LO, THETA_HI)
    idx = np.array([NAMES.index(n) for n in free])
    lo = np.array([np.log(THETA_LO[i]) if LOG[i] else THETA_LO[i] for i in idx])
    hi = np.array([np.log(THETA_HI[i]) if LOG[i] else THETA_HI[i] for i in idx])

    def to_x(t):
        return np.array([np.log(t[i]) if LOG[i] else t[i] for i in idx])

    def to_theta(x):
        t = th.copy()
        t[idx] = np.where(LOG[idx], np.exp(x), x)
        return t

    def grad_x(g, t):  # dL/dx: d/d ln b = b d/db
        return np.where(LOG[idx], g[idx] * t[idx], g[idx])

    x = to_x(th)
    L, g, _ = loss_and_grad(workload, k_target, th)
    if not np.isfinite(L):
        raise ValueError("the starting theta does not give a finite loss")
    gx = grad_x(g, th)
    nev = 1
    n = idx.size
    H = np.eye(n)
    hist = [(th.copy(), L)]
    if log is not None:
        log(0, th, L)
    for it in range(1, iters + 1):
        if np.linalg.norm(gx) <= gtol:
            break
        d = -H @ gx
        if gx @ d >= 0:  # not a descent direction: restart from steepest descent
            H = np.eye(n)
            d = -gx
        t = min(1.0, max_step / np.max(np.abs(d)))
        accepted = False
        for _ in range(12):
            xn = np.clip(x + t * d, lo, hi)
            tn = to_theta(xn)
            Ln, gn, _ = loss_and_grad(workload, k_target, tn)
            nev += 1
            if np.isfinite(Ln) and Ln <= L + 1e-4 * (gx @ (xn - x)):
                accepted = True
                break
            t *= 0.5
        if not accepted:
            break
        gxn = grad_x(gn, tn)
        s, y = xn - x, gxn - gx
        sy = s @ y
        if sy > 1e-300:
            rho = 1.0 / sy
            V = np.eye(n) - rho * np.outer(s, y)
            H = V @ H @ V.T + rho * np.outer(s, s)
        x, th, L, gx = xn, tn, Ln, gxn
        hist.append((th.copy(), L))
        if log is not None:
            log(it, th, L)
    return FitResult(theta=th, loss=L, evaluations=nev, history=hist)
