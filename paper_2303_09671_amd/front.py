"""Time series of the solidification front (pf_front) while stepping.

The interface temperature and velocity of Sec. V.C / Figs. 8-9 are read from
the phi = 1/2 front: every ``every`` steps the library reports the front
height z (lab frame) and (T_I - T_s)/dT0.  All arithmetic on the fields runs
in the HIP library; this module records those scalars and post-processes the
series: the interface velocity is the centred difference of the recorded
heights in time (a derived diagnostic of the time series, not part of a step).
"""
from __future__ import annotations

import numpy as np

from . import pf


def front_series(h: pf.Handle, nsteps: int, every: int, dt):
    """Step ``h`` by ``nsteps``, reading the front every ``every`` steps (and at
    the start).  ``dt``: the time step (a scalar, or one per run).  Returns a
    dict of arrays shaped (samples, runs): n, t, z, T, and v (dz/dt, centred
    inside, one-sided at the ends; NaN where the front is missing)."""
    n0 = pf.pf_get_step(h)
    ns, zs, Ts = [], [], []
    done = 0
    while True:
        fr = pf.pf_front(h)
        ns.append(n0 + done)
        zs.append(fr["z"])
        Ts.append(fr["T"])
        if done >= nsteps:
            break
        m = min(every, nsteps - done)
        pf.pf_step(h, m)
        done += m
    n = np.asarray(ns, dtype=np.int64)
    t = n[:, None] * np.broadcast_to(np.asarray(dt, dtype=np.float64), (h.nrun,))[None, :]
    z = np.asarray(zs)
    T = np.asarray(Ts)
    v = np.gradient(z, t[:, 0], axis=0) if len(n) > 1 and np.all(t[:, 0] == t[:, -1]) else _grad_runs(z, t)
    return dict(n=n, t=t, z=z, T=T, v=v)


def _grad_runs(z, t):
    v = np.full_like(z, np.nan)
    if len(z) < 2:
        return v
    for r in range(z.shape[1]):
        v[:, r] = np.gradient(z[:, r], t[:, r])
    return v


def oscillation(ser, run: int = 0, t_from: float = 0.0) -> dict:
    """Post-processing of a front series (one run) from time ``t_from`` on:
    range of the interface velocity and temperature, the number of upward
    crossings of the mean velocity and the mean period between them (NaN
    with fewer than two), and the band wavelength V_mean x period."""
    t = ser["t"][:, run]
    sel = t >= t_from
    t, v, T = t[sel], ser["v"][sel, run], ser["T"][sel, run]
    vm = float(np.mean(v))
    d = v - vm
    up = np.nonzero((d[:-1] < 0.0) & (d[1:] >= 0.0))[0]
    period = float(np.mean(np.diff(t[up]))) if len(up) >= 2 else float("nan")
    return dict(v_min=float(v.min()), v_mean=vm, v_max=float(v.max()), T_min=float(T.min()),
                T_mean=float(np.mean(T)), T_max=float(T.max()), crossings=int(len(up)), period=period,
                wavelength=vm * period)


def front_state(ser, run: int, V: float, t_from: float = 0.0, tol: float = 0.02) -> str:
    """Classify a run's front from time ``t_from`` on (post-processing of a
    front series): "steady" when the interface velocity stays within ``tol``
    of the pulling speed V; "oscillating" when it swings by more than that
    around its mean, crosses the mean upwards at least twice and the largest
    deviation from V in the second half of the window is at least half of
    that in the first (a sustained oscillation); "transient" otherwise (a
    slow or damped approach to V, or drift)."""
    o = oscillation(ser, run, t_from)
    if max(abs(o["v_min"] / V - 1.0), abs(o["v_max"] / V - 1.0)) < tol:
        return "steady"
    t = ser["t"][:, run]
    dv = np.abs(ser["v"][t >= t_from, run] - V)
    h = len(dv) // 2
    sustained = h > 0 and dv[h:].max() >= 0.5 * dv[:h].max()
    if o["crossings"] >= 2 and (o["v_max"] - o["v_min"]) > 2.0 * tol * V and sustained:
        return "oscillating"
    return "transient"
