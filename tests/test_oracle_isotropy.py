"""Isotropy pin of the oracle's 2D operators (transverse face gradients).

The equations of motion (Sec. II) contain no preferred direction, so for fields
that depend on position only through the normal coordinate
zeta = (z - z_c) cos(theta) - (x - x_c) sin(theta) of a tilted planar
interface, the right-hand sides are those of the 1D equations along zeta.
The scheme is second-order accurate in space (Sec. V.A: all spatial
derivatives to second order), so one explicit step of the 2D oracle on such a
tilted state must approach the 1D right-hand side, evaluated on a grid 16x
finer, as O(dx^2): halving dx from 0.2 W to 0.1 W must cut the discrepancy about
4x (measured: orders 2.00, 1.99, 1.97 for phi, c_s, c_l).  A
transverse face gradient taken from one of the two cells only is first order
(planted mistake ``mutate = 5``) and fails the rate (measured order 1.07 for c_s).
"""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

L = 16.0  # box edge, in W
THETA = np.deg2rad(30.0)
KEEP = 6  # cells next to the mirror boundaries left out (dependency radius of a step: 3)


def _profiles(zeta, ke):
    phi = 1.0 / (1.0 + np.exp(np.sqrt(2.0) * zeta))
    cs = ke * (1.0 + 0.3 * np.tanh(zeta / 3.0))
    cl = 1.0 + 0.25 * np.exp(-zeta * zeta / 20.0) + 0.1 * np.tanh(zeta / 4.0)
    return phi, cs, cl


def _base(oracle, **kw):
    p = dict(V=0.0, inv_lT=0.0, A=2.0, b=1e-2, Ds=0.05, lambda0=0.3, ke=0.14, eps_grad=1e-20, dt=1.0, W=1.0,
             Mphi=1.0)
    p.update(kw)
    return p


def _rhs_2d(oracle, dx, **kw):
    n = int(round(L / dx))
    p = oracle.params(**_base(oracle, dim=2, n=(n, n, 1), periodic=(0, 0, 0), dx=dx, **kw))
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)  # [z][x]
    zeta = (Z - L / 2) * np.cos(THETA) - (X - L / 2) * np.sin(THETA)
    u0 = [a.ravel() for a in _profiles(zeta, p["ke"])]
    u1 = oracle.step(p, *u0, 1)[:3]  # dt = 1: u1 - u0 is the right-hand side
    rhs = [(b - a).reshape(n, n) for a, b in zip(u0, u1)]
    inner = (slice(KEEP, n - KEEP), slice(KEEP, n - KEEP))
    return [r[inner] for r in rhs], zeta[inner]


def _rhs_1d_fine(oracle, h, zmin, zmax, **kw):
    m = int(np.ceil((zmax - zmin) / h)) + 40
    p = oracle.params(**_base(oracle, dim=1, n=(m, 1, 1), dx=h, **kw))
    z = zmin - 20 * h + (np.arange(m) + 0.5) * h
    u0 = list(_profiles(z, p["ke"]))
    u1 = oracle.step(p, *u0, 1)[:3]
    return z, [b - a for a, b in zip(u0, u1)]


def _errors(oracle, dx, **kw):
    rhs2, zeta = _rhs_2d(oracle, dx, **kw)
    z, rhs1 = _rhs_1d_fine(oracle, dx / 16.0, zeta.min() - 1.0, zeta.max() + 1.0, **kw)
    errs = []
    for r2, r1 in zip(rhs2, rhs1):
        ref = CubicSpline(z, r1)(zeta)
        errs.append(float(np.max(np.abs(r2 - ref)) / np.max(np.abs(ref))))
    return np.array(errs)


def _orders(oracle, **kw):
    e1 = _errors(oracle, 0.2, **kw)
    e2 = _errors(oracle, 0.1, **kw)
    return e1, e2, np.log2(e1 / e2)


def test_tilted_front_converges_at_second_order(oracle):
    e1, e2, order = _orders(oracle)
    assert np.all(e2 < 1e-2), f"2D vs 1D discrepancy at dx = 0.1: {e2}"
    assert np.all(order > 1.8), f"convergence orders (phi, c_s, c_l): {order}, errors {e1} -> {e2}"


def test_planted_one_sided_transverse_gradient_fails(oracle):
    e1, e2, order = _orders(oracle, mutate=5)
    assert np.min(order) < 1.4, f"mutate=5 still converges at orders {order}"
