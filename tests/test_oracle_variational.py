"""Pins of the oracle's variational structure and equilibrium.

* Free-energy decrease (Sec. II, Eqs. model10-model12: dF/dt <= 0 for positive
  mobilities): isothermal, closed, unshifted runs from undercooled and
  supersaturated starts (also with mu_s != mu_l, which exercises the drag) have
  a non-increasing discrete energy.  Planted mistake: the printed reduced drive
  (opposite drag sign, Eq. drivingforce_nonvar) raises the energy over a single
  small step from a state where only the drag term changes sign.
* Equilibrium (supplement Sec. S-I): with uniform equilibrium phase
  concentrations (c_s = k_e c_l = c^eq) at uniform temperature, the discrete
  kink of W^2 lap(phi) = f_dw'(phi) -- solved here independently by Newton's
  method -- is stationary under the full step.
* Interfacial energy gamma = I W H with I = 1/(3 sqrt 2) (Eq. eq34): the
  oracle's discrete energy of the equilibrium kink minus the bulk grand
  potential converges to I W as dx -> 0.
"""
import math

import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I


def _energy_trace(oracle, cs0, dim=1, steps=1500, every=5):
    N = 160
    if dim == 1:
        P = oracle.params(dim=1, n=(N, 1, 1), V=0.0, inv_lT=0.0, z0=N * 0.8 / 2, dt=0.128)
    else:
        P = oracle.params(dim=2, n=(8, N, 1), periodic=(1, 0, 0), V=0.0, inv_lT=0.0, z0=N * 0.8 / 2, dt=0.032)
    phi, cs, cl = I.planar_front(dim, P["n"], 0.8, P["z0"], P["ke"], amp=(2e-2 if dim == 2 else 0.0), seed=5)
    phi, cl = phi.ravel(), cl.ravel()
    cs = np.full_like(phi, cs0)
    E = [oracle.energy(P, phi, cs, cl)]
    n = 0
    for _ in range(steps // every):
        phi, cs, cl, _ = oracle.step(P, phi, cs, cl, every, n0=n)
        n += every
        E.append(oracle.energy(P, phi, cs, cl, n))
    return np.array(E)


@pytest.mark.parametrize("cs0", [0.14, 0.3, 0.05])
def test_energy_decreases_1d(oracle, cs0):
    E = _energy_trace(oracle, cs0)
    assert np.isfinite(E).all()
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert E[-1] < E[0] - 1.0


def test_energy_decreases_2d(oracle):
    E = _energy_trace(oracle, 0.3, dim=2, steps=600, every=20)
    assert np.isfinite(E).all()
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))


def test_printed_drag_sign_raises_energy(oracle):
    """A drag-dominated state: c_l at its equilibrium value c_inf/k_e and
    c_s = 0.05 << k_e c_l, so mu_s - mu_l is large and negative.  The drive
    of Eq. model18 lowers the energy over one small step; the printed reduced
    drive (drag with the opposite sign) raises it."""
    N = 64
    P = oracle.params(dim=1, n=(N, 1, 1), V=0.0, inv_lT=0.0, z0=N * 0.8 / 2, dt=1e-4, A=2.0, b=1.0, Ds=1.0)
    phi, _, _ = I.planar_front(1, (N,), 0.8, P["z0"], P["ke"])
    cl = np.full(N, 1.0 / P["ke"])
    cs = np.full(N, 0.05)
    dE = []
    for variant in (0, 1):
        Pv = dict(P, drag_variant=variant)
        E0 = oracle.energy(Pv, phi, cs, cl)
        phi2, cs2, cl2, _ = oracle.step(Pv, phi, cs, cl, 1)
        dE.append(oracle.energy(Pv, phi2, cs2, cl2, 1) - E0)
    assert dE[0] < -1e-4
    assert dE[1] > 1e-4


def discrete_kink(N, dx, W=1.0, iters=60):
    """Newton solve of W^2 (phi_{i+1} - 2 phi_i + phi_{i-1})/dx^2 = f_dw'(phi_i)
    with mirror ends, started from the tanh profile centred on the middle face."""
    z = (np.arange(N) + 0.5) * dx
    phi = 0.5 * (1.0 - np.tanh((z - N * dx / 2) / (math.sqrt(2.0) * W)))
    c = W * W / dx ** 2
    for _ in range(iters):
        lap = np.empty(N)
        lap[1:-1] = phi[2:] - 2 * phi[1:-1] + phi[:-2]
        lap[0] = phi[1] - phi[0]
        lap[-1] = phi[-2] - phi[-1]
        fp = 2 * phi * (1 - phi) * (1 - 2 * phi)
        r = c * lap - fp
        fpp = 2 * (1 - 6 * phi + 6 * phi * phi)
        J = np.zeros((N, N))
        idx = np.arange(N)
        J[idx, idx] = -2 * c - fpp
        J[0, 0] = -c - fpp[0]
        J[-1, -1] = -c - fpp[-1]
        J[idx[:-1], idx[1:]] = c
        J[idx[1:], idx[:-1]] = c
        dphi = np.linalg.solve(J, -r)
        phi = phi + dphi
        if np.max(np.abs(dphi)) < 1e-16:
            break
    return phi, np.max(np.abs(r))


def test_equilibrium_kink_is_stationary(oracle):
    """A = 1 switches off the (1-A) interface terms: the equilibrium state is
    stationary up to accumulated rounding (~3 ulp per step)."""
    N, dx = 80, 0.8
    phi, res = discrete_kink(N, dx)
    assert res < 1e-14
    P = oracle.params(dim=1, n=(N, 1, 1), V=0.0, inv_lT=0.0, z0=N * dx / 2, dt=0.128, A=1.0)
    ke = P["ke"]
    cs = np.full(N, 1.0)           # c_s^eq = c_inf at T_s
    cl = np.full(N, 1.0 / ke)      # c_l^eq = c_inf / k_e
    phi2, cs2, cl2, _ = oracle.step(P, phi, cs, cl, 2000)
    assert np.max(np.abs(phi2 - phi)) < 1e-14
    assert np.max(np.abs(cs2 - cs)) < 5e-12
    assert np.max(np.abs(cl2 - cl)) < 5e-12 / ke


@pytest.mark.parametrize("A", [0.0, 1.2, 2.0])
def test_equilibrium_phi_rate_vanishes(oracle, A):
    """For any A the phi-equation rate of the equilibrium state is rounding
    (drive zero, uniform c so the cross term vanishes, Allen-Cahn kink)."""
    N, dx = 48, 0.8
    phi, _ = discrete_kink(N, dx)
    P = oracle.params(dim=1, n=(N, 1, 1), V=0.0, inv_lT=0.0, z0=N * dx / 2, A=A)
    pt = oracle.phi_t(P, phi, np.full(N, 1.0), np.full(N, 1.0 / P["ke"]))
    assert np.max(np.abs(pt)) < 1e-14


def test_interfacial_energy_converges(oracle):
    """F_h - lambda (omega L + mu C) -> I W, omega = -1/k_e, mu = -ln k_e."""
    I_exact = 1.0 / (3.0 * math.sqrt(2.0))
    errs = []
    for dx in (0.8, 0.4, 0.2):
        N = int(round(48.0 / dx))
        phi, _ = discrete_kink(N, dx)
        P = oracle.params(dim=1, n=(N, 1, 1), V=0.0, inv_lT=0.0, dx=dx, z0=N * dx / 2)
        ke, lam = P["ke"], P["lambda0"]
        cs = np.full(N, 1.0)
        cl = np.full(N, 1.0 / ke)
        F = oracle.energy(P, phi, cs, cl)
        C, _, _ = oracle.solute(P, phi, cs, cl)
        gamma = F - lam * ((-1.0 / ke) * N * dx + (-math.log(ke)) * C)
        errs.append(abs(gamma - I_exact))
    assert errs[2] < 2e-3 * I_exact
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5
