"""Pins of the oracle's equal-potential model (model = 1: mu_s = mu_l imposed,
the model of the asymptotic analysis, Sec. II.C; KKS for A = 1, Sec. IV).

* The split: after every step c_s = k_e c_l (Eq. dil1 with mu_s = mu_l).
* The mixture c = p c_s + (1-p) c_l is updated in conservative form, so closed
  unshifted two-phase runs conserve the total solute to rounding in 1D and 2D.
  (The separate-kinetics model only converges to conservation.)
* Bulk phases diffuse as the textbook FTCS scheme: a cosine mode decays by
  1 - 4 D dt/dx^2 sin^2(k dx/2) per step with D = 1 in the liquid and D_s in
  the solid.
* KKS reduction: with A = 1 and b = k_e D_s/D_l, one step equals a plain
  staggered discretisation of Eqs. KKS1 and KKS2.  That step is written out
  here from the free energies, and uses q = M_s p + M_l (1-p) and
  grad mu_l = grad ln c_l.
* Equilibrium: the discrete kink with c_l = c_l^eq, c_s = k_e c_l^eq is stationary.
* Variational structure: for A = 1 (KKS) and A = 0 (the non-diagonal model of
  Ohno et al.) the discrete free energy does not increase.
* Trapping control: steady fronts with A = 1.2 trap more than with A = 0.5.
  The asymptotic relation of Eq. partition1 predicts the same ordering, with
  the model's own mobility ratio M_s/M_l = k_e D_s/D_l.  The two agree within
  20 %.  A sign slip or a dropped anti-trapping term in the mixture flux would
  reverse or remove the ordering.
"""
import math

import numpy as np
import pytest

from paper_2303_09671_amd import asymptotics as asy
from paper_2303_09671_amd import inputs as I
from tests.test_oracle_transport import _mode
from tests.test_oracle_variational import discrete_kink


def _front(oracle, N=160, **kw):
    P = oracle.params(dim=1, n=(N, 1, 1), model=1, **kw)
    phi, cs, cl = I.planar_front(1, (N,), P["dx"], P["z0"], P["ke"])
    return P, phi, cs, cl


def test_split_holds_after_every_step(oracle):
    P, phi, cs, cl = _front(oracle, N=300, z0=75 * 0.8, V=0.3, dt=0.06, A=1.2, eps_grad=1e-4)
    s = 0
    for n0 in range(0, 600, 200):
        phi, cs, cl, s = oracle.step(P, phi, cs, cl, 200, n0=n0, shift=s)
        assert np.max(np.abs(cs - P["ke"] * cl) / cl) < 1e-15
    assert s > 0  # the window moved


@pytest.mark.parametrize("dim", [1, 2])
def test_two_phase_conservation_exact(oracle, dim):
    if dim == 1:
        P = oracle.params(dim=1, n=(120, 1, 1), model=1, V=0.0, inv_lT=0.0, z0=48.0, dt=0.05, A=1.3,
                          eps_grad=1e-4)
    else:
        P = oracle.params(dim=2, n=(10, 60, 1), periodic=(1, 0, 0), model=1, V=0.0, inv_lT=0.0, z0=24.0,
                          dt=0.02, A=0.7, eps_grad=1e-4)
    phi, cs, cl = I.planar_front(dim, P["n"], P["dx"], P["z0"], P["ke"], amp=0.05 if dim == 2 else 0.0, seed=9)
    phi, cs, cl = (a.ravel() for a in (phi, cs, cl))
    cl = cl * (1.3 + 0.1 * np.sin(np.arange(cl.size)))  # supersaturated, non-uniform
    cs = P["ke"] * cl
    t0, _, _ = oracle.solute(P, phi, cs, cl)
    phi2, cs2, cl2, _ = oracle.step(P, phi, cs, cl, 400)
    t1, _, _ = oracle.solute(P, phi2, cs2, cl2)
    assert np.max(np.abs(phi2 - phi)) > 1e-3  # the front moved
    assert abs(t1 - t0) < 1e-13 * abs(t0)


@pytest.mark.parametrize("phase", [0.0, 1.0])
def test_bulk_ftcs_amplification(oracle, phase):
    n, per, m = (12, 10, 1), (1, 0, 0), (2, 3)
    dx, dt, Ds = 0.8, 0.05, 0.3
    P = oracle.params(dim=2, n=n, periodic=per, dx=dx, dt=dt, Ds=Ds, V=0.0, inv_lT=0.0, A=1.7, model=1)
    mode, ks = _mode(2, n, dx, per, m)
    phi = np.full(mode.size, phase)
    cl = 1.0 + 1e-3 * mode
    cs = P["ke"] * cl
    steps = 7
    phi2, cs2, cl2, _ = oracle.step(P, phi, cs, cl, steps)
    D = 1.0 if phase == 0.0 else Ds
    lam = 1.0 - sum(4 * D * dt / dx ** 2 * math.sin(k * dx / 2) ** 2 for k in ks)
    assert np.max(np.abs(cl2 - (1.0 + 1e-3 * lam ** steps * mode))) < 1e-14 / (P["ke"] if phase else 1.0)
    assert np.array_equal(phi2, phi)


def _kks_step(P, phi, cs, cl):
    """One explicit step of Eqs. KKS1, KKS2 (1D, mirror ends, isothermal), plain."""
    ke, dx, dt, W, lam = P["ke"], P["dx"], P["dt"], P["W"], P["lambda0"] * P["W"]
    alpha = P["W"] / P["Mphi"]
    h = lambda f: f ** 3 * (6 * f * f - 15 * f + 10)
    dh = lambda f: 30 * (f * (1 - f)) ** 2
    cleq = 1.0 / ke  # T = T_s everywhere
    fs = cs * np.log(cs) - cs - cs * math.log(ke) + (ke - 1.0) * cleq
    fl = cl * np.log(cl) - cl
    mu = np.log(cl)                                    # mu_l, equal to mu_s
    ext = lambda u: np.concatenate([[u[0]], u, [u[-1]]])
    pe = ext(phi)
    lap = (pe[2:] - 2 * phi + pe[:-2]) / dx ** 2
    fdw = 2 * phi * (1 - phi) * (1 - 2 * phi)
    phit = (W * W * lap - fdw - lam * (fs - fl - mu * (cs - cl)) * dh(phi)) / alpha  # Eq. KKS1
    pf = h(0.5 * (phi[1:] + phi[:-1]))
    q = P["Ds"] * 0.5 * (cs[1:] + cs[:-1]) * pf + 0.5 * (cl[1:] + cl[:-1]) * (1 - pf)
    J = np.concatenate([[0.0], q * (mu[1:] - mu[:-1]) / dx, [0.0]])               # Eq. KKS2
    c = h(phi) * cs + (1 - h(phi)) * cl + dt * (J[1:] - J[:-1]) / dx
    phi2 = phi + dt * phit
    cl2 = c / (ke * h(phi2) + 1 - h(phi2))
    return phi2, ke * cl2, cl2


def test_kks_reduction(oracle):
    N = 40
    ke, Ds = 0.3, 0.05
    P = oracle.params(dim=1, n=(N, 1, 1), model=1, A=1.0, ke=ke, Ds=Ds, b=ke * Ds, V=0.0, inv_lT=0.0,
                      z0=16.0, dt=0.01, lambda0=0.2, eps_grad=1e-20)
    z = (np.arange(N) + 0.5) * P["dx"]
    phi = 1.0 / (1.0 + np.exp(math.sqrt(2.0) * (z - 16.0) / 1.3))  # every |grad phi| well above eps
    cl = 1.0 / ke * (1.0 + 0.2 * np.sin(0.37 * np.arange(N)))
    cs = ke * cl
    ref = _kks_step(P, phi, cs, cl)
    out = oracle.step(P, phi, cs, cl, 1)
    for a, b in zip(out[:3], ref):
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    # the step is not trivial
    assert np.max(np.abs(out[2] - cl)) > 1e-3 and np.max(np.abs(out[0] - phi)) > 1e-4


@pytest.mark.parametrize("A", [1.0, 0.0, 1.7])
def test_equilibrium_kink_is_stationary(oracle, A):
    N, dx = 80, 0.8
    phi, res = discrete_kink(N, dx)
    assert res < 1e-14
    P = oracle.params(dim=1, n=(N, 1, 1), model=1, V=0.0, inv_lT=0.0, z0=N * dx / 2, dt=0.128, A=A)
    ke = P["ke"]
    cl = np.full(N, 1.0 / ke)
    cs = ke * cl
    phi2, cs2, cl2, _ = oracle.step(P, phi, cs, cl, 1000)
    assert np.max(np.abs(phi2 - phi)) < 1e-13
    assert np.max(np.abs(cl2 - cl)) < 1e-11 / ke


@pytest.mark.parametrize("A", [1.0, 0.0])
def test_energy_decreases(oracle, A):
    N = 160
    P = oracle.params(dim=1, n=(N, 1, 1), model=1, V=0.0, inv_lT=0.0, z0=N * 0.8 / 2, dt=0.1, A=A,
                      eps_grad=1e-4)
    phi, _, _ = I.planar_front(1, (N,), 0.8, P["z0"], P["ke"])
    cl = np.full(N, 1.2)  # below c_l^eq = 1/k_e: the solid grows, solute is rejected
    cs = P["ke"] * cl
    E = [oracle.energy(P, phi, cs, cl)]
    n = 0
    for _ in range(200):
        phi, cs, cl, _ = oracle.step(P, phi, cs, cl, 5, n0=n)
        n += 5
        E.append(oracle.energy(P, phi, cs, cl, n))
    E = np.array(E)
    assert np.isfinite(E).all()
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert E[-1] < E[0] - 0.1


def _steady_k(oracle, A, V, N=512, steps=20000):
    ke, Ds, b = 0.3, 1e-3, 1e-3
    P = oracle.params(dim=1, n=(N, 1, 1), model=1, ke=ke, Ds=Ds, b=b, A=A, V=V, dt=0.06, eps_grad=1e-4,
                      lambda0=asy.I_DW * ke / (1 - ke) ** 2, z0=(N // 4) * 0.8)
    f = I.planar_front(1, (N,), 0.8, P["z0"], ke)
    phi, cs, cl, _ = oracle.step(P, *f, steps)
    return 1.0 / oracle.solute(P, phi, cs, cl)[1]


def test_trapping_follows_A_as_partition1_predicts(oracle):
    V = 0.5
    k_lo, k_hi = _steady_k(oracle, 0.5, V), _steady_k(oracle, 1.2, V)
    p_lo = asy.kv_curve([V], 0.5, 1e-3, 0.3 * 1e-3, 0.3)[0][0]
    p_hi = asy.kv_curve([V], 1.2, 1e-3, 0.3 * 1e-3, 0.3)[0][0]
    assert p_hi - p_lo > 0.05 and k_hi - k_lo > 0.03
    assert abs(k_lo / p_lo - 1) < 0.2 and abs(k_hi / p_hi - 1) < 0.2
