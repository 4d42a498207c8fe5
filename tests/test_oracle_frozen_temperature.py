"""Pin of the oracle's frozen temperature field (Sec. III, directional
solidification, Eq. ds1) and of the lab coordinate of the moving window.

Physical content: the temperature is T(z, t) = T_s + G (z - z0 - V t) in the
lab frame (the isotherms move towards the liquid at the pulling speed; T_s,
the solidus of c_inf, sits at the initial front z0), and the liquidus of the
linearised phase diagram gives the equilibrium liquid concentration at T
(Eq. dil7).  So at any time:

* a solid/liquid pair in equilibrium at the solidus of c_inf (c_s = c_inf,
  c_l = c_inf / k_e) has zero driving force exactly on the T_s isotherm,
  z = z0 + V t: colder cells below it solidify, hotter cells above it melt;
* the pair in equilibrium at the liquidus of c_inf (c_s = k_e c_inf,
  c_l = c_inf) has zero driving force on the T_l isotherm, which lies the
  freezing range above: T_l - T_s = dT0 = G l_T, i.e. at z = z0 + V t + l_T;
* the window shift count s only relabels cells: cell i sits at the lab height
  (i + s + 1/2) dx, so the isotherms do not move when s changes.

The test reads the driving force from phi_t of a uniform phase field (phi =
1/2, no gradients: phi_t = -lambda Delta G p'(phi) / alpha with Delta G the
crystallisation free energy of the pair) and locates its zero crossing.
"""
import numpy as np
import pytest

N, DX = 400, 0.8
V, DT, LT, Z0 = 0.3, 0.1, 100.0, 40.0


def _zero_crossing(oracle, cs0, cl0, n, s, mutate=0):
    P = oracle.params(dim=1, n=(N, 1, 1), dx=DX, dt=DT, V=V, inv_lT=1.0 / LT, z0=Z0, mutate=mutate)
    phi = np.full(N, 0.5)
    pt = oracle.phi_t(P, phi, np.full(N, cs0), np.full(N, cl0), n, s)
    z = (np.arange(N) + s + 0.5) * DX  # lab heights of the window's cells
    slope, icpt = np.polyfit(z, pt, 1)
    resid = np.max(np.abs(pt - (slope * z + icpt)))
    return -icpt / slope, slope, resid, np.max(np.abs(pt))


CASES = [(0, 0), (500, 18), (500, 37), (1234, 46), (1234, 101)]


@pytest.mark.parametrize("n,s", CASES)
def test_isotherms_move_with_the_pulling_speed(oracle, n, s):
    ke = oracle.params()["ke"]
    t = n * DT
    zs, slope_s, res_s, mag = _zero_crossing(oracle, 1.0, 1.0 / ke, n, s)  # solidus pair
    zl, slope_l, res_l, _ = _zero_crossing(oracle, ke, 1.0, n, s)        # liquidus pair
    assert res_s <= 1e-12 * mag and res_l <= 1e-12 * mag  # linear in z: a uniform gradient
    assert zs == pytest.approx(Z0 + V * t, abs=1e-9)
    assert zl == pytest.approx(Z0 + V * t + LT, abs=1e-9)
    assert slope_s < 0 and slope_l < 0  # solidify below the isotherm, melt above it


@pytest.mark.parametrize("mutate,what", [(6, "isotherms pulled backwards"), (7, "lab height without the shift")])
def test_planted_isotherm_mistakes_fail(oracle, mutate, what):
    ke = oracle.params()["ke"]
    bad = 0
    for n, s in CASES:
        zs = _zero_crossing(oracle, 1.0, 1.0 / ke, n, s, mutate)[0]
        bad += abs(zs - (Z0 + V * n * DT)) > 1e-6
    assert bad > 0, f"mutate={mutate} ({what}) passes the isotherm pin"
