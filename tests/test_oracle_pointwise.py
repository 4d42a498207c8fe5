"""Pins of the oracle's pointwise algebra against the paper's definitions.

* interpolation functions: p(0)=0, p(1)=1, p'(0)=p'(1)=0, antisymmetry
  p(1-phi) = 1 - p(phi) (Sec. II, Eq. interpolation2), p' against a central
  difference of p, h(1/2) = 1/2;
* the driving force of the oracle against an independent evaluation of the
  general equation of motion (Eq. model18) built from the dilute free energies
  f_s, f_l (Eqs. dil1, dil_linear) and the set-2 mobilities M^n = M/h_n,
  M/(1-h_n) (Eq. interpolation1), with S_s = S_l = -A(c_s-c_l);
* the reduced drag coefficient D = [M_s(1-p)(1-A(1-p)) + A b M_l p^2]/Mbar of
  that drive, D(A=1) = p (the FID value D = g), and the printed form of
  Eq. drivingforce_nonvar differing from it (sign and the missing b);
* zero drive at the equilibrium of the dilute alloy (c_s = k_e c_l = c^eq).
"""
import math

import numpy as np
import pytest


def test_interp_endpoints_and_symmetry(oracle):
    for quintic in (0, 1):
        for ap in (0.0, 1.88396579, 11.05):
            p = oracle.params(quintic=quintic, ap=ap)
            q0 = oracle.pointwise(p, 0.0, 0.5, 1.0, 1.0)
            q1 = oracle.pointwise(p, 1.0, 0.5, 1.0, 1.0)
            assert q0["p"] == 0.0 and q1["p"] == 1.0
            assert q0["dp"] == 0.0 and q1["dp"] == 0.0
            assert q0["h"] == 0.0 and q1["h"] == 1.0
            assert oracle.pointwise(p, 0.5, 0.5, 1.0, 1.0)["h"] == 0.5
            for phi in np.linspace(0.01, 0.99, 23):
                a = oracle.pointwise(p, phi, 0.5, 1.0, 1.0)["p"]
                b = oracle.pointwise(p, 1.0 - phi, 0.5, 1.0, 1.0)["p"]
                assert a + b == pytest.approx(1.0, abs=2e-15)


def test_dp_is_derivative_of_p(oracle):
    for quintic in (0, 1):
        for ap in (0.0, 4.51654):
            p = oracle.params(quintic=quintic, ap=ap)
            for phi in np.linspace(0.05, 0.95, 19):
                e = 1e-6
                fd = (oracle.pointwise(p, phi + e, 0.5, 1.0, 1.0)["p"] -
                      oracle.pointwise(p, phi - e, 0.5, 1.0, 1.0)["p"]) / (2 * e)
                assert oracle.pointwise(p, phi, 0.5, 1.0, 1.0)["dp"] == pytest.approx(fd, rel=1e-8, abs=1e-9)
                # the double-well derivative: d/dphi phi^2 (1-phi)^2
                fd2 = ((phi + e) ** 2 * (1 - phi - e) ** 2 - (phi - e) ** 2 * (1 - phi + e) ** 2) / (2 * e)
                assert oracle.pointwise(p, phi, 0.5, 1.0, 1.0)["dfdw"] == pytest.approx(fd2, rel=1e-8, abs=1e-10)


def _free_energies(cs, cl, ke, cleq):
    """Dilute ideal alloy (Eq. dil_linear) in units of Omega c_inf, with the
    pure-solvent difference f_s^A - f_l^A = Omega (c_s^eq - c_l^eq) (Eq. dil5)
    and eps_s - eps_l = -Omega ln k_e (Eq. dil2); eps_l set to zero."""
    eps_s = -math.log(ke)
    fs = (ke - 1.0) * cleq + eps_s * cs + (cs * math.log(cs) - cs)
    fl = cl * math.log(cl) - cl
    mus = eps_s + math.log(cs)
    mul = math.log(cl)
    return fs, fl, mus, mul


def _model18_drive(phi, cs, cl, cleq, P):
    """Drive of Eq. model18 from the general mobilities of Eq. interpolation1."""
    from oracle.oracle import DEFAULTS  # noqa: F401  (parameters only)
    ke, A, b, Ds, ap = P["ke"], P["A"], P["b"], P["Ds"], P["ap"]
    h = phi ** 3 * (6 * phi ** 2 - 15 * phi + 10)
    p = h + ap * (phi - 0.5) * phi ** 2 * (1 - phi) ** 2
    hn = b * p / (b * p + 1 - p)
    Ms, Ml = Ds * cs, cl                      # M_i = D_i c_i / Omega
    Msn, Mln = Ms / hn, Ml / (1 - hn)         # normal mobilities
    Mbo = Msn + Mln                           # Mbar of Eq. model15
    fs, fl, mus, mul = _free_energies(cs, cl, ke, cleq)
    S = -A * (cs - cl)
    bs = fs - fl - (cs - cl) * mus - S * (1 - p) * (mus - mul)
    bl = fs - fl - (cs - cl) * mul - S * p * (mul - mus)
    return (Msn / Mbo) * bs + (Mln / Mbo) * bl, p, Ms, Ml


@pytest.mark.parametrize("A", [0.0, 0.7, 1.0, 1.2, 2.0])
@pytest.mark.parametrize("b", [1.0, 1e-3])
def test_drive_matches_model18(oracle, A, b):
    P = oracle.params(A=A, b=b)
    rng = np.random.default_rng(11)
    for _ in range(40):
        phi = rng.uniform(0.02, 0.98)
        cs, cl = rng.uniform(0.05, 2.0), rng.uniform(0.3, 5.0)
        cleq = rng.uniform(3.0, 9.0)
        ref, p, Ms, Ml = _model18_drive(phi, cs, cl, cleq, P)
        got = oracle.pointwise(P, phi, cs, cl, cleq)["dG"]
        assert got == pytest.approx(ref, rel=1e-11, abs=1e-12)
        # the same drive in the CGM form dG_c - D (c_s-c_l)(mu_s-mu_l)
        fs, fl, mus, mul = _free_energies(cs, cl, P["ke"], cleq)
        Mbar = Ms * (1 - p) + b * Ml * p
        D = (Ms * (1 - p) * (1 - A * (1 - p)) + A * b * Ml * p * p) / Mbar
        dGc = fs - fl - mul * (cs - cl)
        assert got == pytest.approx(dGc - D * (cs - cl) * (mus - mul), rel=1e-10, abs=1e-12)
        if A == 1.0:
            assert D == pytest.approx(p, rel=1e-12)
        # the printed reduced form differs (opposite sign of the drag, no b)
        Pp = dict(P, drag_variant=1)
        printed = oracle.pointwise(Pp, phi, cs, cl, cleq)["dG"]
        if abs(D * (cs - cl) * (mus - mul)) > 1e-6:
            assert abs(printed - got) > 1e-8


def test_zero_drive_at_equilibrium(oracle):
    P = oracle.params()
    ke = P["ke"]
    for cleq in (1.0 / ke, 3.0, 9.5):
        for phi in (0.1, 0.5, 0.9):
            q = oracle.pointwise(P, phi, ke * cleq, cleq, cleq)
            assert abs(q["dmu"]) < 1e-15
            assert abs(q["dG"]) < 1e-14 * cleq
