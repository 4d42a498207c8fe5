"""Pins of the asymptotic parameter selection (Sec. IV, Eqs. integral1-3,
normal2, shape_function, partition1), against constructions that do not go
through the module's own algebra:

* q_n and a(phi) from the general definitions (Eqs. normal, antitrapping) with
  the set-2 mobilities M_s^n = M_s / h_n, M_l^n = M_l / (1 - h_n);
* b = 1 (inverse interpolation, Eq. inverse): G^+ = G^- for every a_p, as the
  paper states for that interpolation;
* the smallest a_p root of b = 1e-3 satisfies G^+ = G^- when G is integrated
  independently (adaptive quadrature in phi, the plain formulas);
* F^{+-} in closed form (polynomial division plus ln 2) when p~ is a polynomial
  in phi (b = 1, A = 1), and by adaptive quadrature of the plain Eq. integral2
  in general;
* the symmetric interface (M_s = M_l, b = 1) has dF = 0, so k_v = k_e;
* the root of Eq. partition1 against its Lambert-W closed form and its
  small-V slope;
* the double-well constant I, and the Table 1 unit map.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import Polynomial as P
from scipy.integrate import quad
from scipy.special import lambertw

from paper_2303_09671_amd import asymptotics as asy

SQ2 = math.sqrt(2.0)


def _p_plain(phi, ap, quintic=True):
    h = phi ** 3 * (6 * phi ** 2 - 15 * phi + 10) if quintic else phi ** 2 * (3 - 2 * phi)
    return h + ap * (phi - 0.5) * phi ** 2 * (1 - phi) ** 2


def _plain(phi, A, b, m, ap, quintic=True):
    """q_n / M_l0 and a(phi) written from Eqs. normal and antitrapping (M_l = 1,
    M_s = m): M_s^n = M_s / h_n, M_l^n = M_l / (1 - h_n), Mbar = M_s^n + M_l^n."""
    p = _p_plain(phi, ap, quintic)
    hn = b * p / (b * p + 1 - p)
    Msn, Mln = m / hn, 1.0 / (1 - hn)
    Mbar = Msn + Mln
    qn = Msn * Mln / Mbar
    a = (Msn * p - Mln * (1 - p)) / Mbar
    return p, qn, a


@pytest.mark.parametrize("b,m,ap,quintic", [(1e-3, 3e-4, 0.0, True), (0.2, 0.05, -1.5, True),
                                            (1e-5, 1e-3, 0.0, False), (1.0, 0.3, 0.7, True)])
def test_qn_and_shape_from_general_definitions(b, m, ap, quintic):
    phi = np.linspace(0.02, 0.98, 49)
    _, qn, a = _plain(phi, 1.0, b, m, ap, quintic)
    itf = asy.Interface(A=1.0, b=b, m=m, ap=ap, quintic=quintic)
    np.testing.assert_allclose(itf.ml_over_qn(phi), 1.0 / qn, rtol=1e-11)
    np.testing.assert_allclose(itf.shape(phi), a, rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("m,ap,quintic", [(3e-4, 0.0, True), (0.3, -2.0, True), (1e-2, 1.3, False)])
def test_inverse_interpolation_has_no_kapitza_jump(m, ap, quintic):
    gm, gp = asy.Interface(A=1.0, b=1.0, m=m, ap=ap, quintic=quintic).G()
    assert abs(gp - gm) <= 1e-12 * abs(gp)
    assert asy.ap_roots(1.0, m, quintic=quintic, n=40) == [0.0]


def test_ap_roots_do_not_depend_on_m():
    # G^+ - G^- = (1/m - 1) (int_0^inf h_n - int_-inf^0 (1 - h_n)): only b sets the roots
    r1 = asy.ap_roots(1e-3, 3e-4, amax=4.0, n=80)[:3]
    r2 = asy.ap_roots(1e-3, 0.3, amax=4.0, n=80)[:3]
    assert len(r1) == 3
    np.testing.assert_allclose(r1, r2, rtol=1e-9)


def test_smallest_root_balances_G_by_independent_quadrature():
    b, m = 1e-3, 0.3
    a_star = asy.ap_roots(b, m, amax=4.0, n=80)[0]
    assert 1.0 < a_star < 3.0

    def R(phi):  # M_l0 / q_n
        _, qn, _ = _plain(phi, 1.0, b, m, a_star)
        return 1.0 / qn

    jac = lambda phi: 1.0 / (SQ2 * phi * (1.0 - phi))  # d eta = -jac d phi
    gp = quad(lambda f: (R(f) - 1.0) * jac(f), 0.0, 0.5, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    gm = -quad(lambda f: (R(f) - 1.0 / m) * jac(f), 0.5, 1.0, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    assert abs(gp - gm) <= 1e-8 * abs(gp)
    # and a neighbouring a_p does not balance them
    gm2, gp2 = asy.Interface(A=1.0, b=b, m=m, ap=a_star + 0.05).G()
    assert abs(gp2 - gm2) > 1e-4 * abs(gp2)


def _poly_p(ap, quintic):
    x = P([0.0, 1.0])
    h = x ** 3 * (6 * x ** 2 - 15 * x + 10) if quintic else x ** 2 * (3 - 2 * x)
    return h + ap * (x - 0.5) * x ** 2 * (1 - x) ** 2


def _int_over_interface(Pn, lo, hi):
    """int_lo^hi Pn(phi) / (phi (1 - phi)) d phi, exactly: Pn / (phi (1-phi)) =
    Q + Pn(0)/phi + Pn(1)/(1-phi) with Q a polynomial."""
    x = P([0.0, 1.0])
    num = Pn - Pn(0.0) * (1 - x) - Pn(1.0) * x
    Q, r = divmod(num, x * (1 - x))
    assert np.max(np.abs(r.coef)) < 1e-9
    Qi = Q.integ()
    log = lambda t: math.log(t) if t > 0 else 0.0
    val = Qi(hi) - Qi(lo)
    if Pn(0.0) != 0.0:
        val += Pn(0.0) * (log(hi) - log(lo))
    if abs(Pn(1.0)) > 0.0:
        val += Pn(1.0) * (-(log(1 - hi) if hi < 1 else 0.0) + log(1 - lo))
    return val


@pytest.mark.parametrize("m,ap,quintic", [(3e-4, 0.0, True), (0.25, -1.0, True), (0.05, 0.0, False)])
def test_F_closed_form_polynomial_case(m, ap, quintic):
    # b = 1: h_n = p; A = 1: no shape term.  p~ = -(1 - p)(p/m + 1 - p), a polynomial.
    p = _poly_p(ap, quintic)
    q = 1 - p
    pt = -q * (p / m + q)
    Fp = _int_over_interface(pt + 1.0, 0.0, 0.5) / SQ2   # pt + 1 vanishes at phi = 0
    Fm = -_int_over_interface(pt, 0.5, 1.0) / SQ2        # pt vanishes at phi = 1
    fm, fp = asy.Interface(A=1.0, b=1.0, m=m, ap=ap, quintic=quintic).F()
    assert abs(fp - Fp) <= 1e-11 * max(1.0, abs(Fp))
    assert abs(fm - Fm) <= 1e-11 * max(1.0, abs(Fm))


@pytest.mark.parametrize("A,b,m,ap", [(1.7, 0.1, 0.3, 0.0), (0.4, 1e-2, 5e-3, -0.8), (2.0, 0.5, 0.05, 0.0)])
def test_F_against_plain_integral2(A, b, m, ap):
    def ptilde(phi):
        p, qn, a = _plain(phi, A, b, m, ap)
        return (p - 1.0 - (1.0 - A) * a) / qn

    jac = lambda phi: 1.0 / (SQ2 * phi * (1.0 - phi))
    Fp = quad(lambda f: (ptilde(f) + 1.0) * jac(f), 0.0, 0.5, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    Fm = -quad(lambda f: ptilde(f) * jac(f), 0.5, 1.0, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    fm, fp = asy.Interface(A=A, b=b, m=m, ap=ap).F()
    assert abs(fp - Fp) <= 1e-9 * max(1.0, abs(Fp))
    assert abs(fm - Fm) <= 1e-9 * max(1.0, abs(Fm))


@pytest.mark.parametrize("A", [0.0, 1.0, 2.0])
def test_symmetric_interface_does_not_trap(A):
    dF = asy.Interface(A=A, b=1.0, m=1.0).dF()
    assert abs(dF) < 1e-13
    k, _ = asy.kv_curve([0.1, 1.0, 10.0], A, 1.0, 1.0, 0.3)
    np.testing.assert_allclose(k, 0.3, rtol=1e-12)


def test_dF_affine_in_A():
    d = [asy.Interface(A=A, b=1e-3, m=3e-4).dF() for A in (0.0, 1.0, 2.5)]
    assert abs(d[2] - (d[1] + (1.0 - 2.5) * (d[0] - d[1]))) < 1e-12 * abs(d[1])


@pytest.mark.parametrize("S", [0.5, 3.0, 20.0])
@pytest.mark.parametrize("ke", [0.14, 0.3, 0.5])
def test_kv_against_lambert_w(S, ke):
    for V in (1e-3, 0.05, 0.3, 1.0, 10.0):
        s = V * S
        ref = float(lambertw(s * ke * math.exp(s)).real) / s  # s k e^{s k} = s k_e e^s
        assert abs(asy.k_v(V, S, ke) - ref) <= 1e-13
    # small V: k - k_e ~ k_e (1 - k_e) S V
    V = 1e-7
    assert abs((asy.k_v(V, S, ke) - ke) / V - ke * (1 - ke) * S) <= 1e-5 * ke * S


def test_double_well_constant():
    d = lambda e: -1.0 / (2.0 * SQ2 * np.cosh(e / SQ2) ** 2)  # d phi0 / d eta
    I = quad(lambda e: d(e) ** 2, -50.0, 50.0, epsabs=1e-15, epsrel=1e-13)[0]
    assert abs(I - asy.I_DW) < 1e-13
    e = np.linspace(-6, 6, 13)
    np.testing.assert_allclose((asy.phi0(e + 1e-6) - asy.phi0(e - 1e-6)) / 2e-6, d(e), atol=1e-9)


def test_fits_invert_the_curve():
    Vs = np.array([0.02, 0.1, 0.3, 0.6])
    k, _ = asy.kv_curve(Vs, 1.35, 1e-4, 1.4e-5, 0.14, W=1.3)
    A, S = asy.A_for_curve(Vs, k, 1e-4, 1.4e-5, 0.14, W=1.3)
    assert abs(A - 1.35) < 1e-6
    k2, _ = asy.kv_curve(Vs, 1.0, 1e-3, 1e-3, 0.3, W=0.7)
    with pytest.raises(ValueError):
        asy.A_for_curve(Vs, k2, 1e-3, 1e-3, 0.3)  # M_s = b M_l: A has no effect
    W, _ = asy.W_for_curve(Vs, k2, 1.0, 1e-3, 1e-3, 0.3)
    assert abs(W - 0.7) < 1e-6
    th, _ = asy.start_theta(Vs, k2, (1.2, 1.1, 1.0), b=1e-3, Ds=1e-3, ke=0.3, chi=1.0)
    assert abs(th[2] - 0.7) < 1e-6 and th[0] == 1.2 and th[1] == 1.1


def test_admissible_a_p():
    assert asy.admissible(0.0, 1e-3)
    assert asy.admissible(-2.0, 1e-3)
    assert not asy.admissible(0.4, 1e-3)  # p''(0) = -a_p: p < 0 next to the liquid
    # the roots of G+ = G- for b = 1e-3 are positive, so none is admissible
    assert all(r > 0 and not asy.admissible(r, 1e-3) for r in asy.ap_roots(1e-3, 1e-3, amax=4.0, n=80))


def test_table1_unit_map():
    s = asy.nondim("Si-9As", 13.5e-9, [0.3, 1.0], G=1.4e6)
    np.testing.assert_allclose(s["V"], [0.27, 0.9], rtol=1e-12)
    assert abs(s["dT0"] - 84.0) < 1e-12
    assert abs(1.0 / s["inv_lT"] - 4444.444444444444) < 1e-6
    assert abs(s["lambda0"] - asy.I_DW * 0.3 / 0.49) < 1e-15  # W = d0
    n = asy.nondim("Ni-5Cu", 26e-9, 1.0)
    assert abs(n["dT0"] - 10.0) < 1e-12 and abs(n["V"] - 26e-9 / 3e-9) < 1e-12


def test_band_workload_matches_table1_map():
    """The solute-band workload is the Table 1 alloy Si-9%As at W = 13.5 nm,
    v_p = 0.3 m/s and G = 1.4e6 K/m mapped to the library's units."""
    from paper_2303_09671_amd import inputs as I
    p, _ = I.config_bands()
    s = asy.nondim("Si-9As", 13.5e-9, 0.3, G=1.4e6)
    assert abs(p["V"] - s["V"]) < 1e-12 and p["ke"] == s["ke"]
    assert abs(p["inv_lT"] - s["inv_lT"]) < 1e-3 * s["inv_lT"]  # l_T rounded to 4444 W
    assert abs(p["lambda0"] - s["lambda0"]) < 1e-15


def test_ti_curve_workload_matches_table1_map():
    """The T_I(V) workload is the Table 1 alloy Si-9%As at W = 13.5 nm and
    G = 1.4e7 K/m mapped to the library's units."""
    from paper_2303_09671_amd import inputs as I
    base, runs, _, vp = I.config_ti_curve(1.2)
    s = asy.nondim("Si-9As", 13.5e-9, vp, G=1.4e7)
    assert np.allclose([r["V"] for r in runs], s["V"], rtol=1e-12, atol=0.0) and base["ke"] == s["ke"]
    assert abs(base["inv_lT"] - s["inv_lT"]) < 1e-12 * s["inv_lT"]
    assert abs(base["lambda0"] - s["lambda0"]) < 1e-15
