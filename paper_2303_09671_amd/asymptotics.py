"""Parameter selection from the thin-interface asymptotics (Sec. IV, Sec. V.C).

The paper's asymptotic analysis is carried out for the model with pointwise
equal diffusion potentials.  To first order it gives the jump of the diffusion
potential across a moving interface (Eq. jump).  For a dilute alloy that jump
turns into a transcendental relation for the velocity-dependent partition
coefficient (Eq. partition1):

    ln(k_v / k_e) = (V W / D_l) (1 - k_v) dF,   dF = F^- - F^+.

F^{+-} (Eqs. integral1, integral2) integrate p~(phi0) - p~(phi0 at +-inf) over the
equilibrium profile phi0(eta) = [1 - tanh(eta / sqrt 2)] / 2, with the solid at
eta < 0.  Here

    p~ = [p - 1 - (1 - A) a] M_l0 / q_n,

where q_n is the normal mobility of Eqs. normal2 and interpolation1 and a(phi)
is the shape function of Eq. shape_function.  Both are written with
m = M_s / M_l0:

    M_l0 / q_n = h_n / m + 1 - h_n,          h_n = b p / (b p + 1 - p),
    a          = (m - b) p (1 - p) / (m (1 - p) + b p),

with p the interpolation of Eq. interpolation2, p = h + a_p (phi - 1/2) phi^2 (1 - phi)^2.

The Kapitza term of Eq. jump vanishes when G^+ = G^- (Eq. integral3), and
that condition fixes a_p.  The paper takes the smaller roots.

Every quantity here is a function of phi0 alone.  It is evaluated from phi0
and 1 - phi0 = phi0(-eta), using 1 - h(phi) = h(1 - phi).  The difference
1 - p is therefore never formed next to the solid.  This matters because
b and m reach 1e-5, and 1/m multiplies that difference.  The integrals use
composite Gauss-Legendre quadrature in eta on [-L, 0] and [0, L].

The module computes, on the host and for scalars only:
* a_p roots;
* a k_v(V) curve for given (A, b, W);
* the A that best reproduces a target curve at a given W, which is the starting
  point of the adjoint-driven fit (fit.py).

The mobility ratio m = M_s / M_l0 = chi D_s/D_l is an input.  For the dilute
ideal alloy chi = (dc_s/dmu) / (dc_l/dmu) = c_s / c_l, which is k_e at
equilibrium.  The paper instead compares b directly with D_s/D_l when it
discusses the shape of q_n, which is chi = 1.  Both readings are available;
the default is chi = 1.

The paper reads Eq. partition1 as a first estimate, because the equations
that are actually stepped do not hold mu_s = mu_l.  The simulated k is
measured separately and is not expected to match to better than that.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.optimize import brentq, minimize_scalar

SQRT2 = math.sqrt(2.0)
I_DW = 1.0 / (3.0 * SQRT2)  # int (d phi0 / d eta)^2 d eta for f_dw = phi^2 (1 - phi)^2

_L = 40.0       # |eta| beyond which every integrand is below 1e-24
_PANEL = 0.25   # panel width of the composite rule
_NODES = 20     # Gauss-Legendre nodes per panel


def _rule(lo: float, hi: float):
    x, w = np.polynomial.legendre.leggauss(_NODES)
    edges = np.linspace(lo, hi, int(round((hi - lo) / _PANEL)) + 1)
    a, b = edges[:-1, None], edges[1:, None]
    return ((b - a) * 0.5 * x + (a + b) * 0.5).ravel(), ((b - a) * 0.5 * w + 0.0 * a).ravel()


_ETA_P, _W_P = _rule(0.0, _L)     # liquid side, eta in [0, L]
_ETA_M, _W_M = _rule(-_L, 0.0)    # solid side, eta in [-L, 0]


def phi0(eta):
    """Equilibrium profile (solid phi = 1 for eta -> -inf)."""
    return 0.5 * (1.0 - np.tanh(np.asarray(eta, dtype=np.float64) / SQRT2))


def _h(x, quintic: bool):
    return x ** 3 * (x * (6.0 * x - 15.0) + 10.0) if quintic else x * x * (3.0 - 2.0 * x)


def p_and_q(phi, psi, ap: float = 0.0, quintic: bool = True):
    """p(phi) of Eq. interpolation2 and q = 1 - p, from phi and psi = 1 - phi
    (each side evaluated where it is small)."""
    bump = ap * (phi - 0.5) * phi * phi * psi * psi
    return _h(phi, quintic) + bump, _h(psi, quintic) - bump


@dataclass(frozen=True)
class Interface:
    """Constants of the set-2 interpolation (Eqs. normal2, interpolation1,
    interpolation2, shape_function): A, b, a_p and m = M_s / M_l0 = chi D_s/D_l."""
    A: float
    b: float
    m: float
    ap: float = 0.0
    quintic: bool = True

    def _parts(self, eta):
        phi, psi = phi0(eta), phi0(-np.asarray(eta, dtype=np.float64))
        p, q = p_and_q(phi, psi, self.ap, self.quintic)
        with np.errstate(divide="ignore", invalid="ignore"):  # an a_p far outside the admissible range
            den = self.b * p + q
            hn, one_m_hn = self.b * p / den, q / den
            R = hn / self.m + one_m_hn                     # M_l0 / q_n
            a = (self.m - self.b) * p * q / (self.m * q + self.b * p)
        return p, q, hn, one_m_hn, R, a

    def ml_over_qn(self, phi):
        """M_l0 / q_n at phi (from Eqs. normal2 and interpolation1)."""
        eta = SQRT2 * np.arctanh(1.0 - 2.0 * np.asarray(phi, dtype=np.float64))
        return self._parts(eta)[4]

    def shape(self, phi):
        """a(phi) of Eq. shape_function."""
        eta = SQRT2 * np.arctanh(1.0 - 2.0 * np.asarray(phi, dtype=np.float64))
        return self._parts(eta)[5]

    def F(self):
        """(F^-, F^+) of Eqs. integral1, integral2.

        Liquid side: p~ -> -1, and the integrand p~ + 1 is expanded as
        p - q h_n (1/m - 1) - (1 - A) a R.  Solid side: p~ -> 0, and
        F^- = int_{-inf}^0 (q + (1 - A) a) R d eta."""
        p, q, hn, _, R, a = self._parts(_ETA_P)
        fp = np.dot(_W_P, p - q * hn * (1.0 / self.m - 1.0) - (1.0 - self.A) * a * R)
        p, q, hn, _, R, a = self._parts(_ETA_M)
        fm = np.dot(_W_M, (q + (1.0 - self.A) * a) * R)
        return float(fm), float(fp)

    def dF(self) -> float:
        fm, fp = self.F()
        return fm - fp

    def G(self):
        """(G^-, G^+) of Eq. integral3 in units of M_l0:
        G^+ = (1/m - 1) int_0^inf h_n, G^- = (1/m - 1) int_{-inf}^0 (1 - h_n)."""
        c = 1.0 / self.m - 1.0
        gp = c * np.dot(_W_P, self._parts(_ETA_P)[2])
        gm = c * np.dot(_W_M, self._parts(_ETA_M)[3])
        return float(gm), float(gp)


def k_v(V: float, S: float, ke: float) -> float:
    """Root in [k_e, 1) of ln(k / k_e) = V S (1 - k), S = W dF / D_l
    (Eq. partition1); k_e when V S <= 0 would put it below k_e (V S = 0)."""
    s = V * S
    if s <= 0.0:
        if s == 0.0:
            return ke
        return brentq(lambda k: math.log(k / ke) - s * (1.0 - k), 1e-300, ke, xtol=1e-300, rtol=1e-15,
                      maxiter=400)
    return brentq(lambda k: math.log(k / ke) - s * (1.0 - k), ke, 1.0, xtol=1e-300, rtol=1e-15, maxiter=400)


def kv_curve(Vs, A: float, b: float, m: float, ke: float, W: float = 1.0, ap: float = 0.0,
             quintic: bool = True):
    """k_v at nondimensional velocities Vs (lengths in W0, time in W0^2/D_l) and
    the dF it was computed with."""
    dF = Interface(A=A, b=b, m=m, ap=ap, quintic=quintic).dF()
    return np.array([k_v(float(V), W * dF, ke) for V in np.atleast_1d(Vs)]), dF


def ap_roots(b: float, m: float, quintic: bool = True, amax: float = 30.0, n: int = 600):
    """Values of a_p with G^+ = G^- (Eq. integral3).  Sign changes of
    G^+ - G^- are found on a uniform grid over [-amax, amax] and refined with
    Brent's method.  The roots are sorted by magnitude; the paper prefers the
    smaller ones.

    With b = 1, h_n = p, and p - 1/2 is odd in eta for every a_p.  G^+ = G^-
    then holds for all a_p; this is the inverse interpolation of Eq. inverse,
    which has no Kapitza jump.  In that case the function returns [0.0]."""
    def g(a):
        gm, gp = Interface(A=1.0, b=b, m=m, ap=a, quintic=quintic).G()
        return gp - gm, abs(gp) + abs(gm)

    xs = np.linspace(-amax, amax, n + 1)
    vals, scale = np.array([g(x) for x in xs]).T
    zero = np.abs(vals) <= 1e-12 * scale
    if zero.all():
        return [0.0]
    roots = [float(x) for x in xs[zero]]
    for i in range(n):
        if not (zero[i] or zero[i + 1]) and vals[i] * vals[i + 1] < 0.0:
            roots.append(brentq(lambda a: g(a)[0], xs[i], xs[i + 1], xtol=1e-13, rtol=1e-15))
    return sorted(roots, key=abs)


def admissible(ap: float, b: float, quintic: bool = True) -> bool:
    """Whether (b, a_p) gives p in [0, 1] and b p + 1 - p > 0 over phi in [0, 1].
    Together these keep q_n >= 0, which Sec. IV requires for the phase
    concentration equations, and they are what the library accepts."""
    phi = np.linspace(0.0, 1.0, 4001)
    p, q = p_and_q(phi, 1.0 - phi, ap, quintic)
    return bool(p.min() >= -1e-12 and q.min() >= -1e-12 and (b * p + q).min() > 0.0)


def fit_S(Vs, k_target, ke: float) -> float:
    """S = W dF / D_l of Eq. partition1 that minimises sum (k_v(V_i; S) - k*_i)^2."""
    Vs = np.asarray(Vs, dtype=np.float64)
    kt = np.asarray(k_target, dtype=np.float64)
    # each point alone gives S_i = ln(k_i/k_e) / (V_i (1 - k_i)); bracket the fit with them
    ok = (kt > ke) & (kt < 1.0) & (Vs > 0.0)
    if not np.any(ok):
        raise ValueError("no target point with k_e < k < 1 and V > 0")
    Si = np.log(kt[ok] / ke) / (Vs[ok] * (1.0 - kt[ok]))
    lo, hi = 0.5 * Si.min(), 2.0 * Si.max()

    def loss(S):
        return float(sum((k_v(V, S, ke) - k) ** 2 for V, k in zip(Vs, kt)))

    return float(minimize_scalar(loss, bounds=(lo, hi), method="bounded",
                                 options=dict(xatol=1e-12 * hi)).x)


def A_for_curve(Vs, k_target, b: float, m: float, ke: float, W: float = 1.0, ap: float = 0.0,
                quintic: bool = True):
    """The source strength A whose Eq. partition1 curve at interface width W
    best fits (V, k*).  dF is affine in A (p~ is), dF(A) = dF(1) + (1 - A) D,
    so A = 1 - (S / W - dF(1)) / D.  Returns (A, S).  Raises if a(phi) vanishes
    (m = b), where A has no effect on the curve."""
    S = fit_S(Vs, k_target, ke)
    d1 = Interface(A=1.0, b=b, m=m, ap=ap, quintic=quintic).dF()
    d0 = Interface(A=0.0, b=b, m=m, ap=ap, quintic=quintic).dF()
    D = d0 - d1
    if abs(D) < 1e-14 * max(1.0, abs(d1)):
        raise ValueError("a(phi) vanishes (M_s = b M_l): A does not change the curve")
    return 1.0 - (S / W - d1) / D, S


def W_for_curve(Vs, k_target, A: float, b: float, m: float, ke: float, ap: float = 0.0,
                quintic: bool = True):
    """The interface width W (in W0) whose Eq. partition1 curve at source
    strength A best fits (V, k*): W = S / dF(A).  Returns (W, S)."""
    S = fit_S(Vs, k_target, ke)
    dF = Interface(A=A, b=b, m=m, ap=ap, quintic=quintic).dF()
    if not dF > 0.0:
        raise ValueError("dF <= 0: the curve has no trapping at any W")
    return S / dF, S


def start_theta(Vs, k_target, theta, b: float, Ds: float, ke: float, chi: float = 1.0, ap: float = 0.0,
                quintic: bool = True):
    """A starting theta = (A, M_phi, W) for the adjoint fit.

    theta holds the caller's current values.  A is chosen at the current W
    when a(phi) depends on A (M_s != b M_l).  Otherwise W is chosen at the
    current A.  M_phi does not enter Eq. partition1 and is kept.
    The mobility ratio is m = chi D_s/D_l.  Returns (theta0, S)."""
    A, Mphi, W = (float(v) for v in theta)
    m = chi * Ds
    try:
        A, S = A_for_curve(Vs, k_target, b, m, ke, W=W, ap=ap, quintic=quintic)
    except ValueError:
        W, S = W_for_curve(Vs, k_target, A, b, m, ke, ap=ap, quintic=quintic)
    return np.array([A, Mphi, W]), S


# Table 1 of the paper, SI units; liquidus slope in K per at.%, c_inf in at.%.
ALLOYS = {
    "Si-9As": dict(ke=0.3, Tm=1685.0, m_liq=-4.0, cinf=9.0, Gamma=3.4e-7, d0=13.5e-9, Dl=15e-9, beta=0.595),
    "Ni-5Cu": dict(ke=0.5, Tm=1728.0, m_liq=-2.0, cinf=5.0, Gamma=2.6e-7, d0=26e-9, Dl=3e-9, beta=0.2),
}


def nondim(alloy: str, W: float, v_p, G: float = 1.4e7) -> dict:
    """Map an alloy of Table 1 to the library's units at interface width W (m):
    W0 = W, t0 = W^2 / D_l.  Returns the nondimensional pulling speeds
    V = v_p W / D_l, the freezing range dT0 = |m| c_inf (1 - k_e) / k_e, the
    inverse thermal length inv_lT = W G / dT0, lambda0 = I (W / d0) k_e / (1 - k_e)^2
    and the time unit in seconds."""
    a = ALLOYS[alloy]
    ke = a["ke"]
    dT0 = abs(a["m_liq"]) * a["cinf"] * (1.0 - ke) / ke
    return dict(ke=ke, V=np.asarray(v_p, dtype=np.float64) * W / a["Dl"], dT0=dT0, inv_lT=W * G / dT0,
                lambda0=I_DW * (W / a["d0"]) * ke / (1.0 - ke) ** 2, t0=W * W / a["Dl"])
