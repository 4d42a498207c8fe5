"""Pins of the oracle's interface terms, each with the planted mistakes it catches.

The set-2 equations the oracle steps (Eqs. cs_nonvar, cl_nonvar,
phasefield_nonvar) are reductions of the general equations of motion of
Sec. II.  These tests rebuild the interface terms from the general forms and
from the paper's constraints, written out here independently of the oracle:

* phi_t from Eq. model18 with the general normal mobilities
  M_s^n = M_s / h_n, M_l^n = M_l / (1 - h_n) (Eq. normal2, h_n of
  Eq. interpolation1), g = p, S_s = S_l = -A (c_s - c_l) (so that
  c~_s - c~_l = (1 - A)(c_s - c_l)), the dilute free energies (Eqs. dil1,
  dil_linear) and the frozen temperature (Eq. ds1).  This fixes the kinetic
  prefactor with its (1 - A)^2 term and the cross term X.
* The fluxes from Eqs. model16, model17 with the same mobilities and the
  tangential mobilities M_s^t = M_s / p, M_l^t = M_l / (1 - p).  This fixes
  the anti-trapping terms: their sign and the weights M_s^n / Mbar_n =
  M_s (1 - p) / Mbar and M_l^n / Mbar_n = b M_l p / Mbar.
* The Stefan-like condition Eq. model14, (c~_s - c~_l) phi_t =
  (J_s - J_l) . grad phi in the sign convention dc/dt = div J, at every face
  of a 1D interface.
* The overall solute flux Eq. solute_nonvar: p J_s + (1 - p) J_l equals the
  bracket of Eq. solute_nonvar with a(phi) of Eq. shape_function, here the
  oracle's separately written mixture flux of the equal-potential model,
  compared on states with mu_s = mu_l.

Discretisation: cell gradients are central differences with mirror ghosts,
the Laplacian is compact, face values are means of the two cells, face
gradients compact along the face normal (Sec. V.A); 1 - p is evaluated as
p(1 - phi) (antisymmetry of p); M_i grad mu_i of the tangential and cross
terms is D_i grad c_i (local mobility M_i = D_i c_i / Omega).

The table at the end plants each mistake in the oracle (its ``mutate``
switch) and asserts that at least one of these pins fails.
"""
import numpy as np
import pytest

N = 48
DX = 0.8


def _state(seed, equal_potential=False):
    r = np.random.default_rng(seed)
    z = (np.arange(N) + 0.5) * DX
    z0 = N * DX * 0.45 + r.uniform(0.0, DX)
    W = r.uniform(0.8, 1.5)
    phi = 1.0 / (1.0 + np.exp(np.sqrt(2.0) * (z - z0) / W))
    k = r.integers(1, 5, size=2)
    cl = 1.0 + 0.4 * r.uniform(-1, 1) * np.cos(k[1] * np.pi * z / z[-1] + r.uniform(0, 6)) + 0.3 * r.uniform()
    if equal_potential:
        cs = 0.14 * cl
    else:
        cs = 0.14 * (1.0 + 0.5 * r.uniform(-1, 1) * np.cos(k[0] * np.pi * z / z[-1] + r.uniform(0, 6))
                     + 0.5 * r.uniform())
    return phi, cs, cl


def _params(oracle, seed, **kw):
    r = np.random.default_rng(1000 + seed)
    p = dict(dim=1, n=(N, 1, 1), dx=DX, dt=1e-3, A=float(r.choice([2.0, 0.0, -0.7, 1.4, 3.0])),
             b=float(r.choice([1e-4, 1e-2, 1.0])), Ds=float(r.choice([1e-4, 1e-2, 0.3])),
             lambda0=float(r.uniform(0.02, 0.5)), W=float(r.uniform(0.8, 1.3)), Mphi=float(r.uniform(0.5, 2.0)),
             ke=0.14, eps_grad=1e-20, V=0.3, inv_lT=1.0 / 60.0, z0=10.0, quintic=1,
             ap=float(r.choice([0.0, 0.0, 1.2])))
    p.update(kw)
    return oracle.params(**p)


def _p_of(phi, P):
    h = phi ** 3 * (phi * (6.0 * phi - 15.0) + 10.0) if P["quintic"] else phi * phi * (3.0 - 2.0 * phi)
    return h + P["ap"] * (phi - 0.5) * phi ** 2 * (1.0 - phi) ** 2


def _dp_of(phi, P):
    w = phi * (1.0 - phi)
    dh = 30.0 * w * w if P["quintic"] else 6.0 * w
    return dh + P["ap"] * (w * w + (phi - 0.5) * 2.0 * w * (1.0 - 2.0 * phi))


def _cdiff(u):  # central difference / (2 dx), mirror ghosts
    up = np.concatenate([u[1:], u[-1:]])
    um = np.concatenate([u[:1], u[:-1]])
    return (up - um) / (2.0 * DX), up, um


def _mobilities(P, p, q, cs, cl):
    """Set-2 normal mobilities M^n = M/h_n, M/(1-h_n) and their sum."""
    hn = P["b"] * p / (P["b"] * p + q)
    one_m_hn = q / (P["b"] * p + q)
    Ms, Ml = P["Ds"] * cs, cl
    Msn, Mln = Ms / hn, Ml / one_m_hn
    return Ms, Ml, Msn, Mln, Msn + Mln


def _gate(G, P):
    return G / (G * G + P["eps_grad"] ** 2)


def model18_phi_t(P, phi, cs, cl, n=0, s=0):
    """phi_t of Eq. model18 (nondimensional: divided by H, lambda = Omega c_inf / H)."""
    W, alpha, lam = P["W"], P["W"] / P["Mphi"], P["lambda0"] * P["W"]
    ke, A = P["ke"], P["A"]
    p, q, dp = _p_of(phi, P), _p_of(1.0 - phi, P), _dp_of(phi, P)
    Ms, Ml, Msn, Mln, Mbn = _mobilities(P, p, q, cs, cl)
    z = (np.arange(N) + s + 0.5) * DX
    cleq = (1.0 - (1.0 - ke) * (z - P["z0"] - P["V"] * n * P["dt"]) * P["inv_lT"]) / ke
    fs = cs * np.log(cs) - cs - cs * np.log(ke) + (ke - 1.0) * cleq
    fl = cl * np.log(cl) - cl
    mus, mul = np.log(cs) - np.log(ke), np.log(cl)
    S = -A * (cs - cl)
    dct = (cs - cl) + S * p + S * q  # c~_s - c~_l
    Bs = fs - fl - (cs - cl) * mus - S * q * (mus - mul)
    Bl = fs - fl - (cs - cl) * mul - S * p * (mul - mus)
    gphi, pp, pm = _cdiff(phi)
    gcs, _, _ = _cdiff(cs)
    gcl, _, _ = _cdiff(cl)
    lap = (pp - 2.0 * phi + pm) / (DX * DX)
    gam = _gate(gphi * gphi, P)
    # M_s^n g grad mu_s - M_l^n (1-g) grad mu_l with M_i grad mu_i = D_i grad c_i
    vec = (Msn * p / Ms) * (P["Ds"] * gcs) - (Mln * q / Ml) * gcl
    X = lam * dct / Mbn * vec * gphi * gam
    pref = alpha + lam * dct * dct * gam / Mbn
    fdw = 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi)
    rhs = W * W * lap - fdw - lam * (Msn / Mbn * Bs + Mln / Mbn * Bl) * dp + X
    return rhs / pref


def model16_17_fluxes(P, phi, cs, cl, phit):
    """Face fluxes of Eqs. model16, model17 (returned as J with dc/dt = div J +
    sources, i.e. minus the paper's J) through the faces i + 1/2, i = 0..N-2."""
    A, ke = P["A"], P["ke"]
    a, b = slice(0, N - 1), slice(1, N)
    phf, csf, clf = 0.5 * (phi[a] + phi[b]), 0.5 * (cs[a] + cs[b]), 0.5 * (cl[a] + cl[b])
    ptf = 0.5 * (phit[a] + phit[b])
    pf, qf = _p_of(phf, P), _p_of(1.0 - phf, P)
    Ms, Ml, Msn, Mln, Mbn = _mobilities(P, pf, qf, csf, clf)
    p_c, q_c = _p_of(phi, P), _p_of(1.0 - phi, P)
    mubar = p_c * (np.log(cs) - np.log(ke)) + q_c * np.log(cl)
    g = {k: (u[b] - u[a]) / DX for k, u in (("phi", phi), ("mu", mubar), ("cs", cs), ("cl", cl))}
    gam = _gate(g["phi"] ** 2, P)
    Pn = gam * g["phi"] ** 2  # normal projector in 1D
    qn = Msn * Mln / Mbn
    dct = (1.0 - A) * (csf - clf)
    anti = dct * g["phi"] * gam * ptf  # (c~_s - c~_l) phi_t grad phi / |grad phi|^2
    Js = qn * Pn * g["mu"] + P["Ds"] * (1.0 - Pn) * g["cs"] + (Msn / Mbn) * anti
    Jl = qn * Pn * g["mu"] + (1.0 - Pn) * g["cl"] - (Mln / Mbn) * anti
    return Js, Jl, dct, ptf, g["phi"], Pn


def _rel(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


# ---- the pins, as discrepancies -----------------------------------------------

def pin_model18(oracle, P, seeds):
    e = 0.0
    for s in seeds:
        phi, cs, cl = _state(s)
        for n, sh in ((0, 0), (37, 3)):
            e = max(e, _rel(oracle.phi_t(P, phi, cs, cl, n, sh), model18_phi_t(P, phi, cs, cl, n, sh)))
    return e


def pin_model16_17(oracle, P, seeds):
    e = 0.0
    for s in seeds:
        phi, cs, cl = _state(s)
        js, jl, _, _ = oracle.face_fluxes(P, phi, cs, cl, 0)
        Js, Jl, *_ = model16_17_fluxes(P, phi, cs, cl, oracle.phi_t(P, phi, cs, cl))
        e = max(e, _rel(js[:-1], Js), _rel(jl[:-1], Jl))
    return e


def pin_stefan(oracle, P, seeds):
    """Eq. model14 at the faces where the normal projector is 1."""
    e = 0.0
    for s in seeds:
        phi, cs, cl = _state(s)
        js, jl, _, _ = oracle.face_fluxes(P, phi, cs, cl, 0)
        _, _, dct, ptf, gph, Pn = model16_17_fluxes(P, phi, cs, cl, oracle.phi_t(P, phi, cs, cl))
        m = Pn > 1.0 - 1e-13
        lhs = dct[m] * ptf[m]
        rhs = (js[:-1][m] - jl[:-1][m]) * gph[m]
        e = max(e, _rel(rhs, lhs))
    return e


def pin_solute_nonvar(oracle, P, seeds):
    e = 0.0
    for s in seeds:
        phi, cs, cl = _state(s, equal_potential=True)
        js, jl, jm, pf = oracle.face_fluxes(P, phi, cs, cl, 0)
        qf = 1.0 - pf
        e = max(e, _rel(pf[:-1] * js[:-1] + qf[:-1] * jl[:-1], jm[:-1]))
    return e


PINS = {"model18": pin_model18, "model16_17": pin_model16_17, "stefan": pin_stefan,
        "solute_nonvar": pin_solute_nonvar}
TOL = {"model18": 1e-10, "model16_17": 1e-10, "stefan": 1e-10, "solute_nonvar": 1e-10}
SEEDS = range(6)


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("pin", sorted(PINS))
def test_interface_pins_hold(oracle, pin, case):
    P = _params(oracle, case)
    e = PINS[pin](oracle, P, SEEDS)
    assert e <= TOL[pin], f"{pin}: relative discrepancy {e:.3e} (params {P})"


# Planted mistakes (oracle ``mutate`` codes) and the pins each must fail.
MUTATIONS = {
    1: ("anti-trapping weights exchanged", {"model16_17", "solute_nonvar"}),
    2: ("anti-trapping sign flipped", {"model16_17", "stefan", "solute_nonvar"}),
    3: ("cross term X dropped", {"model18"}),
    4: ("(1-A)^2 prefactor term dropped", {"model18"}),
}


@pytest.mark.parametrize("mut", sorted(MUTATIONS))
def test_planted_mistakes_fail_their_pins(oracle, mut):
    what, expect = MUTATIONS[mut]
    failed = set()
    for case in range(4):
        P = _params(oracle, case, mutate=mut, A=2.0)
        for pin in PINS:
            if PINS[pin](oracle, P, SEEDS) > 1e3 * TOL[pin]:
                failed.add(pin)
    assert expect <= failed, f"mutation {mut} ({what}): expected {sorted(expect)} to fail, failed {sorted(failed)}"
