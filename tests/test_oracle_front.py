"""Pins of the oracle's front diagnostic (the phi = 1/2 crossing and its
temperature, Sec. V.C), against independent constructions:

* a front centred on a cell face is found exactly there, by symmetry;
* off-face fronts: numpy's linear interpolation of the monotone profile
  (np.interp on z(phi)) gives the same crossing;
* shifting the profile down by s cells with shift count s leaves the lab height
  unchanged;
* a solid band above the front: the topmost crossing is the one reported;
* no crossing: NaN and zero columns;
* 2D: mean / min / max over columns equal numpy's reductions of per-column
  np.interp crossings;
* the temperature vanishes where the front sits on the isotherm of T_s
  (z = z0 + V t) and changes by dz / l_T when the front moves by dz.
"""
import numpy as np

from paper_2303_09671_amd import inputs as I
from tests.helpers import oracle_params


def _logistic(z, zc):
    return 1.0 / (1.0 + np.exp(np.sqrt(2.0) * (z - zc)))


def _zc(N, dx):
    return (np.arange(N) + 0.5) * dx


def test_front_on_a_face(oracle):
    p, _ = I.config_1d(N=200)
    z0 = 50 * I.DX
    p = dict(p, z0=z0)
    phi = _logistic(_zc(200, I.DX), z0)
    r = oracle.front(oracle_params(oracle, p), phi)
    assert abs(r["z"] - z0) <= 1e-12 and r["ncol"] == 1
    assert abs(r["T"]) <= 1e-14


def test_front_matches_numpy_interp(oracle):
    p, _ = I.config_1d(N=300)
    po = oracle_params(oracle, p)
    z = _zc(300, I.DX)
    for zc in (61.3, 100.05, 133.77):
        phi = _logistic(z, zc)
        ref = np.interp(0.5, phi[::-1], z[::-1])
        r = oracle.front(po, phi)
        assert abs(r["z"] - ref) <= 1e-12, (zc, r["z"], ref)
        assert abs(r["z"] - zc) < 0.05  # linear interpolation of the logistic profile


def test_front_shift_invariant(oracle):
    p, _ = I.config_1d(N=300)
    po = oracle_params(oracle, p)
    z = _zc(300, I.DX)
    phi = _logistic(z, 120.4)
    s = 7
    shifted = np.concatenate([phi[s:], np.zeros(s)])
    a = oracle.front(po, phi)["z"]
    b = oracle.front(po, shifted, shift=s)["z"]
    assert abs(a - b) <= 1e-12


def test_topmost_crossing(oracle):
    p, _ = I.config_1d(N=300)
    po = oracle_params(oracle, p)
    z = _zc(300, I.DX)
    phi = _logistic(z, 80.0)
    band = (z > 150.0) & (z < 170.0)  # a solid band above the liquid gap
    phi = np.where(band, 1.0, phi)
    r = oracle.front(po, phi)
    ref = z[np.nonzero(band)[0][-1]] + 0.5 * I.DX  # its top: 1 -> 0 half way between cells
    assert abs(r["z"] - ref) <= 1e-12


def test_no_crossing(oracle):
    p, _ = I.config_1d(N=100)
    r = oracle.front(oracle_params(oracle, p), np.zeros(100))
    assert np.isnan(r["z"]) and np.isnan(r["T"]) and r["ncol"] == 0


def test_front_2d_reductions(oracle):
    nx, nz = 9, 120
    p, _, _ = I.config_2d(nx=nx, nz=nz)
    z = _zc(nz, I.DX)
    centres = 30.0 + 3.3 * np.sin(np.arange(nx))
    phi = np.stack([_logistic(z, c) for c in centres], axis=1)  # [nz][nx]
    r = oracle.front(oracle_params(oracle, p), phi.ravel())
    cols = np.array([np.interp(0.5, phi[::-1, i], z[::-1]) for i in range(nx)])
    assert r["ncol"] == nx
    assert abs(r["z"] - cols.mean()) <= 1e-12
    assert abs(r["zmin"] - cols.min()) <= 1e-12 and abs(r["zmax"] - cols.max()) <= 1e-12


def test_front_temperature(oracle):
    p, _ = I.config_1d(N=400)
    n = 1000
    t = n * p["dt"]
    z_iso = p["z0"] + p["V"] * t  # the isotherm of T_s at time t
    po = oracle_params(oracle, p)
    z = _zc(400, I.DX)
    r0 = oracle.front(po, _logistic(z, z_iso), n=n)
    assert abs(r0["z"] - z_iso) < 0.05
    r1 = oracle.front(po, _logistic(z, z_iso + 8.0), n=n)
    assert abs((r1["T"] - r0["T"]) - (r1["z"] - r0["z"]) * p["inv_lT"]) <= 1e-14
    assert abs(r0["T"] - (r0["z"] - z_iso) * p["inv_lT"]) <= 1e-14
