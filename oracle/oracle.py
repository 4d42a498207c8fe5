"""ctypes binding of the CPU oracle -- TEST INFRASTRUCTURE, NOT THE PRODUCT PATH.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It loads ``oracle/liborc.so`` (built by
``oracle/build.py`` with g++, independent of the HIP library) and exposes:

* :func:`step`      -- advance (phi, c_s, c_l) by n explicit steps
                       (Eqs. cs_nonvar, cl_nonvar, phasefield_nonvar; Sec. V.A);
* :func:`jvp`       -- the same steps on dual numbers: exact directional
                       derivative w.r.t. the fields and theta = (A, M_phi, W);
* :func:`energy`    -- discrete free energy (Eq. model1.1, dilute alloy Eq. dil_linear);
* :func:`solute`    -- total solute, max c and its first index (Eq. model1, k_v of Sec. V.C);
* :func:`front`     -- the phi = 1/2 front (topmost crossing per column) and its
                       temperature (interface temperature of Sec. V.C);
* :func:`pointwise`, :func:`phi_t` and :func:`face_fluxes` -- per-cell and
                       per-face quantities for the pins.

``mutate`` (default 0) plants one known mistake in the oracle so that a test
can show which pin catches it; only the pin tests set it.

Parameters are a plain ``dict`` (see :data:`DEFAULTS`); fields are float64
numpy arrays in the grid layout (axis 0 fastest, growth axis last).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")
LIB_OMP_PATH = os.path.join(_HERE, "liborc_omp.so")

#: Default nondimensional parameters (lengths in W0, time in W0^2/D_l, c in c_inf).
DEFAULTS = dict(
    dim=1, n=(1024, 1, 1), periodic=(0, 0, 0), quintic=1, drag_variant=0, model=0, mutate=0,
    dx=0.8, dt=0.128, W=1.0, Mphi=1.0, lambda0=0.04462, Ds=1e-4, ke=0.14, A=1.2,
    b=1e-4, ap=0.0, inv_lT=1.0 / 444.0, V=0.1, z0=256 * 0.8, eps_grad=3e-3,
)


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
        ("quintic", C.c_int32), ("drag_variant", C.c_int32), ("model", C.c_int32),
        ("mutate", C.c_int32), ("pad_", C.c_int32), ("dx", C.c_double), ("dt", C.c_double), ("W", C.c_double), ("Mphi", C.c_double),
        ("lambda0", C.c_double), ("Ds", C.c_double), ("ke", C.c_double), ("A", C.c_double),
        ("b", C.c_double), ("ap", C.c_double), ("inv_lT", C.c_double), ("V", C.c_double),
        ("z0", C.c_double), ("eps_grad", C.c_double),
    ]


_lib = None
_lib_omp = None


def lib(openmp: bool = False):
    """Load the oracle shared library (raises if it has not been built).
    openmp=True loads the build with OpenMP cell loops (same source and
    results; used only to time the oracle on all host cores)."""
    global _lib, _lib_omp
    if openmp:
        if _lib_omp is None:
            _lib_omp = _load(LIB_OMP_PATH)
        return _lib_omp
    if _lib is None:
        _lib = _load(LIB_PATH)
    return _lib


def _load(path):
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library missing: {path} (run oracle/build.py)")
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.orc_params_size.restype = C.c_int
    L.orc_step.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_long, C.c_long, C.POINTER(C.c_int64)]
    L.orc_step.restype = C.c_int
    L.orc_jvp.argtypes = [C.POINTER(_Params), dp, dp, dp, dp, dp, dp, dp, C.c_long, C.c_long,
                          C.POINTER(C.c_int64)]
    L.orc_jvp.restype = C.c_int
    L.orc_energy.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_long, C.c_int64]
    L.orc_energy.restype = C.c_double
    L.orc_solute.argtypes = [C.POINTER(_Params), dp, dp, dp, dp, dp, C.POINTER(C.c_long)]
    L.orc_solute.restype = C.c_int
    L.orc_pointwise.argtypes = [C.POINTER(_Params), C.c_double, C.c_double, C.c_double, C.c_double, dp]
    L.orc_pointwise.restype = C.c_int
    L.orc_phi_t.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_long, C.c_int64, dp]
    L.orc_phi_t.restype = C.c_int
    L.orc_front.argtypes = [C.POINTER(_Params), dp, C.c_long, C.c_int64, dp]
    L.orc_front.restype = C.c_int
    L.orc_face_fluxes.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_long, C.c_int64, C.c_int, dp, dp, dp, dp]
    L.orc_face_fluxes.restype = C.c_int
    if L.orc_params_size() != C.sizeof(_Params):
        raise RuntimeError("oracle parameter layout mismatch")
    return L


def params(**kw) -> dict:
    """DEFAULTS updated by keyword arguments."""
    p = dict(DEFAULTS)
    unknown = set(kw) - set(p)
    if unknown:
        raise KeyError(f"unknown oracle parameters: {sorted(unknown)}")
    p.update(kw)
    return p


def _cparams(p: dict) -> _Params:
    s = _Params()
    s.dim = int(p["dim"])
    n = list(p["n"]) + [1] * (3 - len(p["n"]))
    per = list(p["periodic"]) + [0] * (3 - len(p["periodic"]))
    for k in range(3):
        s.n[k] = int(n[k])
        s.periodic[k] = int(per[k])
    s.quintic = int(p["quintic"])
    s.drag_variant = int(p["drag_variant"])
    s.model = int(p.get("model", 0))
    s.mutate = int(p.get("mutate", 0))
    for f in ("dx", "dt", "W", "Mphi", "lambda0", "Ds", "ke", "A", "b", "ap", "inv_lT", "V", "z0",
              "eps_grad"):
        setattr(s, f, float(p[f]))
    return s


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ncell(p: dict) -> int:
    n = list(p["n"]) + [1, 1, 1]
    return int(np.prod([n[k] if k < p["dim"] else 1 for k in range(3)]))


def _fields(phi, cs, cl, p):
    out = []
    for a in (phi, cs, cl):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).copy()
        if a.size != _ncell(p):
            raise ValueError("field size does not match the grid")
        out.append(a)
    return out


def step(p: dict, phi, cs, cl, nsteps: int, n0: int = 0, shift: int = 0, openmp: bool = False):
    """Advance copies of the fields by ``nsteps`` steps from step index ``n0``.

    Returns ``(phi, cs, cl, shift)`` with ``shift`` the updated window count.
    openmp=True runs the same steps on all host cores (OMP_NUM_THREADS)."""
    phi, cs, cl = _fields(phi, cs, cl, p)
    s = C.c_int64(int(shift))
    rc = lib(openmp).orc_step(C.byref(_cparams(p)), _ptr(phi), _ptr(cs), _ptr(cl), int(n0), int(nsteps), C.byref(s))
    if rc != 0:
        raise RuntimeError("orc_step failed")
    return phi, cs, cl, int(s.value)


def jvp(p: dict, phi, cs, cl, dphi, dcs, dcl, dtheta, nsteps: int, n0: int = 0, shift: int = 0):
    """Dual-number forward mode: returns ``(u_out(3), du_out(3), shift)``.
    ``dtheta`` is the tangent of theta = (A, M_phi, W, b) (a 3-vector leaves b fixed)."""
    phi, cs, cl = _fields(phi, cs, cl, p)
    dphi, dcs, dcl = _fields(dphi, dcs, dcl, p)
    th = np.zeros(4)
    dth = np.asarray(dtheta, dtype=np.float64).ravel()
    th[:dth.size] = dth
    s = C.c_int64(int(shift))
    rc = lib().orc_jvp(C.byref(_cparams(p)), _ptr(phi), _ptr(cs), _ptr(cl), _ptr(dphi), _ptr(dcs),
                       _ptr(dcl), _ptr(th), int(n0), int(nsteps), C.byref(s))
    if rc != 0:
        raise RuntimeError("orc_jvp failed")
    return (phi, cs, cl), (dphi, dcs, dcl), int(s.value)


def energy(p: dict, phi, cs, cl, n: int = 0, shift: int = 0) -> float:
    phi, cs, cl = _fields(phi, cs, cl, p)
    return float(lib().orc_energy(C.byref(_cparams(p)), _ptr(phi), _ptr(cs), _ptr(cl), int(n), int(shift)))


def solute(p: dict, phi, cs, cl):
    """Returns ``(total, cmax, argmax)``."""
    phi, cs, cl = _fields(phi, cs, cl, p)
    tot, cm, am = C.c_double(), C.c_double(), C.c_long()
    lib().orc_solute(C.byref(_cparams(p)), _ptr(phi), _ptr(cs), _ptr(cl), C.byref(tot), C.byref(cm), C.byref(am))
    return float(tot.value), float(cm.value), int(am.value)


def front(p: dict, phi, n: int = 0, shift: int = 0) -> dict:
    """The phi = 1/2 front: mean, min and max height over the columns that
    cross, (mean - z0 - V n dt) / l_T and the number of crossing columns."""
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).ravel())
    out = np.zeros(5)
    lib().orc_front(C.byref(_cparams(p)), _ptr(phi), int(n), int(shift), _ptr(out))
    return dict(z=out[0], zmin=out[1], zmax=out[2], T=out[3], ncol=int(out[4]))


def face_fluxes(p: dict, phi, cs, cl, k: int, n: int = 0, shift: int = 0):
    """Fluxes through the face between each cell and its neighbour +e_k:
    ``(J_s, J_l, J_mix, p_face)`` (d c/dt = div J convention; zero on
    boundary faces).  J_mix is the equal-potential model's flux (Eq.
    solute_nonvar); J_s, J_l those of the separate-kinetics model."""
    phi, cs, cl = _fields(phi, cs, cl, p)
    js, jl, jm, pf = (np.zeros_like(phi) for _ in range(4))
    rc = lib().orc_face_fluxes(C.byref(_cparams(p)), _ptr(phi), _ptr(cs), _ptr(cl), int(n), int(shift), int(k),
                               _ptr(js), _ptr(jl), _ptr(jm), _ptr(pf))
    if rc != 0:
        raise RuntimeError("orc_face_fluxes failed")
    return js, jl, jm, pf


def pointwise(p: dict, phi: float, cs: float, cl: float, cleq: float) -> dict:
    out = np.zeros(7)
    lib().orc_pointwise(C.byref(_cparams(p)), float(phi), float(cs), float(cl), float(cleq), _ptr(out))
    keys = ("h", "p", "dp", "dfdw", "dmu", "mubar", "dG")
    return dict(zip(keys, out.tolist()))


def phi_t(p: dict, phi, cs, cl, n: int = 0, shift: int = 0) -> np.ndarray:
    phi, cs, cl = _fields(phi, cs, cl, p)
    out = np.zeros_like(phi)
    lib().orc_phi_t(C.byref(_cparams(p)), _ptr(phi), _ptr(cs), _ptr(cl), int(n), int(shift), _ptr(out))
    return out
