"""Thin ctypes binding of the HIP library ``libpf.so`` (C ABI of ``include/pf.h``).

Argument marshalling only: torch supplies device memory (float64 CUDA/HIP
tensors) and the stream; every step of the method runs in the library's
kernels.  The functions carry the C names (``pf_create``, ``pf_step``, ...).
Loading fails loudly if the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")

PF_OK, PF_EINVAL, PF_EUNSTABLE_DT, PF_ENONFINITE, PF_ENEGCONC, PF_EDEVICE, PF_ENOMEM = 0, -1, -2, -3, -4, -5, -6

#: C symbols the header declares (checked by the CPU test of the library).
EXPORTS = ("pf_create", "pf_step", "pf_step_traj", "pf_get_step", "pf_set_step", "pf_energy", "pf_solute",
           "pf_front", "pf_check", "pf_adjoint_step", "pf_adjoint_segment", "pf_kv_seed", "pf_destroy", "pf_strerror",
           "pf_last_error_detail", "pf_solute_noalloc")


class PFError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


class pf_params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3), ("quintic", C.c_int32),
        ("shift", C.c_int32), ("check_every", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double), ("W", C.c_double), ("Mphi", C.c_double),
        ("lambda0", C.c_double), ("Ds", C.c_double), ("ke", C.c_double), ("A", C.c_double),
        ("b", C.c_double), ("ap", C.c_double), ("inv_lT", C.c_double), ("V", C.c_double),
        ("z0", C.c_double), ("eps_grad", C.c_double),
        ("nbatch", C.c_int32), ("model", C.c_int32),
        ("run_n", C.POINTER(C.c_int32)), ("run_off", C.POINTER(C.c_int64)), ("run_V", C.POINTER(C.c_double)),
        ("run_dt", C.POINTER(C.c_double)), ("run_z0", C.POINTER(C.c_double)),
    ]


_lib = None


def lib() -> C.CDLL:
    """Load libpf.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2303_09671_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
        L.pf_create.argtypes = [C.POINTER(pf_params), vp, vp, vp, vp, C.POINTER(vp)]
        L.pf_step.argtypes = [vp, i64]
        L.pf_step_traj.argtypes = [vp, i64, vp, vp, vp, i64]
        L.pf_get_step.argtypes = [vp, C.POINTER(i64)]
        L.pf_set_step.argtypes = [vp, i64]
        L.pf_energy.argtypes = [vp, dp]
        L.pf_solute.argtypes = [vp, dp, dp, C.POINTER(i64)]
        L.pf_front.argtypes = [vp, dp, dp, dp, dp, C.POINTER(i64)]
        L.pf_solute_noalloc.argtypes = [C.POINTER(pf_params), vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.pf_check.argtypes = [vp]
        L.pf_adjoint_step.argtypes = [vp, i64, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
        L.pf_adjoint_segment.argtypes = [vp, i64, i64, vp, vp, vp, i64, C.POINTER(vp), C.POINTER(vp), vp]
        L.pf_kv_seed.argtypes = [vp, dp, C.POINTER(vp)]
        L.pf_destroy.argtypes = [vp]
        L.pf_destroy.restype = None
        L.pf_strerror.argtypes = [C.c_int]
        L.pf_strerror.restype = C.c_char_p
        L.pf_last_error_detail.argtypes = []
        L.pf_last_error_detail.restype = C.c_char_p
        for name in ("pf_create", "pf_step", "pf_step_traj", "pf_get_step", "pf_set_step", "pf_energy",
                     "pf_solute", "pf_front", "pf_check", "pf_adjoint_step", "pf_adjoint_segment", "pf_kv_seed",
                     "pf_solute_noalloc"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != PF_OK:
        raise PFError(rc, where, lib().pf_last_error_detail().decode())


def _dev_ptr(t) -> int:
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("fields must be contiguous float64 device tensors")
    return t.data_ptr()


class Handle:
    """An open pf_handle plus the objects whose memory it references."""

    def __init__(self, ptr: int, fields, params: dict, nrun: int, keep, stream=None):
        self.ptr = C.c_void_p(ptr)
        self.fields = fields
        self.params = params
        self.nrun = nrun
        self.stream = stream  # the torch stream every call of this handle is ordered on
        self._keep = keep

    def __del__(self):
        try:
            pf_destroy(self)
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def _make_params(p: dict, runs=None, offsets=None):
    s = pf_params()
    s.dim = int(p["dim"])
    n = list(p["n"]) + [1, 1, 1]
    per = list(p.get("periodic", (0, 0, 0))) + [0, 0, 0]
    for k in range(3):
        s.n[k] = int(n[k])
        s.periodic[k] = int(per[k])
    s.quintic = int(p.get("quintic", 1))
    s.shift = int(p.get("shift", 1))
    s.check_every = int(p.get("check_every", 0))
    s.model = int(p.get("model", 0))
    for f in ("dx", "dt", "W", "Mphi", "lambda0", "Ds", "ke", "A", "b", "ap", "inv_lT", "V", "z0", "eps_grad"):
        setattr(s, f, float(p[f]))
    keep = []
    if runs is not None:
        s.nbatch = len(runs)
        rn = np.ascontiguousarray([r["N"] for r in runs], dtype=np.int32)
        ro = np.ascontiguousarray(offsets, dtype=np.int64)
        rv = np.ascontiguousarray([r["V"] for r in runs], dtype=np.float64)
        rdt = np.ascontiguousarray([r["dt"] for r in runs], dtype=np.float64)
        rz = np.ascontiguousarray([r["z0"] for r in runs], dtype=np.float64)
        keep = [rn, ro, rv, rdt, rz]
        s.run_n = rn.ctypes.data_as(C.POINTER(C.c_int32))
        s.run_off = ro.ctypes.data_as(C.POINTER(C.c_int64))
        s.run_V = rv.ctypes.data_as(C.POINTER(C.c_double))
        s.run_dt = rdt.ctypes.data_as(C.POINTER(C.c_double))
        s.run_z0 = rz.ctypes.data_as(C.POINTER(C.c_double))
    return s, keep


def pf_create(params: dict, phi, cs, cl, stream=None, runs=None, offsets=None) -> Handle:
    """Open a handle over device tensors (phi, cs, cl).  ``runs``/``offsets``
    select batched 1D mode (list of dicts with N, V, dt, z0)."""
    import torch
    s, keep = _make_params(params, runs, offsets)
    if stream is None:
        stream = torch.cuda.current_stream()
    out = C.c_void_p()
    rc = lib().pf_create(C.byref(s), C.c_void_p(_dev_ptr(phi)), C.c_void_p(_dev_ptr(cs)), C.c_void_p(_dev_ptr(cl)),
                         C.c_void_p(stream.cuda_stream), C.byref(out))
    _check(rc, "pf_create")
    return Handle(out.value, (phi, cs, cl), dict(params), len(runs) if runs is not None else 1, keep + [stream],
                  stream)


def pf_step(h: Handle, nsteps: int):
    _check(lib().pf_step(h.ptr, int(nsteps)), "pf_step")


def pf_step_traj(h: Handle, nsteps: int, traj):
    """traj: three device tensors of shape (nsteps + 1, stride)."""
    stride = traj[0].shape[1]
    _check(lib().pf_step_traj(h.ptr, int(nsteps), C.c_void_p(_dev_ptr(traj[0])), C.c_void_p(_dev_ptr(traj[1])),
                              C.c_void_p(_dev_ptr(traj[2])), int(stride)), "pf_step_traj")


def pf_get_step(h: Handle) -> int:
    n = C.c_int64()
    _check(lib().pf_get_step(h.ptr, C.byref(n)), "pf_get_step")
    return int(n.value)


def pf_set_step(h: Handle, n: int):
    _check(lib().pf_set_step(h.ptr, int(n)), "pf_set_step")


def pf_energy(h: Handle) -> np.ndarray:
    out = np.zeros(h.nrun)
    _check(lib().pf_energy(h.ptr, out.ctypes.data_as(C.POINTER(C.c_double))), "pf_energy")
    return out


def pf_solute(h: Handle):
    """Returns (total, cmax, argmax) arrays (one entry per run)."""
    tot = np.zeros(h.nrun)
    cm = np.zeros(h.nrun)
    am = np.zeros(h.nrun, dtype=np.int64)
    _check(lib().pf_solute(h.ptr, tot.ctypes.data_as(C.POINTER(C.c_double)), cm.ctypes.data_as(C.POINTER(C.c_double)),
                           am.ctypes.data_as(C.POINTER(C.c_int64))), "pf_solute")
    return tot, cm, am


def pf_solute_noalloc(params: dict, phi, cs, cl, n: int, out, stream=None):
    """Handle-free, allocation-free diagnostics of one domain: writes
    (total, c_max, argmax, energy) into the device tensors ``out`` =
    (float64[1], float64[1], int64[1], float64[1]) asynchronously on the stream."""
    import torch
    s, _ = _make_params(params)
    if stream is None:
        stream = torch.cuda.current_stream()
    for t, dt in zip(out, (torch.float64, torch.float64, torch.int64, torch.float64)):
        if not (t.is_cuda and t.dtype == dt and t.numel() >= 1):
            raise TypeError("outputs must be device tensors (float64, float64, int64, float64)")
    _check(lib().pf_solute_noalloc(C.byref(s), C.c_void_p(_dev_ptr(phi)), C.c_void_p(_dev_ptr(cs)),
                                   C.c_void_p(_dev_ptr(cl)), int(n), C.c_void_p(stream.cuda_stream),
                                   C.c_void_p(out[0].data_ptr()), C.c_void_p(out[1].data_ptr()),
                                   C.c_void_p(out[2].data_ptr()), C.c_void_p(out[3].data_ptr())), "pf_solute_noalloc")


def pf_front(h: Handle) -> dict:
    """The phi = 1/2 front: arrays (one entry per run) z, zmin, zmax, T, ncol."""
    z, zmin, zmax, T = (np.zeros(h.nrun) for _ in range(4))
    nc = np.zeros(h.nrun, dtype=np.int64)
    dpp = C.POINTER(C.c_double)
    _check(lib().pf_front(h.ptr, z.ctypes.data_as(dpp), zmin.ctypes.data_as(dpp), zmax.ctypes.data_as(dpp),
                          T.ctypes.data_as(dpp), nc.ctypes.data_as(C.POINTER(C.c_int64))), "pf_front")
    return dict(z=z, zmin=zmin, zmax=zmax, T=T, ncol=nc)


def pf_check(h: Handle) -> int:
    """Error word since the last check: PF_OK, PF_ENONFINITE or PF_ENEGCONC."""
    return int(lib().pf_check(h.ptr))


def _ptr3(ts):
    arr = (C.c_void_p * 3)()
    for k in range(3):
        arr[k] = _dev_ptr(ts[k])
    return arr


def pf_adjoint_step(h: Handle, n: int, u_n, lam_np1, lam_n, dtheta):
    _check(lib().pf_adjoint_step(h.ptr, int(n), _ptr3(u_n), _ptr3(lam_np1), _ptr3(lam_n),
                                 C.c_void_p(_dev_ptr(dtheta))), "pf_adjoint_step")


def pf_adjoint_segment(h: Handle, n0: int, m: int, traj, lam, work, dtheta):
    """traj: three device tensors of shape (>= m, stride) (row j = state at step
    n0 + j); lam: lam^{n0+m} in, lam^{n0} out; work: three scratch fields."""
    stride = traj[0].shape[1]
    _check(lib().pf_adjoint_segment(h.ptr, int(n0), int(m), C.c_void_p(_dev_ptr(traj[0])),
                                    C.c_void_p(_dev_ptr(traj[1])), C.c_void_p(_dev_ptr(traj[2])), int(stride),
                                    _ptr3(lam), _ptr3(work), C.c_void_p(_dev_ptr(dtheta))), "pf_adjoint_segment")


def pf_kv_seed(h: Handle, dL_dk, lam):
    d = np.ascontiguousarray(np.asarray(dL_dk, dtype=np.float64).reshape(h.nrun))
    _check(lib().pf_kv_seed(h.ptr, d.ctypes.data_as(C.POINTER(C.c_double)), _ptr3(lam)), "pf_kv_seed")


def pf_destroy(h: Handle):
    if h.ptr is not None and h.ptr.value:
        lib().pf_destroy(h.ptr)
        h.ptr = C.c_void_p()


def pf_strerror(code: int) -> str:
    return lib().pf_strerror(int(code)).decode()
