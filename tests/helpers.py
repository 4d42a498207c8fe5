"""Shared helpers of the GPU parity tests: parameter dicts for both sides, the
parity metric and oracle runs of batched 1D workloads."""
import numpy as np

from paper_2303_09671_amd import inputs as I

ORACLE_KEYS = ("dim", "n", "periodic", "quintic", "dx", "dt", "W", "Mphi", "lambda0", "Ds", "ke", "A", "b",
               "ap", "inv_lT", "V", "z0", "eps_grad", "model")

TOL = 1e-10  # max relative field error: max|x - ref| / max|ref| per field


def oracle_params(oracle, p: dict) -> dict:
    return oracle.params(**{k: p[k] for k in ORACLE_KEYS if k in p})


def rel_err(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def assert_parity(gpu_fields, ref_fields, tol=TOL, what=""):
    for name, g, r in zip(("phi", "c_s", "c_l"), gpu_fields, ref_fields):
        g = np.asarray(g).ravel()
        r = np.asarray(r).ravel()
        assert np.isfinite(r).all(), f"{what}: oracle {name} not finite"
        e = rel_err(g, r)
        assert e <= tol, f"{what}: {name} max relative error {e:.3e} > {tol:.0e}"


def oracle_batch(oracle, base: dict, runs, nsteps: int, n0: int = 0, fields=None, offsets=None):
    """Run each 1D run separately on the oracle; returns concatenated fields."""
    out = []
    for r_i, r in enumerate(runs):
        p = oracle_params(oracle, dict(base, dim=1, n=(r["N"], 1, 1), V=r["V"], dt=r["dt"], z0=r["z0"]))
        if fields is None:
            f = I.planar_front(1, (r["N"],), base["dx"], r["z0"], base["ke"], base.get("W", 1.0))
        else:
            o = offsets[r_i]
            f = tuple(a[o:o + r["N"]] for a in fields)
        s = int(np.floor(r["V"] * (n0 * r["dt"]) / base["dx"]))
        res = oracle.step(p, *f, nsteps, n0=n0, shift=s)
        out.append(res[:3])
    return out
