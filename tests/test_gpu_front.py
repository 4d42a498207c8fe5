"""GPU front diagnostic (pf_front through the C ABI) against the oracle's,
evaluated on the same fields (the GPU state copied to the host), so the
crossing index -- an integer decided by FP64 comparisons -- must agree exactly
and the heights to rounding.  Batched 1D runs with window shifts, 2D and 3D
grids after shifts, and a state with no crossing."""
import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I
from tests.helpers import oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def _close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(b), 1.0)


def test_front_batch(torch_dev, oracle):
    from paper_2303_09671_amd import pf
    runs = [dict(N=N, V=V, dt=I.run_dt(V), z0=(N // 4) * I.DX) for N, V in ((600, 0.3), (1500, 0.05), (3001, 0.6))]
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    t = [_dev(torch_dev, a) for a in (phi, cs, cl)]
    h = pf.pf_create(base, *t, runs=runs, offsets=offs)
    steps = 700
    print(f"case: front batch steps={steps}", flush=True)
    pf.pf_step(h, steps)
    g = pf.pf_front(h)
    ph = t[0].cpu().numpy()
    for i, (r, o) in enumerate(zip(runs, offs)):
        po = oracle_params(oracle, dict(base, n=(r["N"], 1, 1), V=r["V"], dt=r["dt"], z0=r["z0"]))
        s = int(np.floor(r["V"] * (steps * r["dt"]) / base["dx"]))
        ref = oracle.front(po, ph[o:o + r["N"]], n=steps, shift=s)
        assert g["ncol"][i] == ref["ncol"] == 1
        assert _close(g["z"][i], ref["z"]) and _close(g["T"][i], ref["T"], 1e-10), (i, g, ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_front_grid(torch_dev, oracle, dim):
    from paper_2303_09671_amd import pf
    if dim == 2:
        p, _, pert = I.config_2d(nx=150, nz=75)
        p = dict(p, V=0.5)
        steps = 260
    else:
        p, _, pert = I.config_3d(n=8)
        p = dict(p, n=(40, 12, 45), V=0.6, z0=14 * 0.8)
        steps = 90
    f = [a.ravel() for a in I.planar_front(dim, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
    t = [_dev(torch_dev, a) for a in f]
    h = pf.pf_create(p, *t)
    print(f"case: front {dim}D steps={steps}", flush=True)
    pf.pf_step(h, steps)
    g = pf.pf_front(h)
    s = int(np.floor(p["V"] * (steps * p["dt"]) / p["dx"]))
    assert s >= 1
    ref = oracle.front(oracle_params(oracle, p), t[0].cpu().numpy(), n=steps, shift=s)
    assert g["ncol"][0] == ref["ncol"] == int(np.prod(p["n"][:dim - 1]))
    assert _close(g["z"][0], ref["z"]) and _close(g["zmin"][0], ref["zmin"]) and _close(g["zmax"][0], ref["zmax"])
    assert _close(g["T"][0], ref["T"], 1e-10)


def test_front_none(torch_dev):
    from paper_2303_09671_amd import pf
    p, _, _ = I.config_2d(nx=40, nz=30)
    N = 40 * 30
    t = [_dev(torch_dev, np.full(N, v)) for v in (0.0, p["ke"], 1.0)]
    h = pf.pf_create(p, *t)
    g = pf.pf_front(h)
    assert g["ncol"][0] == 0 and np.isnan(g["z"][0]) and np.isnan(g["T"][0])
