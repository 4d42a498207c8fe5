"""The 1D workload at the paper's operating point A = 2 (Sec. V.D) on the GPU.

At A = 2 the front dynamics amplify perturbations: on the oracle, a relative
perturbation of 1e-15 of the initial state stays below 1e-12 for the first
8000 steps and then grows about 10x per 1000 steps.  Two implementations that
round differently therefore agree to 1e-10 over that first stretch only, and
that is where the parity bar applies (8000 steps, elementwise against the
oracle).  The configured 20000 steps are checked for what holds at any
rounding: finite, positive concentrations, a front inside the window and a
partition coefficient between k_e and 1, as on the oracle.
"""
import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I
from tests.helpers import assert_parity, oracle_params

pytestmark = pytest.mark.gpu


def _run(torch, p, steps):
    from paper_2303_09671_amd import pf
    f = [torch.from_numpy(a.ravel().copy()).cuda() for a in I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])]
    h = pf.pf_create(p, *f)
    pf.pf_step(h, steps)
    torch.cuda.synchronize()
    return h, [t.cpu().numpy() for t in f]


def test_a2_parity_over_the_stable_stretch(oracle):
    import torch
    p, _ = I.config_1d_a2()
    steps = 8000
    print(f"case: 1D A = {p['A']} parity, {steps} steps", flush=True)
    _, g = _run(torch, p, steps)
    f0 = I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])
    ref = oracle.step(oracle_params(oracle, p), *f0, steps)
    assert_parity(g, ref[:3], what=f"1D A=2, {steps} steps")


def test_a2_full_run_is_physical():
    import torch
    from paper_2303_09671_amd import pf
    p, steps = I.config_1d_a2()
    print(f"case: 1D A = {p['A']}, full {steps} steps", flush=True)
    h, g = _run(torch, p, steps)
    assert pf.pf_check(h) == pf.PF_OK
    assert all(np.isfinite(a).all() for a in g) and g[1].min() > 0 and g[2].min() > 0
    _, cm, _ = pf.pf_solute(h)
    assert p["ke"] < 1.0 / cm[0] < 1.0
    fr = pf.pf_front(h)
    assert fr["ncol"][0] == 1
