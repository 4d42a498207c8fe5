"""Edge and degenerate cases of the forward step through the C ABI.

* Uniform single-phase states (all liquid at (phi, c_s, c_l) = (0, k_e, 1),
  all solid at phi = 1) have no gradients, p'(0) = p'(1) = 0 and a vanishing
  double-well slope, so every rate is exactly zero: the GPU must keep them bit
  for bit (the regularised 1/|grad phi|^2 gives 0, not 0/0), with and without
  the window shift (whose fresh layer is the liquid state).
* Tiny and thin grids (single-cell transverse extents, growth axes shorter than
  a z chunk, tiles much wider than the grid): parity with the oracle at the
  usual 1e-10.
* Zero steps leave the fields and the step counter untouched.

The uniform-phase and tiny-grid cases run for both models: the separate phase
kinetics (model 0) and equal potentials imposed (model 1).  For model 1, a
uniform solid is kept to rounding rather than bit for bit: each step splits
c = c_s through the reciprocal of k_e.
"""
import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I
from tests.helpers import assert_parity, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("dim,phase,V", [(3, "liquid", 0.6), (3, "solid", 0.0), (2, "liquid", 0.8),
                                         (2, "solid", 0.0), (1, "liquid", 0.3), (1, "solid", 0.0)])
def test_uniform_phase_stays_exact(torch_dev, dim, phase, V, model):
    from paper_2303_09671_amd import pf
    torch = torch_dev
    n = {1: (200, 1, 1), 2: (40, 50, 1), 3: (20, 12, 30)}[dim]
    dt = I.run_dt(max(V, 1e-3)) if dim == 1 else 0.2 * I.DX * I.DX / 4.0
    p = I.base_params(dim=dim, n=n, periodic=(1, 1, 0) if dim == 3 else (1, 0, 0), V=V, dt=dt, z0=5 * I.DX,
                      model=model)
    N = int(np.prod(n[:dim]))
    ke = p["ke"]
    if phase == "liquid":
        vals = (0.0, ke, 1.0)
    else:
        vals = (1.0, 0.7, 0.7 / ke)
    f = [_dev(torch, np.full(N, v)) for v in vals]
    print(f"case: uniform {phase} dim={dim} V={V} model={model}", flush=True)
    h = pf.pf_create(p, *f)
    pf.pf_step(h, 150)
    torch.cuda.synchronize()
    assert pf.pf_check(h) == pf.PF_OK
    for x, v in zip(f, vals):
        ref = torch.full((N,), v, dtype=torch.float64)
        if model == 1 and phase == "solid":
            assert torch.allclose(x.cpu(), ref, rtol=1e-13, atol=0.0), (phase, v)
        else:
            assert torch.equal(x.cpu(), ref), (phase, v)


@pytest.mark.parametrize("dim,n,periodic", [
    (3, (1, 1, 9), (1, 1, 0)),     # a 1D column embedded in 3D
    (3, (3, 2, 7), (0, 1, 0)),     # mirror x of width 3
    (3, (33, 9, 5), (1, 0, 0)),    # one cell past a tile in x and y; growth axis < z chunk
    (2, (1, 40, 1), (1, 0, 0)),    # 2D of width 1
    (2, (65, 6, 1), (0, 0, 0)),    # one cell past a 64-wide tile, 6 planes
])
@pytest.mark.parametrize("model", [0, 1])
def test_tiny_grids(torch_dev, oracle, dim, n, periodic, model):
    from paper_2303_09671_amd import pf
    torch = torch_dev
    nz = n[dim - 1]
    p = I.base_params(dim=dim, n=n, periodic=periodic, V=0.5, dt=I.run_dt(0.5) / 4.0, z0=(nz // 3) * I.DX + 0.4,
                      model=model)
    f = [a.ravel() for a in I.planar_front(dim, n, p["dx"], p["z0"], p["ke"], amp=0.05, seed=9)]
    steps = 60
    print(f"case: tiny grid dim={dim} n={n} periodic={periodic} model={model}", flush=True)
    t = [_dev(torch, a) for a in f]
    h = pf.pf_create(p, *t)
    pf.pf_step(h, steps)
    torch.cuda.synchronize()
    g = [x.cpu().numpy() for x in t]
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert ref[3] >= 1  # the window shifted at least once
    assert_parity(g, ref[:3], what=f"tiny {n}")


def test_zero_steps(torch_dev):
    from paper_2303_09671_amd import pf
    torch = torch_dev
    p, _, pert = I.config_3d(n=8)
    p = dict(p, n=(40, 12, 45))
    f = [a.ravel() for a in I.planar_front(3, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=1)]
    t = [_dev(torch, a) for a in f]
    h = pf.pf_create(p, *t)
    pf.pf_set_step(h, 17)
    pf.pf_step(h, 0)
    torch.cuda.synchronize()
    assert pf.pf_get_step(h) == 17
    for x, a in zip(t, f):
        assert np.array_equal(x.cpu().numpy(), a)


def test_api_errors(torch_dev):
    """Invalid calls are rejected with PF_EINVAL before any launch."""
    from paper_2303_09671_amd import pf
    torch = torch_dev
    p, _, pert = I.config_3d(n=8)
    p = dict(p, n=(16, 8, 20))
    f = [_dev(torch, a) for a in I.planar_front(3, p["n"], p["dx"], p["z0"], p["ke"])]
    h = pf.pf_create(p, *f)
    N = f[0].numel()
    lam = [torch.zeros(N, dtype=torch.float64, device="cuda") for _ in range(3)]
    out = [torch.zeros_like(x) for x in lam]
    dth = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PFError) as e:  # no 3D adjoint
        pf.pf_adjoint_step(h, 0, f, lam, out, dth)
    assert e.value.code == pf.PF_EINVAL
    with pytest.raises(pf.PFError) as e:  # trajectory rows shorter than the field
        pf.pf_step_traj(h, 2, [torch.zeros((3, N - 1), dtype=torch.float64, device="cuda") for _ in range(3)])
    assert e.value.code == pf.PF_EINVAL
    # 2D adjoint: output aliasing the input cotangent, and a periodic axis narrower than a tile box
    p2, _, _ = I.config_2d(nx=40, nz=30)
    f2 = [_dev(torch, a.ravel()) for a in I.planar_front(2, p2["n"], p2["dx"], p2["z0"], p2["ke"])]
    h2 = pf.pf_create(p2, *f2)
    l2 = [torch.zeros_like(x) for x in f2]
    with pytest.raises(pf.PFError) as e:
        pf.pf_adjoint_step(h2, 0, f2, l2, [l2[1], torch.zeros_like(l2[0]), torch.zeros_like(l2[0])], dth)
    assert e.value.code == pf.PF_EINVAL
    p3, _, _ = I.config_2d(nx=12, nz=30)
    f3 = [_dev(torch, a.ravel()) for a in I.planar_front(2, p3["n"], p3["dx"], p3["z0"], p3["ke"])]
    h3 = pf.pf_create(p3, *f3)
    l3 = [torch.zeros_like(x) for x in f3]
    with pytest.raises(pf.PFError) as e:
        pf.pf_adjoint_step(h3, 0, f3, l3, [torch.zeros_like(x) for x in l3], dth)
    assert e.value.code == pf.PF_EINVAL
    # a 1D run longer than the persistent kernel holds, and a bad grid
    pl, _ = I.config_1d(N=9000)
    fl = [_dev(torch, a) for a in I.planar_front(1, pl["n"], pl["dx"], pl["z0"], pl["ke"])]
    with pytest.raises(pf.PFError) as e:
        pf.pf_create(pl, *fl)
    assert e.value.code == pf.PF_EINVAL
    with pytest.raises(pf.PFError) as e:
        pf.pf_create(dict(p, n=(16, 8, 2)), *f)
    assert e.value.code == pf.PF_EINVAL
