"""pf_solute_noalloc (the allocation-free, handle-free diagnostics entry point)
against pf_solute / pf_energy of a handle, through the C ABI.

Both run the same reduction kernels in the same order, so the results agree
exactly.  Two calls in a row on one GPU, the second on a smaller grid, check
that the shared static scratch carries nothing over from the first call."""
import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I

pytestmark = pytest.mark.gpu


def _case(torch, nx, nz, steps, seed):
    from paper_2303_09671_amd import pf
    p, _, pert = I.config_2d(nx=nx, nz=nz, seed=seed)
    f = [torch.from_numpy(a.ravel().copy()).cuda() for a in
         I.planar_front(2, p["n"], p["dx"], p["z0"], p["ke"], amp=0.02, seed=pert["seed"])]
    h = pf.pf_create(p, *f)
    pf.pf_step(h, steps)
    tot, cm, am = pf.pf_solute(h)
    en = pf.pf_energy(h)
    out = (torch.full((1,), np.nan, dtype=torch.float64, device="cuda"),
           torch.full((1,), np.nan, dtype=torch.float64, device="cuda"),
           torch.full((1,), -7, dtype=torch.int64, device="cuda"),
           torch.full((1,), np.nan, dtype=torch.float64, device="cuda"))
    pf.pf_solute_noalloc(p, *f, steps, out)
    torch.cuda.synchronize()
    got = [o.cpu().numpy()[0] for o in out]
    assert got[0] == tot[0] and got[1] == cm[0] and got[2] == am[0] and got[3] == en[0], (got, tot, cm, am, en)
    return got


def test_noalloc_matches_handle_twice():
    import torch
    print("case: pf_solute_noalloc 2D 300x400 then 70x48", flush=True)
    big = _case(torch, 300, 400, 60, 1)
    small = _case(torch, 70, 48, 30, 2)
    assert small[0] < big[0]  # the second call reduced the smaller grid only


def test_noalloc_rejects_oversize_and_bad_args():
    import torch
    from paper_2303_09671_amd import pf
    p, _, _ = I.config_3d(n=8)
    p = dict(p, n=(1024, 1024, 300))  # 3.1e8 cells > 2^28: rejected before any field is read
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = (t[0:1], t[1:2], torch.zeros(1, dtype=torch.int64, device="cuda"), t[2:3])
    with pytest.raises(pf.PFError) as e:
        pf.pf_solute_noalloc(p, t, t, t, 0, out)
    assert e.value.code == pf.PF_EINVAL and "exceed" in str(e.value)
    with pytest.raises(pf.PFError) as e:
        pf.pf_solute_noalloc(dict(p, n=(8, 8, 8), ke=1.5), t, t, t, 0, out)
    assert e.value.code == pf.PF_EINVAL
