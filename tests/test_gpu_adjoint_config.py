"""The adjoint fit workload at its configured size: 64 1D runs (N = 2048, V
log-spaced 1e-2..1) plus one 2D 512^2 run, 10000 steps, checkpoints every 100
steps; loss L = sum (k - k*)^2 against the seeded Aziz-form target curve.
dL/dtheta, theta = (A, M_phi, W, b), from the adjoint must agree with central
finite differences to 1e-5 relative (for b ~ 1e-4 the step is h b, the same
relative step); the argmax cell of every run must not move
between the +h and -h runs (max() is differentiated through it).

Checked at h = 1e-6 (the configured step; bar 1e-5 relative per component)
and, as a cross-check that the agreement is not an artefact of the FD
truncation error, at h = 1e-8.  At h = 1e-8 the quotient carries the rounding
noise of the 10000-step forward, delta L / (2 h) with delta L ~ 1e-14 (a few
1e-7 absolute), so there the floor is 1e-5 of the largest component rather than
of each one.  Both need the step map to be smooth: the regularised
1/|grad phi|^2 = G/(G^2 + eps^2) is (a hard gate at G = eps made the
10000-step map a patchwork of jumps in the far tails).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_adjoint_workload_gradient():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_09671_amd import inputs as I
    from paper_2303_09671_amd import pf
    from paper_2303_09671_amd.adjoint import PartitionCoefficient, Workload, forward_k
    one_d, two_d, k1t, k2t = I.adjoint_workloads()
    wls = [Workload(**one_d), Workload(**two_d)]
    tgts = [torch.tensor(k1t, dtype=torch.float64), torch.tensor([k2t], dtype=torch.float64)]
    base = one_d["params"]
    theta0 = np.array([base["A"], base["Mphi"], base["W"], base["b"]])
    scale = np.array([1.0, 1.0, 1.0, base["b"]])  # FD step of each component = h * scale
    for wl, kt, name in zip(wls, tgts, ("1D x64", "2D 512^2")):
        print(f"case: adjoint workload {name}", flush=True)
        theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
        k = PartitionCoefficient.apply(theta, wl)
        assert torch.isfinite(k).all()
        L = ((k - kt) ** 2).sum()
        L.backward()
        g = theta.grad.numpy()
        fds = {}
        for h in (1e-8, 1e-6):
            fd = np.zeros(4)
            for i in range(4):
                tp, tm = theta0.copy(), theta0.copy()
                tp[i] += h * scale[i]
                tm[i] -= h * scale[i]
                kp, hp, _, _ = forward_k(wl, tp)
                km, hm, _, _ = forward_k(wl, tm)
                if True:
                    assert np.array_equal(pf.pf_solute(hp)[2], pf.pf_solute(hm)[2]), "argmax moved"
                fd[i] = (((kp - kt) ** 2).sum() - ((km - kt) ** 2).sum()).item() / (2 * h * scale[i])
            fds[h] = fd
        print(f"  grad {g} fd(1e-6) {fds[1e-6]} fd(1e-8) {fds[1e-8]}", flush=True)
        for h, fd in fds.items():
            floor = 1e-9 if h == 1e-6 else 1e-5  # relative to max |fd|: FD rounding noise at h = 1e-8
            for i in range(4):
                # the noise floor of component i scales with 1/scale[i]
                fl = floor * np.abs(fd[:3] * scale[:3]).max() / scale[i]
                assert abs(g[i] - fd[i]) <= 1e-5 * abs(fd[i]) + fl, (name, h, i, g, fd)
