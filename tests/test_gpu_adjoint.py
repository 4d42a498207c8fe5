"""GPU adjoint step (pf_adjoint_step through the C ABI) against the oracle.

* Transpose test: for a realistic state u (a front after some steps), random
  cotangent lam and tangents (du, dtheta), the GPU's <J^T lam, du> +
  <dL/dtheta, dtheta> equals the oracle's <lam, J du + J_theta dtheta>, where
  the oracle's J du is its exact dual-number JVP of the same step.  Each theta
  component (A, M_phi, W, b) is checked on its own.  Cases: 1D single run with and without a
  window shift at the step, two batched runs, 2D periodic and mirror x.
* Gradient test: dL/dtheta of L = sum_r (k_r - k*_r)^2 over checkpointed runs
  (autograd Function, replay + adjoint) against central finite differences of
  the GPU forward with h = 1e-6: relative error <= 1e-5.
"""
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


def _transpose_check(torch, oracle, p, fields, n, s, seed, runs=None, offsets=None, oracle_runs=None):
    """fields: state at step n (host).  Returns nothing; asserts."""
    from paper_2303_09671_amd import pf
    rng = np.random.default_rng(seed)
    N = fields[0].size
    phi = fields[0]
    lam = [rng.standard_normal(N), rng.standard_normal(N) * 0.3, rng.standard_normal(N) * 0.1]
    du = [rng.standard_normal(N) * 4 * phi * (1 - phi), rng.standard_normal(N) * 0.1 * fields[1],
          rng.standard_normal(N) * 0.1 * fields[2]]
    # GPU: lam_n = J^T lam, dtheta
    t = [_dev(torch, a) for a in fields]
    h = pf.pf_create(p, *t, runs=runs, offsets=offsets)
    lt = [_dev(torch, a) for a in lam]
    lo = [torch.empty_like(x) for x in lt]
    dth = torch.zeros(4, dtype=torch.float64, device="cuda")
    pf.pf_adjoint_step(h, n, t, lt, lo, dth)
    torch.cuda.synchronize()
    lam_n = [x.cpu().numpy() for x in lo]
    g_theta = dth.cpu().numpy()
    # oracle JVPs (per run in batched mode)
    def jvp(dvec, dtheta):
        if oracle_runs is None:
            _, out, _ = oracle.jvp(oracle_params(oracle, p), *fields, *dvec, dtheta, 1, n0=n, shift=s)
            return out
        outs = [np.zeros(N) for _ in range(3)]
        for (po, sr), r, o in zip(oracle_runs, runs, offsets):
            sl = slice(o, o + r["N"])
            _, out, _ = oracle.jvp(po, *(a[sl] for a in fields), *(d[sl] for d in dvec), dtheta, 1, n0=n, shift=sr)
            for f in range(3):
                outs[f][sl] = out[f]
        return outs
    mask = np.ones(N, dtype=bool)
    if runs is not None:  # cells between runs (alignment padding) are not part of any run
        mask[:] = False
        for r, o in zip(runs, offsets):
            mask[o:o + r["N"]] = True
    Jdu = jvp(du, [0.0, 0.0, 0.0, 0.0])
    lhs = sum(np.dot(lam_n[f][mask], du[f][mask]) for f in range(3))
    rhs = sum(np.dot(lam[f][mask], Jdu[f][mask]) for f in range(3))
    scale = sum(np.abs(lam_n[f][mask] * du[f][mask]).sum() for f in range(3))
    assert abs(lhs - rhs) <= 1e-11 * scale + 1e-14, (lhs, rhs, scale)
    for i in range(4):  # theta = (A, M_phi, W, b)
        e = [0.0, 0.0, 0.0, 0.0]
        e[i] = 1.0
        Jt = jvp([np.zeros(N)] * 3, e)
        ref = sum(np.dot(lam[f][mask], Jt[f][mask]) for f in range(3))
        sc = sum(np.abs(lam[f][mask] * Jt[f][mask]).sum() for f in range(3))
        assert abs(g_theta[i] - ref) <= 1e-10 * sc + 1e-14, (i, g_theta[i], ref, sc)


# step 62 -> 63 shifts the window (V dt / dx = 1/62.5)
@pytest.mark.parametrize("nstep,quintic,ap", [(40, 1, 0.0), (62, 1, 0.0), (62, 0, -1.5)])
def test_transpose_1d(torch_dev, oracle, nstep, quintic, ap):
    p, _ = I.config_1d(N=160)
    p = dict(p, z0=50 * I.DX, quintic=quintic, ap=ap)
    f0 = I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])
    f = oracle.step(oracle_params(oracle, p), *f0, nstep)
    print(f"case: 1D transpose n={nstep} quintic={quintic} ap={ap}", flush=True)
    _transpose_check(torch_dev, oracle, p, f[:3], nstep, f[3], seed=nstep)


def test_transpose_batch(torch_dev, oracle):
    runs = [dict(N=150, V=0.3, dt=I.run_dt(0.3), z0=40 * I.DX), dict(N=300, V=0.05, dt=I.run_dt(0.05), z0=80 * I.DX)]
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    nstep = 33
    state = [phi.copy(), cs.copy(), cl.copy()]
    oruns = []
    for r, o in zip(runs, offs):
        po = oracle_params(oracle, dict(base, n=(r["N"], 1, 1), V=r["V"], dt=r["dt"], z0=r["z0"]))
        sl = slice(o, o + r["N"])
        res = oracle.step(po, phi[sl], cs[sl], cl[sl], nstep)
        for k in range(3):
            state[k][sl] = res[k]
        oruns.append((po, res[3]))
    print("case: batch transpose", flush=True)
    _transpose_check(torch_dev, oracle, base, state, nstep, None, seed=5, runs=runs, offsets=offs, oracle_runs=oruns)


@pytest.mark.parametrize("periodic,nx,V,quintic,ap", [(1, 24, 0.05, 1, 0.0), (0, 20, 0.8, 1, 0.0),
                                                      (1, 40, 0.8, 1, 0.0), (0, 20, 0.8, 0, -1.5),
                                                      (1, 24, 0.8, 1, -2.0)])
def test_transpose_2d(torch_dev, oracle, periodic, nx, V, quintic, ap):
    """Also cubic h and a_p != 0 (the adjoint kernels are compiled separately
    for a_p = 0 and a_p != 0)."""
    p, _, pert = I.config_2d(nx=nx, nz=48)
    p = dict(p, periodic=(periodic, 0, 0), V=V, z0=14 * I.DX, quintic=quintic, ap=ap)
    f0 = [a.ravel() for a in I.planar_front(2, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=3)]
    nstep = 31  # with V = 0.8 the step 31 -> 32 shifts the window (V dt / dx = 1/31.25)
    f = oracle.step(oracle_params(oracle, p), *f0, nstep)
    print(f"case: 2D transpose periodic={periodic} nx={nx} V={V} quintic={quintic} ap={ap} shift_count={f[3]}",
          flush=True)
    _transpose_check(torch_dev, oracle, p, f[:3], nstep, f[3], seed=7)


def test_gradient_vs_finite_difference(torch_dev):
    from paper_2303_09671_amd.adjoint import PartitionCoefficient, Workload, forward_k
    torch = torch_dev
    runs = [dict(N=256, V=V, dt=I.run_dt(V), z0=64 * I.DX) for V in (0.05, 0.2, 0.6)]
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    wl = Workload(params=base, fields0=(phi, cs, cl), nsteps=450, every=100, runs=runs, offsets=offs)
    ktgt = torch.tensor([0.2, 0.25, 0.3], dtype=torch.float64)
    theta = torch.tensor([base["A"], base["Mphi"], base["W"], base["b"]], dtype=torch.float64, requires_grad=True)
    print("case: gradient vs FD (3 runs x 450 steps), theta = (A, M_phi, W, b)", flush=True)
    k = PartitionCoefficient.apply(theta, wl)
    L = ((k - ktgt) ** 2).sum()
    L.backward()
    g = theta.grad.numpy()
    hs = [1e-6, 1e-6, 1e-6, 1e-6 * base["b"]]  # b ~ 1e-4: the same relative step
    fd = np.zeros(4)
    for i in range(4):
        tp = theta.detach().numpy().copy()
        tm = tp.copy()
        tp[i] += hs[i]
        tm[i] -= hs[i]
        kp = forward_k(wl, tp)[0]
        km = forward_k(wl, tm)[0]
        fd[i] = (((kp - ktgt) ** 2).sum() - ((km - ktgt) ** 2).sum()).item() / (2 * hs[i])
    print(f"  grad {g} fd {fd}", flush=True)
    for i in range(4):
        assert abs(g[i] - fd[i]) <= 1e-5 * abs(fd[i]) + 1e-8 * np.abs(fd[:3]).max(), (i, g, fd)


@pytest.mark.parametrize("dim,m", [(1, 7), (2, 6)])
def test_segment_matches_steps(torch_dev, dim, m):
    """pf_adjoint_segment over m replayed steps equals m pf_adjoint_step calls
    to rounding order: the same kernels run, but the LDS scatter of the tiles
    adds contributions in thread-arrival order, and dtheta carries the
    per-block sums over the segment before reducing."""
    from paper_2303_09671_amd import pf
    torch = torch_dev
    if dim == 1:
        runs = [dict(N=300, V=0.3, dt=I.run_dt(0.3), z0=60 * I.DX), dict(N=520, V=0.05, dt=I.run_dt(0.05), z0=90 * I.DX)]
        p = I.base_params(dim=1)
        phi, cs, cl, offs = I.batch_fields(runs)
        f = [_dev(torch, a) for a in (phi, cs, cl)]
        h = pf.pf_create(p, *f, runs=runs, offsets=offs)
        mask = torch.zeros(phi.size, dtype=torch.bool)  # run cells (not the alignment padding)
        for r, o in zip(runs, offs):
            mask[o:o + r["N"]] = True
    else:
        p, _, pert = I.config_2d(nx=48, nz=40)
        p = dict(p, V=0.8, z0=12 * I.DX)
        f = [_dev(torch, a.ravel()) for a in I.planar_front(2, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=3)]
        h = pf.pf_create(p, *f)
        mask = torch.ones(f[0].numel(), dtype=torch.bool)
    print(f"case: segment vs steps dim={dim} m={m}", flush=True)
    n0 = 29  # the 2D window shifts at step 31 -> 32 (V dt / dx = 1/31.25)
    pf.pf_step(h, n0)
    N = f[0].numel()
    traj = [torch.empty((m + 1, N), dtype=torch.float64, device="cuda") for _ in range(3)]
    pf.pf_step_traj(h, m, traj)
    g = torch.Generator(device="cpu").manual_seed(11)
    lam_end = [torch.randn(N, generator=g, dtype=torch.float64).cuda() for _ in range(3)]
    a = [x.clone() for x in lam_end]
    b = [torch.empty_like(x) for x in lam_end]
    th_steps = torch.zeros(4, dtype=torch.float64, device="cuda")
    for j in reversed(range(m)):
        pf.pf_adjoint_step(h, n0 + j, [traj[k][j] for k in range(3)], a, b, th_steps)
        a, b = b, a
    lam = [x.clone() for x in lam_end]
    work = [torch.empty_like(x) for x in lam_end]
    th_seg = torch.zeros(4, dtype=torch.float64, device="cuda")
    pf.pf_adjoint_segment(h, n0, m, traj, lam, work, th_seg)
    torch.cuda.synchronize()
    for k in range(3):
        x, y = lam[k].cpu()[mask].numpy(), a[k].cpu()[mask].numpy()
        assert np.max(np.abs(x - y)) <= 1e-13 * np.max(np.abs(y)), k
    ts, tg = th_steps.cpu().numpy(), th_seg.cpu().numpy()
    assert np.all(np.abs(ts - tg) <= 1e-13 * np.abs(ts).max()), (ts, tg)


@pytest.mark.parametrize("dim", [1, 2])
def test_profile_loss_gradient_vs_finite_difference(torch_dev, dim):
    """An interface-profile loss on the final fields, L = sum w (phi - phi*)^2 +
    sum w (c - c*)^2 with the mixture concentration c = p c_s + (1 - p) c_l
    (Eq. model1) and targets from a run at another theta, differentiated
    through FinalState (torch supplies dL/du, the library's adjoint the rest),
    against central differences with h = 1e-6.  (A loss on a phase
    concentration alone would also weigh its ghost values -- c_l deep in the
    solid, c_s deep in the liquid -- which carry rounding noise amplified by
    the regularised 1/|grad phi|^2 of the far tails; central differences of
    such a loss do not converge as h -> 0, while the mixture c suppresses them
    by p or 1 - p.)"""
    from paper_2303_09671_amd.adjoint import FinalState, Workload
    torch = torch_dev
    if dim == 1:
        runs = [dict(N=300, V=V, dt=I.run_dt(V), z0=80 * I.DX) for V in (0.1, 0.4)]
        base = I.base_params(dim=1)
        phi, cs, cl, offs = I.batch_fields(runs)
        wl = Workload(params=base, fields0=(phi, cs, cl), nsteps=350, every=100, runs=runs, offsets=offs)
        mask = torch.zeros(phi.size, dtype=torch.float64)
        for r, o in zip(runs, offs):
            mask[o:o + r["N"]] = 1.0
    else:
        p, _, pert = I.config_2d(nx=48, nz=40)
        p = dict(p, V=0.5, z0=12 * I.DX)
        f = tuple(a.ravel() for a in I.planar_front(2, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=3))
        wl = Workload(params=p, fields0=f, nsteps=250, every=100)
        mask = torch.ones(f[0].size, dtype=torch.float64)
    mask = mask.cuda()
    theta0 = np.array([1.2, 1.0, 1.0])
    with torch.no_grad():
        ref = FinalState.apply(torch.tensor([1.15, 1.05, 0.97], dtype=torch.float64), wl)

    def mix(u):
        ph = u[0]
        p = ph ** 3 * (ph * (6.0 * ph - 15.0) + 10.0)  # quintic h (a_p = 0)
        return p * u[1] + (1.0 - p) * u[2]

    c_ref = mix(ref)

    def loss(theta):
        u = FinalState.apply(theta, wl)
        return (mask * (u[0] - ref[0]) ** 2).sum() + (mask * (mix(u) - c_ref) ** 2).sum()

    print(f"case: profile loss {dim}D", flush=True)
    th = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    L = loss(th)
    L.backward()
    g = th.grad.numpy()
    h = 1e-6
    fd = np.zeros(3)
    with torch.no_grad():
        for i in range(3):
            tp, tm = theta0.copy(), theta0.copy()
            tp[i] += h
            tm[i] -= h
            fd[i] = (loss(torch.tensor(tp)).item() - loss(torch.tensor(tm)).item()) / (2 * h)
    print(f"  grad {g} fd {fd}", flush=True)
    for i in range(3):
        assert abs(g[i] - fd[i]) <= 1e-5 * max(abs(fd[i]), 1e-3 * np.abs(fd).max()), (i, g, fd)
