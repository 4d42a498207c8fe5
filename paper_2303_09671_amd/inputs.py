"""Seeded synthetic inputs (shared by the tests, the smoke check and the benchmark).

This module builds initial states and run tables only; it contains none of the
time-stepping arithmetic.  Both the HIP path and the CPU oracle receive the
arrays it returns.  Every random number is drawn here from numpy's PCG64 with a
fixed seed and handed to both sides as data.

Recipe (nondimensional: lengths in W0, time in W0^2/D_l, c in c_inf):

* planar front at height ``z0`` (a cell face) on the growth axis, the last
  axis: phi0 = 1 / (1 + exp(sqrt(2) (z - z0) / W)), the equilibrium profile of
  the supplement (Sec. S-I, Eq. eq18) written in logistic form;
* homogeneous phase concentrations c_l = c_inf = 1, c_s = k_e (Sec. V.A);
* optional seeded perturbation phi += amp (2 xi - 1) 4 phi0 (1 - phi0),
  xi ~ U[0, 1), band-limited to the interface so the bulk stays exactly 0/1;
* the five workload definitions of the hot path (1D front, 2D and 3D
  directional solidification, a 256-run k(V) sweep, the adjoint fit runs), the
  1D front at the paper's A = 2 and the solute-band run.
"""
from __future__ import annotations

import math

import numpy as np

#: Alloy and model parameters shared by every workload (nondimensional).
ALLOY = dict(
    ke=0.14,            # equilibrium partition coefficient
    Ds=1e-4,            # D_s / D_l
    W=1.0,              # interface width / W0
    Mphi=1.0,           # phi mobility: alpha = tau D_l / W0^2 = W / Mphi
    lambda0=0.04462,    # Omega c_inf / H at W = W0 (I (W/d0) k_e / (1-k_e)^2 with W/d0 = 1)
    A=1.2,              # source / trapping coefficient (A_FIT = 2 is the Si-As fit of Sec. V.D)
    b=1e-4, ap=0.0,     # interpolation set 2 constants: b = D_s/D_l (symmetric q_n), a_p = 0
    quintic=1,
    inv_lT=1.0 / 444.0, # 1 / thermal length l_T = dT0 / G
    eps_grad=3e-3,      # scale of the smooth gate G / (G^2 + eps^2) on 1/|grad phi|^2
)

DX = 0.8

#: The paper's fitted source coefficient for Si-As (Sec. V.D).  Its runs are
#: unstable to perturbations of the front after about 8000 steps of the 1D
#: workload, so they take the operating-point workload (config_1d_a2), not the
#: full-run parity workloads.
A_FIT = 2.0


def grid_shape(dim: int, n) -> tuple:
    """numpy shape (slowest first) for cells-per-axis ``n`` (axis 0 fastest)."""
    n = tuple(int(v) for v in n)[:dim]
    return tuple(reversed(n))


def planar_front(dim: int, n, dx: float, z0: float, ke: float, W: float = 1.0,
                 amp: float = 0.0, seed: int | None = None):
    """Initial (phi, c_s, c_l) as float64 arrays of shape ``grid_shape(dim, n)``."""
    shape = grid_shape(dim, n)
    nz = shape[0]
    z = (np.arange(nz, dtype=np.float64) + 0.5) * dx
    arg = math.sqrt(2.0) * (z - z0) / W
    with np.errstate(over="ignore"):
        phi1 = 1.0 / (1.0 + np.exp(arg))
    phi = np.broadcast_to(phi1.reshape((nz,) + (1,) * (dim - 1)), shape).copy()
    if amp != 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        xi = rng.random(shape)
        phi = phi + amp * (2.0 * xi - 1.0) * 4.0 * phi * (1.0 - phi)
    cs = np.full(shape, ke, dtype=np.float64)
    cl = np.ones(shape, dtype=np.float64)
    return phi, cs, cl


def device_front(nx: int, ny: int, nz: int, dx: float, z0: float, ke: float, amp: float, seed: int):
    """A perturbed 3D planar front built on the current CUDA device plane by plane
    (no host copy of a multi-GB state): phi0(z) + amp (2 xi - 1) 4 phi0 (1 - phi0)
    with xi from torch's seeded device generator, c_s = k_e, c_l = 1.  Returns
    three contiguous float64 tensors of shape [nz][ny][nx]."""
    import torch
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    z = (torch.arange(nz, dtype=torch.float64, device="cuda") + 0.5) * dx
    prof = 1.0 / (1.0 + torch.exp(math.sqrt(2.0) * (z - z0)))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    for k in range(nz):
        xi = torch.rand((ny, nx), generator=g, dtype=torch.float64, device="cuda")
        p = prof[k]
        phi[k] = p + amp * (2.0 * xi - 1.0) * 4.0 * p * (1.0 - p)
    cs = torch.full((nz, ny, nx), ke, dtype=torch.float64, device="cuda")
    cl = torch.ones((nz, ny, nx), dtype=torch.float64, device="cuda")
    return phi, cs, cl


def base_params(**kw) -> dict:
    p = dict(ALLOY)
    p.update(dict(dx=DX, V=0.1, dt=0.128, z0=0.0, dim=1, n=(1, 1, 1), periodic=(0, 0, 0)))
    p.update(kw)
    return p


def config_1d(N: int = 1024, steps: int = 20000):
    """1D planar rapid-solidification front: N=1024, dx=0.8 W, V=0.1,
    dt = 0.2 dx^2, 20000 steps, front at N/4, no-flux ends."""
    p = base_params(dim=1, n=(N, 1, 1), V=0.1, dt=0.2 * DX * DX, z0=(N // 4) * DX)
    return p, steps


def config_1d_a2(N: int = 1024, steps: int = 20000):
    """The 1D workload at the paper's operating point A = A_FIT = 2 (the Si-As
    fit of Sec. V.D): same grid, speed and time step as config_1d."""
    p, steps = config_1d(N, steps)
    p["A"] = A_FIT
    return p, steps


def config_2d(nx: int = 1024, nz: int = 1024, steps: int = 10000, seed: int = 1, amp: float = 1e-3):
    """2D directional solidification: periodic x, no-flux z, V=0.05,
    dt = 0.2 dx^2 / 4, seeded front perturbation of amplitude 1e-3."""
    p = base_params(dim=2, n=(nx, nz, 1), periodic=(1, 0, 0), V=0.05, dt=0.2 * DX * DX / 4.0,
                    z0=(nz // 4) * DX)
    return p, steps, dict(amp=amp, seed=seed)


def config_3d(n: int = 256, steps: int = 2000, seed: int = 2, amp: float = 1e-3):
    """3D directional solidification, 256^3, x and y periodic, same alloy as 2D."""
    p = base_params(dim=3, n=(n, n, n), periodic=(1, 1, 0), V=0.05, dt=0.2 * DX * DX / 4.0,
                    z0=(n // 4) * DX)
    return p, steps, dict(amp=amp, seed=seed)


def config_bands(N: int = 2048, steps: int = 200000):
    """Long 1D run of the solute-band study (Figs. 8-9): Si-9%As (k_e = 0.3,
    liquidus slope -4 K/%, c_inf = 9 %, so the freezing range is dT0 = 84 K;
    D_l = 1.5e-8 m^2/s) with W = 13.5 nm, G = 1.4e6 K/m (l_T = dT0 / G =
    6e-5 m = 4444 W), v_p = 0.3 m/s (V = v_p W / D_l = 0.27) and D_s/D_l = 1e-3;
    b = 1e-3 and lambda0 = I k_e / (1 - k_e)^2 (W/d0 = 1), A = 2 (the
    paper's Si-As fit);
    dt = 0.2 dx^2, front at N/4, no-flux ends, 200000 steps (about 1.6
    thermal times l_T / V)."""
    I0 = 1.0 / (3.0 * math.sqrt(2.0))
    ke = 0.3
    p = base_params(dim=1, n=(N, 1, 1), V=0.27, dt=0.2 * DX * DX, z0=(N // 4) * DX)
    p.update(ke=ke, Ds=1e-3, b=1e-3, A=A_FIT, lambda0=I0 * ke / (1.0 - ke) ** 2, inv_lT=1.0 / 4444.0)
    return p, steps


def config_bands_osc(N: int = 8192, t_end: float = 60000.0, dx: float = 0.5):
    """The band run with the kinetic coefficient lowered to alpha = W / M_phi
    = 0.5 (M_phi = 2), below the threshold where the planar front turns
    oscillatory: the oscillatory instability of Sec. V.F.  Everything else as
    config_bands, on the paper's main grid spacing dx = 0.5 W (the oscillation
    is grid-converged from dx = 0.5 on, not at 0.8); a window of N = 8192
    cells (front at N/4) holds the front through the swings of T_I, dt from
    the phi-relaxation limit at that alpha, t_end = 60000 (about 3.6 thermal
    times l_T / V)."""
    p, _ = config_bands(N=N)
    p.update(dx=dx, Mphi=2.0, dt=run_dt(p["V"], dx=dx, alpha=p["W"] / 2.0, W=p["W"]), z0=(N // 4) * dx)
    return p, int(round(t_end / p["dt"]))


def config_ti_curve(A: float, N: int = 0, nruns: int = 24, steps: int = 0, dx: float = DX):
    """Interface temperature and k against the pulling speed in the setting of
    Fig. 4 (Sec. V.C): Si-9%As (k_e = 0.3, D_l = 1.5e-8 m^2/s, dT0 = 84 K) at
    W = 13.5 nm, D_s/D_l = 0.1, b = 1, G = 1.4e7 K/m (l_T = dT0 / G = 6 um =
    444.4 W), lambda0 = I k_e / (1 - k_e)^2, source coefficient A; one batch of
    ``nruns`` 1D runs with v_p log-spaced from 0.02 to 1 m/s (V = v_p W / D_l),
    N cells each, the front in mid-window (T_I moves it by up to a few
    hundred W), dt = min(0.2 dx^2, run_dt(V)), ``steps`` steps (about 1.7
    thermal times l_T / V at 0.02 m/s).  N = 0 and steps = 0 take 2048 cells
    and 600000 steps at dx = 0.8, and the same window and time span at
    another grid spacing dx.  Returns (base params, runs, steps, v_p in m/s)."""
    I0 = 1.0 / (3.0 * math.sqrt(2.0))
    ke = 0.3
    N = N or int(round(2048 * DX / dx))
    steps = steps or int(round(600000 * DX * DX / (dx * dx)))
    vp = np.geomspace(0.02, 1.0, nruns)
    runs = [dict(N=N, V=float(v * 13.5e-9 / 1.5e-8),
                 dt=float(min(0.2 * dx * dx, run_dt(v * 13.5e-9 / 1.5e-8, dx=dx))), z0=(N // 2) * dx)
            for v in vp]
    base = base_params(dim=1, dx=dx)
    base.update(ke=ke, Ds=0.1, b=1.0, A=A, lambda0=I0 * ke / (1.0 - ke) ** 2, inv_lT=13.5e-9 * 1.4e7 / 84.0)
    return base, runs, steps, vp


def run_dt(V: float, dx: float = DX, alpha: float = 1.0, W: float = 1.0) -> float:
    """Per-run time step from the run's stability limits (diffusion, window
    advection, phi relaxation)."""
    return min(0.2 * dx * dx, 0.1 * dx / V, 0.4 * alpha * dx * dx / (2.0 * W * W))


def front_cell(N: int, V: float, dx: float = DX) -> int:
    """Initial front cell of a 1D run: the liquid ahead keeps 12 diffusion
    lengths D_l / V of the solute boundary layer (at least 48 W), and the rest
    of the window lies behind the front, where a fast front falls back while
    its kinetic undercooling builds up; never below N/4."""
    ahead = int(math.ceil(max(48.0, 12.0 / V) / dx))
    return max(N // 4, N - ahead)


def batch_runs(nruns: int = 256, seed: int = 3, nmin: int = 512, nmax: int = 8192,
               vmin_log10: float = -3.0, vmax_log10: float = 1.0):
    """k(V) sweep: velocities log-spaced from 1e-3 to 10, lengths uniform in
    [512, 8192] (seeded), per-run dt from ``run_dt``, front at ``front_cell``.

    Returns a list of dicts with keys N, V, dt, z0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.random(nruns)
    runs = []
    for r in range(nruns):
        frac = r / (nruns - 1) if nruns > 1 else 0.0
        V = 10.0 ** (vmin_log10 + (vmax_log10 - vmin_log10) * frac)
        N = nmin + int(math.floor((nmax - nmin + 1) * xi[r]))
        runs.append(dict(N=N, V=V, dt=run_dt(V), z0=front_cell(N, V) * DX))
    return runs


def adjoint_runs(nruns: int = 64, N: int = 2048, seed: int = 4):
    """Adjoint fit workload: 64 runs of N=2048 with V log-spaced 1e-2..1 and a
    seeded target k*(V) = (k_e + V/V_D) / (1 + V/V_D), V_D ~ U[0.1, 1]."""
    runs = batch_runs(nruns=nruns, seed=0, nmin=N, nmax=N, vmin_log10=-2.0, vmax_log10=0.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    VD = 0.1 + 0.9 * rng.random()
    ke = ALLOY["ke"]
    for r in runs:
        r["N"] = N
        r["z0"] = (N // 4) * DX
        r["k_target"] = (ke + r["V"] / VD) / (1.0 + r["V"] / VD)
    return runs, VD


def batch_fields(runs, ke: float = ALLOY["ke"], W: float = 1.0, align: int = 32):
    """Concatenate the runs' 1D initial states with offsets aligned to ``align``
    cells (256 B).  Returns (phi, cs, cl, offsets)."""
    offs = []
    tot = 0
    for r in runs:
        offs.append(tot)
        tot += (r["N"] + align - 1) // align * align
    phi = np.zeros(tot)
    cs = np.full(tot, ke)
    cl = np.ones(tot)
    for r, o in zip(runs, offs):
        f, s, l = planar_front(1, (r["N"],), DX, r["z0"], ke, W)
        phi[o:o + r["N"]] = f
        cs[o:o + r["N"]] = s
        cl[o:o + r["N"]] = l
    return phi, cs, cl, np.asarray(offs, dtype=np.int64)


def adjoint_workloads():
    """The adjoint fit workload: (1D batch workload args, 2D workload args,
    per-run targets, 2D target).  64 runs N = 2048 with V log-spaced in
    [1e-2, 1], one 2D 512^2 run at V = 0.05 (dt = 0.032, seeded 1e-3 front
    perturbation), 10000 steps, checkpoints every 100 steps."""
    runs, VD = adjoint_runs()
    base = base_params(dim=1)
    phi, cs, cl, offs = batch_fields(runs)
    one_d = dict(params=base, fields0=(phi, cs, cl), nsteps=10000, every=100, runs=runs, offsets=offs)
    p2, _, pert = config_2d(nx=512, nz=512, seed=5)
    f2 = tuple(a.ravel() for a in planar_front(2, p2["n"], p2["dx"], p2["z0"], p2["ke"], amp=pert["amp"],
                                                 seed=pert["seed"]))
    two_d = dict(params=p2, fields0=f2, nsteps=10000, every=100)
    ke = ALLOY["ke"]
    k2 = (ke + p2["V"] / VD) / (1.0 + p2["V"] / VD)
    return one_d, two_d, [r["k_target"] for r in runs], k2
