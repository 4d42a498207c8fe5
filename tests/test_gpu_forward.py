"""GPU parity of the forward step (through the C ABI) against the CPU oracle.

Bar: max relative field error max|x - ref| / max|ref| <= 1e-10 per field
after the whole run, element by element, on the same seeded inputs.
Cases span several tiles with ragged tails, the window shift, mirror and
periodic transverse axes, batched runs of uneven length (C = 1..8 cells per
thread), and at the full workload sizes one step on sampled grids.
"""
import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I
from tests.helpers import TOL, assert_parity, oracle_batch, oracle_params, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def _run_gpu(torch, p, fields, nsteps, runs=None, offsets=None, expect=0):
    from paper_2303_09671_amd import pf
    t = [_dev(torch, a) for a in fields]
    h = pf.pf_create(p, *t, runs=runs, offsets=offsets)
    pf.pf_step(h, nsteps)
    torch.cuda.synchronize()
    assert pf.pf_check(h) == expect
    out = [x.cpu().numpy() for x in t]
    return h, t, out


def test_1d_full_run(torch_dev, oracle):
    """The 1D workload as configured: N = 1024, 20000 steps, V = 0.1."""
    p, steps = I.config_1d()
    f = I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])
    print("case: 1D N=1024 steps=20000", flush=True)
    h, t, g = _run_gpu(torch_dev, p, f, steps)
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert_parity(g, ref[:3], what="1D full")
    from paper_2303_09671_amd import pf
    tot, cm, am = pf.pf_solute(h)
    rt, rcm, ram = oracle.solute(oracle_params(oracle, p), *ref[:3])
    assert abs(cm[0] - rcm) <= TOL * rcm and abs(tot[0] - rt) <= 1e-12 * abs(rt)
    assert am[0] == ram or abs(g[0][am[0]] - ref[0][am[0]]) < 1e-9  # unique max, or a tie to rounding
    E = pf.pf_energy(h)[0]
    assert abs(E - oracle.energy(oracle_params(oracle, p), *ref[:3], n=steps, shift=ref[3])) <= 1e-10 * abs(E)


@pytest.mark.parametrize("Ns", [(37, 600, 1024, 1025, 3001), (8192, 512, 4096, 77)])
def test_1d_batch(torch_dev, oracle, Ns):
    """Uneven runs (1..8 cells per thread, ragged chunks).  The 37-cell run is
    too short for its front: the oracle goes non-finite, and so must the GPU
    run, with the error word raised, while the other runs stay exact."""
    runs = []
    for i, N in enumerate(Ns):
        V = [0.02, 0.1, 0.3, 0.05, 0.2][i % 5]
        runs.append(dict(N=N, V=V, dt=I.run_dt(V), z0=(N // 4) * I.DX))
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    steps = 1500
    print(f"case: batch {Ns} steps={steps}", flush=True)
    refs = oracle_batch(oracle, base, runs, steps)
    finite = [all(np.isfinite(a).all() for a in ref) for ref in refs]
    from paper_2303_09671_amd import pf
    h, t, g = _run_gpu(torch_dev, base, (phi, cs, cl), steps, runs=runs, offsets=offs,
                       expect=pf.PF_OK if all(finite) else pf.PF_ENONFINITE)
    for r, o, ref, fin in zip(runs, offs, refs, finite):
        gr = [a[o:o + r["N"]] for a in g]
        if fin:
            assert_parity(gr, ref, what=f"run N={r['N']}")
        else:
            assert not all(np.isfinite(a).all() for a in gr), f"run N={r['N']} should be non-finite"
    tot, cm, am = pf.pf_solute(h)
    E = pf.pf_energy(h)
    for i, (r, ref, fin) in enumerate(zip(runs, refs, finite)):
        if not fin:
            continue
        po = oracle_params(oracle, dict(base, n=(r["N"], 1, 1), V=r["V"], dt=r["dt"], z0=r["z0"]))
        rt, rcm, _ = oracle.solute(po, *ref)
        assert abs(cm[i] - rcm) <= TOL * rcm
        s = int(np.floor(r["V"] * (steps * r["dt"]) / base["dx"]))
        assert abs(E[i] - oracle.energy(po, *ref, n=steps, shift=s)) <= 1e-10 * abs(E[i])


@pytest.mark.parametrize("periodic", [1, 0])
def test_2d_ragged_with_shift(torch_dev, oracle, periodic):
    p, _, pert = I.config_2d(nx=150, nz=75)
    p = dict(p, periodic=(periodic, 0, 0), V=0.5)  # a window shift every 50 steps
    f = [a.ravel() for a in I.planar_front(2, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
    steps = 260
    print(f"case: 2D 150x75 periodic={periodic} steps={steps}", flush=True)
    h, t, g = _run_gpu(torch_dev, p, f, steps)
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert ref[3] == 5
    assert_parity(g, ref[:3], what="2D ragged")
    from paper_2303_09671_amd import pf
    tot, cm, am = pf.pf_solute(h)
    rt, rcm, _ = oracle.solute(oracle_params(oracle, p), *ref[:3])
    assert abs(cm[0] - rcm) <= TOL * rcm and abs(tot[0] - rt) <= 1e-12 * abs(rt)
    E = pf.pf_energy(h)[0]
    assert abs(E - oracle.energy(oracle_params(oracle, p), *ref[:3], n=steps, shift=ref[3])) <= 1e-10 * abs(E)


@pytest.mark.parametrize("periodic", [(1, 1), (0, 1)])
def test_3d_ragged_with_shift(torch_dev, oracle, periodic):
    p, _, pert = I.config_3d(n=8)
    p = dict(p, n=(40, 12, 45), periodic=(periodic[0], periodic[1], 0), V=0.6, z0=14 * 0.8)
    f = [a.ravel() for a in I.planar_front(3, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
    steps = 90  # two shifts
    print(f"case: 3D 40x12x45 periodic={periodic} steps={steps}", flush=True)
    h, t, g = _run_gpu(torch_dev, p, f, steps)
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert ref[3] == 2
    assert_parity(g, ref[:3], what="3D ragged")
    from paper_2303_09671_amd import pf
    E = pf.pf_energy(h)[0]
    assert abs(E - oracle.energy(oracle_params(oracle, p), *ref[:3], n=steps, shift=ref[3])) <= 1e-10 * abs(E)


@pytest.mark.parametrize("dim,quintic,ap", [(2, 1, -2.0), (2, 0, -1.5), (2, 0, 0.0), (3, 0, 0.0), (3, 1, -2.0)])
def test_interpolation_variants(torch_dev, oracle, dim, quintic, ap):
    """Cubic h and a nonzero a_p (Eq. interpolation2) through the 2D/3D step:
    the step kernels are compiled separately for a_p = 0 and a_p != 0."""
    if dim == 2:
        p, _, pert = I.config_2d(nx=70, nz=48)
        p = dict(p, V=0.5, z0=14 * I.DX)
    else:
        p, _, pert = I.config_3d(n=8)
        p = dict(p, n=(36, 10, 40), V=0.6, z0=14 * I.DX)
    p = dict(p, quintic=quintic, ap=ap)
    f = [a.ravel() for a in I.planar_front(dim, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
    steps = 80
    print(f"case: {dim}D quintic={quintic} ap={ap} steps={steps}", flush=True)
    h, t, g = _run_gpu(torch_dev, p, f, steps)
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert ref[3] >= 1
    assert_parity(g, ref[:3], what=f"{dim}D quintic={quintic} ap={ap}")


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_source_A_equals_one(torch_dev, oracle, dim):
    """A = 1 (the special case without anti-trapping: every (1 - A) term of the
    drive, the prefactor and the fluxes vanishes) through each step kernel.
    A < 1 - k_e drives the ghost c_s negative in this scheme (both sides go
    non-finite), so it is not a parity case."""
    if dim == 1:
        p, _ = I.config_1d(N=700)
        p = dict(p, z0=175 * I.DX)
        f = list(I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"]))
        steps = 1500
    elif dim == 2:
        p, _, pert = I.config_2d(nx=70, nz=48)
        p = dict(p, V=0.5, z0=14 * I.DX)
        f = [a.ravel() for a in I.planar_front(2, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
        steps = 200
    else:
        p, _, pert = I.config_3d(n=8)
        p = dict(p, n=(36, 10, 40), V=0.6, z0=14 * I.DX)
        f = [a.ravel() for a in I.planar_front(3, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
        steps = 80
    p = dict(p, A=1.0)
    print(f"case: A = 1, {dim}D, {steps} steps", flush=True)
    h, t, g = _run_gpu(torch_dev, p, f, steps)
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert_parity(g, ref[:3], what=f"A=1 {dim}D")


@pytest.mark.parametrize("dim,n,model", [(3, (64, 16, 40), 0), (3, (41, 13, 40), 0), (2, (150, 1, 60), 0),
                                         (3, (41, 13, 40), 1), (2, (150, 1, 60), 1)])
def test_ring_load_paths_agree(torch_dev, oracle, dim, n, model):
    """The ring planes of the 2D/3D step go from global memory into LDS by DMA
    (16 bytes a lane) where two ring positions are adjacent and 16-byte aligned
    in memory, and through registers otherwise.  Fields passed as views 8 bytes
    off a 16-byte boundary take the register path on every step that reads
    them (the handle's twins stay aligned, so the steps alternate); odd nx and
    ny (41 x 13) put periodic wraps inside pairs and leave every other row and
    plane misaligned.  Both runs must agree bit for bit and match the oracle,
    for both models (the equal-potential one loads no c_s)."""
    if dim == 3:
        p, _, pert = I.config_3d(n=8)
        p = dict(p, n=n, periodic=(1, 1, 0), V=0.6, z0=14 * I.DX)
    else:
        p, _, pert = I.config_2d(nx=n[0], nz=n[2])
        p = dict(p, periodic=(1, 0, 0), V=0.5, z0=14 * I.DX)
    p = dict(p, model=model)
    f = [a.ravel() for a in I.planar_front(dim, p["n"], p["dx"], p["z0"], p["ke"], amp=0.05, seed=pert["seed"])]
    steps = 61
    print(f"case: ring load paths {dim}D {n} model={model} steps={steps}", flush=True)
    from paper_2303_09671_amd import pf
    _, _, g_al = _run_gpu(torch_dev, p, f, steps)
    views = []
    for a in f:
        base = torch_dev.empty(a.size + 1, dtype=torch_dev.float64, device="cuda")
        v = base[1:]
        assert v.data_ptr() % 16 == 8
        v.copy_(torch_dev.from_numpy(np.ascontiguousarray(a, dtype=np.float64)))
        views.append(v)
    h = pf.pf_create(p, *views)
    pf.pf_step(h, steps)
    torch_dev.cuda.synchronize()
    assert pf.pf_check(h) == 0
    g_un = [x.cpu().numpy() for x in views]
    for a, b in zip(g_al, g_un):
        assert np.array_equal(a, b)
    ref = oracle.step(oracle_params(oracle, p), *f, steps)
    assert ref[3] >= 1
    assert_parity(g_al, ref[:3], what=f"ring load paths {dim}D {n} model={model}")


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_full_size_one_step(torch_dev, oracle, which):
    """Workload sizes as configured (2D 1024^2, 3D 256^3), same launch
    configuration as the benchmark: advance 40 steps on the GPU, then compare
    one more GPU step with one oracle step from the GPU's state, on every cell."""
    if which == "2d":
        p, _, pert = I.config_2d()
    else:
        p, _, pert = I.config_3d()
    f = [a.ravel() for a in I.planar_front(p["dim"], p["n"], p["dx"], p["z0"], p["ke"], amp=pert["amp"],
                                           seed=pert["seed"])]
    print(f"case: full-size {which} one step", flush=True)
    from paper_2303_09671_amd import pf
    h, t, g40 = _run_gpu(torch_dev, p, f, 40)
    pf.pf_step(h, 1)
    torch_dev.cuda.synchronize()
    g41 = [x.cpu().numpy() for x in t]
    s40 = int(np.floor(p["V"] * (40 * p["dt"]) / p["dx"]))
    ref = oracle.step(oracle_params(oracle, p), *g40, 1, n0=40, shift=s40)
    assert_parity(g41, ref[:3], what=f"full-size {which}")


def test_error_paths(torch_dev):
    from paper_2303_09671_amd import pf
    p, _ = I.config_1d(N=64)
    p = dict(p, z0=16 * I.DX)
    f = list(I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"]))
    with pytest.raises(pf.PFError) as e:
        pf.pf_create(dict(p, dt=1.0), *[_dev(torch_dev, a) for a in f])
    assert e.value.code == pf.PF_EUNSTABLE_DT
    with pytest.raises(pf.PFError) as e:
        pf.pf_create(dict(p, b=1e-3, ap=11.0), *[_dev(torch_dev, a) for a in f])
    assert e.value.code == pf.PF_EINVAL
    with pytest.raises(pf.PFError) as e:
        pf.pf_create(dict(p, ke=1.5), *[_dev(torch_dev, a) for a in f])
    assert e.value.code == pf.PF_EINVAL
    # a NaN planted by the host is reported
    bad = [a.copy() for a in f]
    bad[1][40] = np.nan
    h = pf.pf_create(p, *[_dev(torch_dev, a) for a in bad])
    pf.pf_step(h, 3)
    assert pf.pf_check(h) == pf.PF_ENONFINITE
    assert pf.pf_check(h) == pf.PF_OK  # cleared
    # a negative concentration is reported; check_every makes pf_step report it
    bad = [a.copy() for a in f]
    bad[2][50] = -0.5
    h = pf.pf_create(dict(p, check_every=2), *[_dev(torch_dev, a) for a in bad])
    with pytest.raises(pf.PFError) as e:
        pf.pf_step(h, 4)
    assert e.value.code in (pf.PF_ENEGCONC, pf.PF_ENONFINITE)


def test_batch_full_sweep_sampled(torch_dev, oracle):
    """The k(V) sweep at its configured size (256 runs, N uniform in
    [512, 8192], V log-spaced 1e-3..10) in the single persistent launch the
    benchmark times, 2000 steps; every 32nd run (and the longest) checked
    against the oracle run alone.  Runs whose front leaves the window go
    non-finite on both sides (the error word is raised)."""
    from paper_2303_09671_amd import pf
    runs = I.batch_runs()
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    steps = 2000
    sample = sorted(set(list(range(0, 256, 32)) + [int(np.argmax([r["N"] for r in runs]))]))
    print(f"case: full sweep, sampled runs {sample}", flush=True)
    refs = oracle_batch(oracle, base, [runs[i] for i in sample], steps)
    t = [_dev(torch_dev, a) for a in (phi, cs, cl)]
    h = pf.pf_create(base, *t, runs=runs, offsets=offs)
    pf.pf_step(h, steps)
    torch_dev.cuda.synchronize()
    g = [x.cpu().numpy() for x in t]
    for i, ref in zip(sample, refs):
        o, N = offs[i], runs[i]["N"]
        gr = [a[o:o + N] for a in g]
        if all(np.isfinite(a).all() for a in ref):
            assert_parity(gr, ref, what=f"run {i} N={N} V={runs[i]['V']:.3g}")
        else:
            assert not all(np.isfinite(a).all() for a in gr), i


def test_batch_full_sweep_20000_steps_sampled(torch_dev, oracle):
    """The k(V) sweep exactly as the benchmark times it: 256 runs, one
    persistent launch of the configured 20000 steps.  Three runs are checked
    against the oracle (the longest, one near V = 0.1 and one at small V); the
    oracle runs are independent and go to threads (ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2303_09671_amd import pf
    runs = I.batch_runs()
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    steps = 20000
    sample = sorted({int(np.argmax([r["N"] for r in runs])), 128, 40})
    print(f"case: full sweep 20000 steps, sampled runs {sample}", flush=True)
    with ThreadPoolExecutor(max_workers=len(sample)) as ex:
        futs = [ex.submit(oracle_batch, oracle, base, [runs[i]], steps) for i in sample]
        t = [_dev(torch_dev, a) for a in (phi, cs, cl)]
        h = pf.pf_create(base, *t, runs=runs, offsets=offs)
        pf.pf_step(h, steps)
        torch_dev.cuda.synchronize()
        g = [x.cpu().numpy() for x in t]
        refs = [f.result()[0] for f in futs]
    for i, ref in zip(sample, refs):
        o, N = offs[i], runs[i]["N"]
        gr = [a[o:o + N] for a in g]
        if all(np.isfinite(a).all() for a in ref):
            assert_parity(gr, ref, what=f"run {i} N={N} V={runs[i]['V']:.3g}")
        else:
            assert not all(np.isfinite(a).all() for a in gr), i


def _window(a, x, y, z, w):
    """(2w+1)^3 window of a [nz][ny][nx] array centred on (x, y, z): periodic
    in x and y, clipped to the domain in z."""
    nz, ny, nx = a.shape
    zs = np.arange(max(z - w, 0), min(z + w + 1, nz))
    xs = np.arange(x - w, x + w + 1) % nx
    ys = np.arange(y - w, y + w + 1) % ny
    return a[np.ix_(zs, ys, xs)], int(zs[0])


@pytest.mark.parametrize("model", [0, 1])
def test_3d_half_billion_cells_sampled(torch_dev, oracle, model):
    """A 1024 x 1024 x 512 grid (5.4e8 cells, 26 GB of fields and twins on
    the device), one step in the production launch configuration.  Sampled
    windows (periodic wrap in x and y, tile and z edges, the seams of the z
    chunks at 96 and 192 planes, the interface on the first of them) are
    compared with an oracle step of the same window on the cells whose
    dependency cone (radius 2) lies inside it."""
    from paper_2303_09671_amd import pf
    torch = torch_dev
    nx, ny, nz = 1024, 1024, 512
    p, _, pert = I.config_3d()
    # the front sits on the seam of the launch's z chunks (96 planes at this size), so the
    # windows around it cross the chunk start and end with the interface inside them
    zi = 96
    p = dict(p, n=(nx, ny, nz), z0=zi * I.DX, model=model)
    print(f"case: 3D {nx}x{ny}x{nz} one step, model={model}", flush=True)
    phi, cs, cl = I.device_front(nx, ny, nz, p["dx"], p["z0"], p["ke"], 1e-3, 11)
    w = 5
    centres = [(0, 0, zi), (31, 7, zi - 1), (32 * 17, 8 * 50 + 7, zi + 2), (nx - 1, ny - 1, zi), (500, 300, 3),
               (700, 900, nz - 2), (100, 200, zi + 30), (600, 40, 2 * zi)]
    host0 = {}
    for (x, y, z) in centres:
        lo, hi = max(z - w, 0), min(z + w + 1, nz)
        sl = [t[lo:hi].cpu().numpy() for t in (phi, cs, cl)]
        host0[(x, y, z)] = [_window(a, x, y, z - lo, w)[0] for a in sl] + [lo]
    h = pf.pf_create(p, phi.view(-1), cs.view(-1), cl.view(-1))
    pf.pf_step(h, 1)
    torch.cuda.synchronize()
    assert pf.pf_check(h) == pf.PF_OK
    for (x, y, z), (wp, ws, wl, lo) in host0.items():
        hi = min(z + w + 1, nz)
        g = [_window(t[lo:hi].cpu().numpy(), x, y, z - lo, w)[0] for t in (phi, cs, cl)]
        nzw = wp.shape[0]
        po = oracle_params(oracle, dict(p, n=(2 * w + 1, 2 * w + 1, nzw), periodic=(0, 0, 0)))
        ref = oracle.step(po, wp.ravel(), ws.ravel(), wl.ravel(), 1, n0=0, shift=lo)
        assert ref[3] == lo  # no window shift in the first step
        # cells at least 3 from every cut face of the window (domain faces in z are real)
        zlo = 0 if lo == 0 else 3
        zhi = nzw if lo + nzw == nz else nzw - 3
        inner = (slice(zlo, zhi), slice(3, 2 * w - 2), slice(3, 2 * w - 2))
        for name, a, r in zip(("phi", "c_s", "c_l"), g, ref[:3]):
            r = r.reshape(a.shape)
            e = float(np.max(np.abs(a[inner] - r[inner])) / np.max(np.abs(r[inner])))
            assert e <= TOL, f"window {(x, y, z)} {name}: {e:.3e}"
