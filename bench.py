"""Benchmark of the hot path on one MI355X.

One bench step = one explicit forward-Euler step of the 3D directional-
solidification workload (256^3 cells, FP64, fields phi, c_s, c_l) through the
C ABI (pf_step), with the diagnostics (pf_energy, pf_solute) every 100 steps
inside the timed region.  Inputs are seeded, synthetic and resident in HBM
before timing starts.  Prints ONE JSON line:

* value      -- whole-job FP64 cell-updates per second (cells x steps / time);
* roofline   -- the fused step kernel against the HBM roofline: algorithmic
                48 B per cell-update (read and write phi, c_s, c_l) divided by
                the kernel's average duration from HIP events on the launch
                stream; traffic from committed rocprofv3 FETCH/WRITE counters
                (profiles/) when they were taken on the current kernel source;
* cpu_baseline -- the CPU oracle on a bounded sample (one step of the same
                256^3 grid), single thread;
* extra      -- the other workloads of the hot path: 2D 1024^2, the 1D front,
                the batched 256-run k(V) sweep against 256 sequential launches,
                the adjoint/forward step-time ratio, and the solute-band run
                (interface temperature and velocity from the phi = 1/2 front).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = 48.0      # read and write phi, c_s, c_l (FP64)
BYTES_PER_CELL_EQ = 40.0   # equal-potential model: read phi, c_l; write phi, c_s, c_l
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stream3d_256_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2303_09671_amd", "csrc", f) for f in ("pf_device.h", "pf_kernels.h")]
# the build flags enter the hash too: a record stays valid only for the same compiled kernel
KERNEL_SOURCES.append(os.path.join(ROOT, "paper_2303_09671_amd", "build.py"))


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code (comments and layout stripped), so a
    traffic record stays valid exactly while the compiled kernel is the same."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        src = open(f).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def time_domain(torch, pf, p, pert, steps, warmup, diag_every=100):
    """Returns (total_s, kernel_s, cells, handle, fields)."""
    from paper_2303_09671_amd import inputs as I
    f = I.planar_front(p["dim"], p["n"], p["dx"], p["z0"], p["ke"], amp=pert["amp"], seed=pert["seed"])
    t = [dev(torch, a) for a in f]
    h = pf.pf_create(p, *t)
    cells = int(np.prod([p["n"][k] for k in range(p["dim"])]))
    if warmup:
        pf.pf_step(h, warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    pairs = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        m = min(diag_every, steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pf.pf_step(h, m)
        b.record(stream)
        pairs.append((a, b))
        done += m
        pf.pf_energy(h)
        pf.pf_solute(h)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    kern = sum(a.elapsed_time(b) for a, b in pairs) / 1e3
    return total, kern, cells, h, t


def bench_batch(torch, pf, steps, seq_steps=2000, tail=1000):
    """256-run k(V) sweep: one persistent launch of `steps` steps (timed) vs
    256 sequential single-run launches from the same fresh initial states,
    `seq_steps` steps each (timed; their per-step cost is extrapolated to
    `steps`).  Per run, after the persistent launch: k = 1/c_max, the front and
    its velocity over `tail` further (untimed) steps (post-processing of two
    pf_front readings); a run is steady when that velocity is within 2 % of its
    pulling speed, and lost when no phi = 1/2 crossing is left in its window."""
    from paper_2303_09671_amd import inputs as I
    runs = I.batch_runs()
    base = I.base_params(dim=1)
    phi, cs, cl, offs = I.batch_fields(runs)
    t = [dev(torch, a) for a in (phi, cs, cl)]
    h = pf.pf_create(base, *t, runs=runs, offsets=offs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pf.pf_step(h, steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    _, cm, _ = pf.pf_solute(h)
    k = 1.0 / cm
    f0 = pf.pf_front(h)
    pf.pf_step(h, tail)
    f1 = pf.pf_front(h)
    V = np.array([r["V"] for r in runs])
    dt = np.array([r["dt"] for r in runs])
    v = (f1["z"] - f0["z"]) / (tail * dt)
    finite = np.isfinite(k)
    lost = (f0["ncol"] == 0) | (f1["ncol"] == 0)
    steady = finite & ~lost & (np.abs(v / V - 1.0) < 0.02)
    # sequential: one handle per run on a fresh copy of the initial state
    ts = [dev(torch, a) for a in (phi, cs, cl)]
    hs = []
    for r, o in zip(runs, offs):
        tt = [x[o:o + r["N"]] for x in ts]
        pr = dict(base, dim=1, n=(r["N"], 1, 1), V=r["V"], dt=r["dt"], z0=r["z0"])
        hs.append(pf.pf_create(pr, *tt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for hh in hs:
        pf.pf_step(hh, seq_steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    cells = sum(r["N"] for r in runs)
    per_run = [dict(V=float(a), N=r["N"], k=(float(b) if np.isfinite(b) else None),
                    status=("lost" if l else "steady" if s_ else "transient" if f_ else "non-finite"))
               for a, r, b, l, s_, f_ in zip(V, runs, k, lost, steady, finite)]
    return dict(runs=len(runs), steps_each=steps, cells_total=cells, persistent_s=t_batch,
                sequential_steps_each=seq_steps, sequential_s=t_seq,
                sequential_extrapolated_s=t_seq * steps / seq_steps,
                speedup_per_step=(t_seq / seq_steps) / (t_batch / steps), cell_updates_per_s=cells * steps / t_batch,
                finite_k=int(finite.sum()), steady=int(steady.sum()), lost=int(lost.sum()),
                transient=int((finite & ~lost & ~steady).sum()),
                steady_V_range=([float(V[steady].min()), float(V[steady].max())] if steady.any() else None),
                per_run=per_run)


def bench_big(torch, pf, p3, steps=40, warmup=5):
    """The 3D step at 1024 x 1024 x 512 cells (5.4e8 cells; 26 GB of fields and
    twins), built on the device: kernel time per step against the same 48 B
    per cell-update."""
    from paper_2303_09671_amd import inputs as I
    nx, ny, nz = 1024, 1024, 512
    p = dict(p3, n=(nx, ny, nz), z0=(nz // 4) * p3["dx"])
    f = I.device_front(nx, ny, nz, p["dx"], p["z0"], p["ke"], 1e-3, 11)
    h = pf.pf_create(p, *(x.view(-1) for x in f))
    pf.pf_step(h, warmup)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    pf.pf_step(h, steps)
    b.record()
    torch.cuda.synchronize()
    k = a.elapsed_time(b) / 1e3 / steps
    cells = nx * ny * nz
    ach = BYTES_PER_CELL * cells / k / 1e9
    del h, f
    torch.cuda.empty_cache()
    return dict(cells=cells, steps=steps, kernel_avg_us=k * 1e6, cell_updates_per_s=cells / k, achieved_GBs=ach,
                frac=ach / HBM_PEAK_GBS)


def bench_adjoint(torch, nsteps=10000):
    """Adjoint/forward step-time ratio on the adjoint fit workloads (64 1D runs
    N = 2048; 2D 512^2), over nsteps with checkpoints every 100 steps: forward
    pass with checkpoints vs backward (segment replay + adjoint steps), with the
    replays overlapped on a second stream (ratio) and one after the other
    (ratio_serial)."""
    from paper_2303_09671_amd import inputs as I
    from paper_2303_09671_amd.adjoint import Workload, adjoint_only_seconds, forward_k
    one_d, two_d, _, _ = I.adjoint_workloads()
    res = {}
    for name, args in (("1d_64x2048", one_d), ("2d_512x512", two_d)):
        wl = Workload(**dict(args, nsteps=nsteps))
        theta = (wl.params["A"], wl.params["Mphi"], wl.params["W"])
        forward_k(wl, theta)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        forward_k(wl, theta, checkpoints=True)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        tb = adjoint_only_seconds(wl, theta)
        ts = adjoint_only_seconds(wl, theta, overlap=False)
        res[name] = dict(steps=nsteps, forward_s=tf, backward_s=tb, ratio=tb / tf,
                         backward_serial_s=ts, ratio_serial=ts / tf)
    return res


def bench_bands(torch, pf, every=2000):
    """The solute-band workload (Si-9%As, G = 1.4e6 K/m, v_p = 0.3 m/s): one
    long 1D run with the phi = 1/2 front read every ``every`` steps; the
    interface temperature and velocity of its second half."""
    from paper_2303_09671_amd import inputs as I
    from paper_2303_09671_amd.front import front_series
    p, steps = I.config_bands()
    f = I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])
    t = [dev(torch, a) for a in f]
    h = pf.pf_create(p, *t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ser = front_series(h, steps, every, p["dt"])
    torch.cuda.synchronize()
    d = time.perf_counter() - t0
    half = len(ser["n"]) // 2
    T, v = ser["T"][half:, 0], ser["v"][half:, 0]
    _, cm, _ = pf.pf_solute(h)
    return dict(cells=p["n"][0], steps=steps, seconds=d, cell_updates_per_s=p["n"][0] * steps / d,
                front_every=every, z_final=float(ser["z"][-1, 0]), k=float(1.0 / cm[0]),
                T_I_second_half=[float(T.min()), float(T.mean()), float(T.max())],
                v_I_second_half=[float(v.min()), float(v.mean()), float(v.max())], V_pull=p["V"])


def bench_bands_osc(torch, pf, g_factor=1.0):
    """The oscillating band run (config_bands_osc: the band workload with the
    kinetic coefficient alpha = 0.5, dx = 0.5, N = 8192), with the temperature
    gradient scaled by ``g_factor``: front every 8 W^2/D_l; velocity and
    temperature swings, period and band wavelength over the last two thirds."""
    from paper_2303_09671_amd import inputs as I
    from paper_2303_09671_amd.front import front_series, oscillation
    p, steps = I.config_bands_osc()
    p["inv_lT"] *= g_factor
    f = I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])
    t = [dev(torch, a) for a in f]
    h = pf.pf_create(p, *t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ser = front_series(h, steps, int(round(8.0 / p["dt"])), p["dt"])
    torch.cuda.synchronize()
    d = time.perf_counter() - t0
    o = oscillation(ser, t_from=steps * p["dt"] / 3.0)
    # physical units of the Si-As map: W = 13.5 nm, W^2 / D_l = 1.215e-8 s
    return dict(cells=p["n"][0], steps=steps, seconds=d, Mphi=p["Mphi"], V_pull=p["V"], G_K_per_m=1.4e6 * g_factor,
                **o, period_s=o["period"] * 1.215e-8, wavelength_um=o["wavelength"] * 0.0135)


def bench_ti_curve(torch, pf, A, every=5000):
    """T_I and k against the pulling speed in the Fig. 4 setting
    (config_ti_curve): the batch stepped in launches of ``every`` steps with a
    pf_front reading after each; per run k = 1/c_max at the end, T_I at the
    end, and over the last third of the run the front's state (steady,
    oscillating or transient: front_state), the range of the interface
    velocity over V and the mean and range of T_I (post-processing of the
    pf_front readings)."""
    from paper_2303_09671_amd import inputs as I
    from paper_2303_09671_amd import asymptotics as asy
    from paper_2303_09671_amd.front import front_series, front_state, oscillation
    base, runs, steps, vp = I.config_ti_curve(A)
    phi, cs, cl, offs = I.batch_fields(runs, ke=base["ke"])
    t = [dev(torch, a) for a in (phi, cs, cl)]
    h = pf.pf_create(base, *t, runs=runs, offsets=offs)
    V = np.array([r["V"] for r in runs])
    dts = np.array([r["dt"] for r in runs])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ser = front_series(h, steps, every, dts)
    torch.cuda.synchronize()
    d = time.perf_counter() - t0
    _, cm, _ = pf.pf_solute(h)
    ncol = pf.pf_front(h)["ncol"]
    state, osc = [], []
    for i in range(len(runs)):
        t_from = steps * dts[i] * 2.0 / 3.0
        state.append(front_state(ser, i, V[i], t_from) if ncol[i] == 1 else "no single front")
        osc.append(oscillation(ser, i, t_from))
    # the first-order asymptotic k of Eq. partition1 at the same speeds (host side)
    k_asy, _ = asy.kv_curve(V, A=A, b=base["b"], m=base["Ds"], ke=base["ke"])
    f = lambda xs: [float(x) for x in xs]
    return dict(A=A, runs=len(runs), steps=steps, front_every=every, seconds=d, v_p_m_per_s=f(vp),
                k=f(1.0 / cm), k_asymptotic=f(k_asy), T_I=f(ser["T"][-1]),
                T_I_last_third_mean=f(o["T_mean"] for o in osc), T_I_last_third_min=f(o["T_min"] for o in osc),
                T_I_last_third_max=f(o["T_max"] for o in osc),
                v_over_V_last_third_min=f(o["v_min"] / v for o, v in zip(osc, V)),
                v_over_V_last_third_max=f(o["v_max"] / v for o, v in zip(osc, V)),
                state=state, steady=[s == "steady" for s in state],
                # oscillating fronts: mean period between upward crossings of the mean velocity and
                # the band wavelength, in the Si-As units (W^2/D_l = 1.215e-8 s, W = 13.5 nm)
                period_us=[o["period"] * 1.215e-2 if s == "oscillating" else None for o, s in zip(osc, state)],
                wavelength_um=[o["wavelength"] * 0.0135 if s == "oscillating" else None for o, s in zip(osc, state)])


def cpu_baseline(p, pert):
    from oracle import oracle as O
    from paper_2303_09671_amd import inputs as I
    keys = ("dim", "n", "periodic", "quintic", "dx", "dt", "W", "Mphi", "lambda0", "Ds", "ke", "A", "b", "ap",
            "inv_lT", "V", "z0", "eps_grad")
    po = O.params(**{k: p[k] for k in keys})
    f = [a.ravel() for a in I.planar_front(p["dim"], p["n"], p["dx"], p["z0"], p["ke"], amp=pert["amp"],
                                           seed=pert["seed"])]
    cells = int(np.prod([p["n"][k] for k in range(p["dim"])]))
    grid = "x".join(str(v) for v in p["n"][:p["dim"]])
    t0 = time.perf_counter()
    O.step(po, *f, 1)
    dt = time.perf_counter() - t0
    out = dict(value=cells / dt, unit="cell-updates/s", cores=1, kind="oracle",
               sample=f"one step of the full {grid} grid ({cells} cell-updates, {dt:.1f} s, single thread)")
    # the same oracle source built with its OpenMP cell loops, on all host cores
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    O.step(po, *f, 1, openmp=True)  # thread-pool start-up outside the timed region
    t0 = time.perf_counter()
    O.step(po, *f, 2, openmp=True)
    dt2 = time.perf_counter() - t0
    out["all_cores"] = dict(value=2 * cells / dt2, unit="cell-updates/s", cores=threads, nproc=os.cpu_count(),
                            cpu=_cpu_model(), kind="oracle (OpenMP cell loops, bit-identical results)",
                            sample=f"two steps of the full {grid} grid ({dt2:.1f} s)")
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def traffic_entry():
    if not os.path.exists(TRAFFIC_FILE):
        return None
    d = json.load(open(TRAFFIC_FILE))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5):
    """A plain device copy of known size (for scaling the FETCH/WRITE counters)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extra", action="store_true", help="time only the 3D workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--copy-calib", action="store_true", help="run the plain copy used to scale counters")
    ap.add_argument("--adjoint-only", type=int, default=0, metavar="NSTEPS",
                    help="time only the adjoint workloads over NSTEPS steps (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return
    import torch
    if args.adjoint_only > 0:
        print(json.dumps({"adjoint": bench_adjoint(torch, nsteps=args.adjoint_only)}), flush=True)
        return
    from paper_2303_09671_amd import inputs as I
    from paper_2303_09671_amd import pf
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pf.lib()

    p3, _, pert3 = I.config_3d()
    total, kern, cells, h, _ = time_domain(torch, pf, p3, pert3, args.steps, args.warmup)
    value = cells * args.steps / total
    k_avg = kern / args.steps
    achieved = BYTES_PER_CELL * cells / k_avg / 1e9
    roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=traffic_entry(), kernel="k_stream<3,32,8,APZ,EQ=false>", kernel_avg_us=k_avg * 1e6,
                algorithmic_bytes_per_launch=BYTES_PER_CELL * cells)
    out = {
        "metric": "FP64 cell-updates/s and % HBM roofline; adjoint/forward step time ratio",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D directional solidification, 256^3 cells, x/y periodic, no-flux z, V=0.05, "
                               "dt=0.032, seeded 1e-3 front perturbation; diagnostics every 100 steps",
                   "cells": cells, "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p3, pert3)
    if not args.no_extra:
        extra = {}
        p2, _, pert2 = I.config_2d()
        steps2 = 10000  # the configured 2D run
        t2, k2, c2, _, _ = time_domain(torch, pf, p2, pert2, steps2, 20)
        extra["2d_1024x1024"] = dict(steps=steps2, cell_updates_per_s=c2 * steps2 / t2, kernel_avg_us=k2 / steps2 * 1e6,
                                     effective_GBs=BYTES_PER_CELL * c2 / (k2 / steps2) / 1e9)
        p1, steps1 = I.config_1d()
        f1 = I.planar_front(1, p1["n"], p1["dx"], p1["z0"], p1["ke"])
        t1 = [dev(torch, a) for a in f1]
        h1 = pf.pf_create(p1, *t1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pf.pf_step(h1, steps1)
        torch.cuda.synchronize()
        d1 = time.perf_counter() - t0
        _, cm, _ = pf.pf_solute(h1)
        extra["1d_1024_20000_steps"] = dict(seconds=d1, cell_updates_per_s=1024 * steps1 / d1, k=float(1.0 / cm[0]))
        extra["batch_256_runs"] = bench_batch(torch, pf, 20000)
        extra["adjoint"] = bench_adjoint(torch)
        extra["bands_1d_2048"] = bench_bands(torch, pf)
        extra["bands_oscillating_1d_8192"] = bench_bands_osc(torch, pf)
        extra["ti_curve_fig4"] = [bench_ti_curve(torch, pf, A) for A in (1.2, 2.0)]
        extra["3d_1024x1024x512"] = bench_big(torch, pf, p3)
        # the equal-potential model (mu_s = mu_l imposed) on the 3D and 1D workloads
        pe = dict(p3, model=1)
        te, ke_, ce, _, _ = time_domain(torch, pf, pe, pert3, 500, 10)
        # its state is (phi, c_l): 16 B read and 24 B written per cell-update
        ae = BYTES_PER_CELL_EQ * ce / (ke_ / 500) / 1e9
        extra["equal_potential_3d_256"] = dict(kernel="k_stream<3,32,8,APZ,EQ=1>", kernel_avg_us=ke_ / 500 * 1e6,
                                               cell_updates_per_s=ce * 500 / te, algorithmic_bytes_per_cell=BYTES_PER_CELL_EQ,
                                               achieved_GBs=ae, frac=ae / HBM_PEAK_GBS)
        t1e = [dev(torch, a) for a in f1]
        h1e = pf.pf_create(dict(p1, model=1), *t1e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pf.pf_step(h1e, steps1)
        torch.cuda.synchronize()
        d1e = time.perf_counter() - t0
        _, cme, _ = pf.pf_solute(h1e)
        extra["equal_potential_1d_1024_20000_steps"] = dict(seconds=d1e, cell_updates_per_s=1024 * steps1 / d1e,
                                                            k=float(1.0 / cme[0]))
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
