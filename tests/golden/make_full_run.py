"""Write the sampled reference cells of the full 2D and 3D directional-
solidification runs (test data for tests/test_gpu_full_run.py).

Calls only the CPU oracle (``oracle/``, its all-cores OpenMP build, whose
results are bit-identical to the single-thread build) and the seeded input
generators of ``paper_2303_09671_amd.inputs``.  Each file holds, after the
configured number of steps from the seeded initial state:

* ``cols``: complete growth-axis columns (phi, c_s, c_l) at a grid of
  transverse positions ``col_xy``;
* ``planes``: two full transverse planes (phi, c_s, c_l) through the front,
  at growth-axis indices ``plane_z`` (the cell holding the mean phi = 1/2
  crossing and the one above it);
* ``energy``, ``solute``, ``cmax``, ``argmax`` (free energy, total solute,
  maximum of c = p c_s + (1 - p) c_l and its first linear index), ``shift``
  (window shift count) and ``steps``.

Usage: python tests/golden/make_full_run.py [2d|3d|both]   (OMP_NUM_THREADS
sets the thread count; about 20 min for 2D and 2-3 h for 3D on 8 cores.)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2303_09671_amd import inputs as I  # noqa: E402

KEYS = ("dim", "n", "periodic", "quintic", "dx", "dt", "W", "Mphi", "lambda0", "Ds", "ke", "A", "b", "ap",
        "inv_lT", "V", "z0", "eps_grad")


def run(dim: int, out: str, chunk: int = 250) -> None:
    if dim == 2:
        p, steps, pert = I.config_2d()
    else:
        p, steps, pert = I.config_3d()
    po = O.params(**{k: p[k] for k in KEYS})
    shape = I.grid_shape(dim, p["n"])
    f = [a.ravel() for a in I.planar_front(dim, p["n"], p["dx"], p["z0"], p["ke"], amp=pert["amp"],
                                            seed=pert["seed"])]
    n, s = 0, 0
    t0 = time.time()
    while n < steps:
        m = min(chunk, steps - n)
        *f, s = O.step(po, *f, m, n0=n, shift=s, openmp=True)
        n += m
        print(f"{dim}D: step {n}/{steps}, shift {s}, {time.time() - t0:.0f} s", flush=True)
        if not all(np.isfinite(a).all() for a in f):
            raise RuntimeError("oracle run went non-finite")
    fr = O.front(po, f[0], n, s)
    zf = int(np.floor(fr["z"] / p["dx"] - s - 0.5))
    plane_z = np.array([zf, zf + 1])
    u = [a.reshape(shape) for a in f]
    nz = shape[0]
    if dim == 2:
        nx = shape[1]
        col_xy = np.array([[x, 0] for x in range(0, nx, nx // 8)])
        cols = np.stack([np.stack([a[:, x] for a in u]) for x, _ in col_xy])      # [ncol][3][nz]
        planes = np.stack([np.stack([a[z, :] for a in u]) for z in plane_z])      # [2][3][nx]
    else:
        ny, nx = shape[1], shape[2]
        col_xy = np.array([[x, y] for y in range(0, ny, ny // 4) for x in range(0, nx, nx // 4)])
        cols = np.stack([np.stack([a[:, y, x] for a in u]) for x, y in col_xy])  # [ncol][3][nz]
        planes = np.stack([np.stack([a[z] for a in u]) for z in plane_z])         # [2][3][ny][nx]
    tot, cmax, am = O.solute(po, *f)
    energy = O.energy(po, *f, n, s)
    np.savez_compressed(out, cols=cols, col_xy=col_xy, planes=planes, plane_z=plane_z, energy=energy,
                        solute=tot, cmax=cmax, argmax=am, shift=s, steps=n, nz=nz)
    print(f"wrote {out}: front z = {fr['z']:.3f} (cell {zf}), k = {1.0 / cmax:.6f}, "
          f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "both"
    if which in ("2d", "both"):
        run(2, os.path.join(HERE, "full_run_2d_1024.npz"))
    if which in ("3d", "both"):
        run(3, os.path.join(HERE, "full_run_3d_256.npz"))
