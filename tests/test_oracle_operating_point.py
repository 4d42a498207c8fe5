"""The paper's operating point A = 2 (the Si-As fit, Sec. V.D) on the oracle.

* With the workloads' gate scale eps = 3e-3 of the regularised 1/|grad phi|^2,
  the 1D workload (N = 1024, dx = 0.8, V = 0.1, dt = 0.2 dx^2) steps its
  20000 steps at A = 2 with positive concentrations, a front in the window and
  a partition coefficient between k_e and 1.
* Without the regularisation (eps = 1e-20) the same run fails within 40 steps,
  and not through the time step: a plateau of phi forms inside the interface
  (the kinetic prefactor, whose (1 - A)^2 term grows as 1/|grad phi|^2, stops
  phi from relaxing there), and the anti-trapping flux, proportional to
  phi_t / |grad phi|, diverges at the flat face.  The first update that drives
  c_l negative sits in that plateau, next to a face whose phi difference is
  almost zero.
"""
import numpy as np

from paper_2303_09671_amd import inputs as I

KEYS = ("dim", "n", "periodic", "quintic", "dx", "dt", "W", "Mphi", "lambda0", "Ds", "ke", "A", "b", "ap",
        "inv_lT", "V", "z0", "eps_grad")


def _setup(oracle, **kw):
    p, steps = I.config_1d_a2()
    p = dict(p, **kw)
    po = oracle.params(**{k: p[k] for k in KEYS})
    f = [a.ravel() for a in I.planar_front(1, p["n"], p["dx"], p["z0"], p["ke"])]
    return po, f, steps


def test_1d_workload_steps_at_A2(oracle):
    po, f, steps = _setup(oracle)
    assert po["A"] == 2.0 and po["eps_grad"] == 3e-3
    phi, cs, cl, s = oracle.step(po, *f, steps)
    for a in (phi, cs, cl):
        assert np.isfinite(a).all()
    assert cs.min() > 0 and cl.min() > 0
    k = 1.0 / oracle.solute(po, phi, cs, cl)[1]
    assert po["ke"] < k < 1.0
    fr = oracle.front(po, phi, steps, s)
    assert fr["ncol"] == 1 and 0.0 < fr["z"] - s * po["dx"] < po["n"][0] * po["dx"]


def test_unregularised_gate_fails_in_an_interface_plateau(oracle):
    po, f, _ = _setup(oracle, eps_grad=1e-20)
    phi, cs, cl = f
    s = 0
    for n in range(40):
        nphi, ncs, ncl, ns = oracle.step(po, phi, cs, cl, 1, n0=n, shift=s)
        if not (np.isfinite(ncl).all() and ncl.min() > 0):
            break
        phi, cs, cl, s = nphi, ncs, ncl, ns
    else:
        raise AssertionError("the unregularised A = 2 run stayed positive for 40 steps")
    i = int(np.argmin(ncl))
    assert 0.8 < phi[i] < 0.95  # inside the interface, on the solid side
    # a nearly flat face next to the failing cell: |grad phi| << its equilibrium value there
    flat = min(abs(phi[i] - phi[i - 1]), abs(phi[i + 1] - phi[i])) / po["dx"]
    eq = np.sqrt(2.0) * phi[i] * (1.0 - phi[i])
    assert flat < 0.1 * eq
