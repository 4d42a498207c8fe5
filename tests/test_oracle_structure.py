"""Structural pins of the oracle (brute force on tiny inputs).

* A 1D state copied along periodic transverse axes evolves exactly like the
  1D run (the normal/tangential split reduces to 1D when grad phi is along z).
* Exchanging the two periodic transverse axes of a 3D state exchanges the
  result (catches x/y index slips in the transverse face gradients).
* A 2D state that varies only along a periodic x axis, with phi = 0, evolves
  like the 1D heat equation along x (transverse-axis fluxes).
* The dual-number directional derivative equals a central finite difference
  of the step, for the fields and for theta = (A, M_phi, W).
* The moving window: after a shift the fresh hot-end layer is (0, k_e, 1) and
  every other layer moved down by one cell (Sec. V.A shifting algorithm).
* The OpenMP build used to time the oracle on all cores steps bit for bit like
  the single-thread build.
"""
import numpy as np
import pytest

from paper_2303_09671_amd import inputs as I


def _front_1d(oracle, N=40, V=0.1):
    P1 = oracle.params(dim=1, n=(N, 1, 1), V=V, dt=0.05, z0=12 * 0.8)
    phi, cs, cl = I.planar_front(1, (N,), 0.8, P1["z0"], P1["ke"])
    # a non-trivial state: a few steps in
    phi, cs, cl, s = oracle.step(P1, phi, cs, cl, 30)
    return P1, phi, cs, cl, s


def test_1d_embedded_in_2d_and_3d(oracle):
    P1, phi, cs, cl, s = _front_1d(oracle)
    N = phi.size
    r1 = oracle.step(P1, phi, cs, cl, 40, n0=30, shift=s)
    for dim, n, per in ((2, (5, N, 1), (1, 0, 0)), (3, (3, 4, N), (1, 1, 0)), (2, (4, N, 1), (0, 0, 0))):
        P = dict(P1, dim=dim, n=n, periodic=per)
        rep = int(np.prod(n[:dim - 1]))
        f = [np.repeat(a, rep) for a in (phi, cs, cl)]
        r = oracle.step(P, *f, 40, n0=30, shift=s)
        for a1, a in zip(r1[:3], r[:3]):
            np.testing.assert_array_equal(a.reshape(N, rep), np.repeat(a1[:, None], rep, axis=1))
        assert r[3] == r1[3]


def test_transverse_axis_exchange_3d(oracle):
    nx, ny, nz = 5, 4, 24
    P = oracle.params(dim=3, n=(nx, ny, nz), periodic=(1, 1, 0), V=0.05, dt=0.02, z0=8 * 0.8)
    phi, cs, cl = I.planar_front(3, P["n"], 0.8, P["z0"], P["ke"], amp=0.05, seed=9)
    cl = cl + 0.1 * np.random.default_rng(1).random(cl.shape)
    r = oracle.step(P, phi.ravel(), cs.ravel(), cl.ravel(), 25)
    PT = dict(P, n=(ny, nx, nz))
    tr = lambda a: np.ascontiguousarray(a.reshape(nz, ny, nx).transpose(0, 2, 1)).ravel()
    rt = oracle.step(PT, tr(phi.ravel()), tr(cs.ravel()), tr(cl.ravel()), 25)
    for a, b in zip(r[:3], rt[:3]):
        np.testing.assert_allclose(tr(a), b, rtol=0, atol=1e-14)


def test_x_only_variation_is_1d_heat(oracle):
    nx, nz = 16, 3
    P = oracle.params(dim=2, n=(nx, nz, 1), periodic=(1, 0, 0), V=0.0, inv_lT=0.0, dt=0.05)
    x = (np.arange(nx) + 0.5) * 0.8
    mode = np.cos(2 * np.pi * 2 * x / (nx * 0.8))
    cl = np.tile(1.0 + 1e-3 * mode, nz)
    cs = np.tile(0.2 + 1e-4 * mode, nz)
    phi = np.zeros(nx * nz)
    _, cs2, cl2, _ = oracle.step(P, phi, cs, cl, 5)
    lam = 1 - 4 * 0.05 / 0.64 * np.sin(2 * np.pi * 2 / nx / 2) ** 2
    np.testing.assert_allclose(cl2, np.tile(1.0 + 1e-3 * lam ** 5 * mode, nz), atol=1e-15)


@pytest.mark.parametrize("dim", [1, 2])
def test_jvp_matches_central_difference(oracle, dim):
    if dim == 1:
        P, phi, cs, cl, s = _front_1d(oracle, N=32)
    else:
        P = oracle.params(dim=2, n=(6, 28, 1), periodic=(1, 0, 0), V=0.05, dt=0.02, z0=9 * 0.8)
        phi, cs, cl = (a.ravel() for a in I.planar_front(2, P["n"], 0.8, P["z0"], P["ke"], amp=0.05, seed=4))
        phi, cs, cl, s = oracle.step(P, phi, cs, cl, 10)
    rng = np.random.default_rng(7)
    N = phi.size
    # band-limited phi tangent: the tails (|grad phi| -> 0) divide by |grad phi|,
    # where a finite difference of any fixed size is not in the linear regime
    d = [rng.standard_normal(N) * 1e-2 * 4 * phi * (1 - phi), rng.standard_normal(N) * 1e-2 * cs,
         rng.standard_normal(N) * 1e-2 * cl]
    th = rng.standard_normal(3) * 0.1
    nst = 5
    _, du, _ = oracle.jvp(P, phi, cs, cl, *d, th, nst, n0=10, shift=s)
    h = 1e-6

    def run(sg):
        Pp = dict(P, A=P["A"] + sg * h * th[0], Mphi=P["Mphi"] + sg * h * th[1], W=P["W"] + sg * h * th[2])
        return oracle.step(Pp, phi + sg * h * d[0], cs + sg * h * d[1], cl + sg * h * d[2], nst, n0=10, shift=s)

    rp, rm = run(+1), run(-1)
    for k in range(3):
        fd = (rp[k] - rm[k]) / (2 * h)
        np.testing.assert_allclose(du[k], fd, rtol=1e-4, atol=1e-5 * np.max(np.abs(fd)))


def test_window_shift(oracle):
    N = 30
    P = oracle.params(dim=1, n=(N, 1, 1), V=0.8 / 0.05 / 3.0, dt=0.05, z0=10 * 0.8)  # V dt / dx = 1/3
    phi, cs, cl = I.planar_front(1, (N,), 0.8, P["z0"], P["ke"])
    a = oracle.step(P, phi, cs, cl, 2)          # steps 0,1: floor(V t/dx) = 0
    assert a[3] == 0
    b = oracle.step(P, *a[:3], 1, n0=2, shift=0)  # step 2 -> t3: floor(1) = 1 > 0 -> shift
    assert b[3] == 1
    Pn = dict(P, V=0.0)  # same update without the window (temperature differs by V t only via cleq)
    assert b[0][-1] == 0.0 and b[1][-1] == P["ke"] and b[2][-1] == 1.0
    # interior cells moved down by one: compare with the unshifted update of the same step
    c = oracle.step(dict(P, V=P["V"]), *a[:3], 1, n0=2, shift=0)
    np.testing.assert_array_equal(b[0], c[0])
    u = oracle.step(dict(P, V=P["V"] * 0.999), *a[:3], 1, n0=2, shift=0)  # no shift: floor(0.999) = 0
    assert u[3] == 0
    del Pn


@pytest.mark.parametrize("model", [0, 1])
def test_openmp_build_is_bit_identical(oracle, model):
    """The all-cores timing build (OpenMP cell loops) steps exactly as the
    single-thread build: every cell is independent within a step."""
    import os
    P = oracle.params(dim=3, n=(12, 10, 16), periodic=(1, 0, 0), V=0.6, dt=0.03, z0=5 * 0.8, model=model)
    phi, cs, cl = (a.ravel() for a in I.planar_front(3, P["n"], 0.8, P["z0"], P["ke"], amp=0.05, seed=3))
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "4"
    try:
        a = oracle.step(P, phi, cs, cl, 80)
        b = oracle.step(P, phi, cs, cl, 80, openmp=True)
    finally:
        if old is None:
            os.environ.pop("OMP_NUM_THREADS")
        else:
            os.environ["OMP_NUM_THREADS"] = old
    assert a[3] == b[3] and a[3] >= 1
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
