"""Pins of the oracle's periodic tricubic B-spline orbitals.

Marsden's identity for the uniform cubic B-spline with integer knots:
sum_j B(t-j) = 1, sum_j j B(t-j) = t, sum_j (j^2 - 1/3) B(t-j) = t^2,
sum_j (j^3 - j) B(t-j) = t^3.  A table filled with these coefficients for a
cubic polynomial per axis reproduces the polynomial, its gradient and its
Laplacian exactly wherever the 4x4x4 stencil does not cross the periodic seam.
"""
import numpy as np

import qmc_inputs as qi


def _marsden_coefs(a, j):
    j = np.asarray(j, dtype=np.float64)
    return a[0] + a[1] * j + a[2] * (j * j - 1.0 / 3.0) + a[3] * (j ** 3 - j)


def _poly(a, t):
    return (a[0] + a[1] * t + a[2] * t * t + a[3] * t ** 3,
            a[1] + 2 * a[2] * t + 3 * a[3] * t * t,
            2 * a[2] + 6 * a[3] * t)


def _workload(coefs, L, n_up=1, n_dn=0):
    g = coefs.shape[0]
    return qi.Workload(name="t", n_up=n_up, n_dn=n_dn, L=L, n_orb=coefs.shape[3], grid=(g, g, g),
                       coefs=coefs, ion_pos=np.zeros((0, 3)), ion_Z=np.zeros(0), j2=None, j1=None,
                       hamiltonian="kinetic", sigma=0.3, seed=0, n_walkers=1, n_sweeps=1)


def test_marsden_polynomial_reproduction(orc):
    rng = np.random.default_rng(1)
    G, L, n_orb = 12, 5.0, 3
    h = G / L
    A = rng.normal(size=(n_orb, 3, 4))          # per orbital, per axis cubic coefficients
    j = np.arange(G)
    coefs = np.zeros((G, G, G, n_orb))
    for o in range(n_orb):
        cx, cy, cz = (_marsden_coefs(A[o, k], j) for k in range(3))
        coefs[..., o] = cx[:, None, None] * cy[None, :, None] * cz[None, None, :]
    sys = orc.OracleSystem(_workload(coefs, L))
    worst = 0.0
    for _ in range(200):
        t = rng.uniform(1.0, G - 2.0, size=3)   # stencil stays inside [0, G-1]
        v, g, lap = sys.spo_vgl(t / h)
        for o in range(n_orb):
            px, py, pz = (_poly(A[o, k], t[k]) for k in range(3))
            ev = px[0] * py[0] * pz[0]
            eg = np.array([px[1] * py[0] * pz[0], px[0] * py[1] * pz[0], px[0] * py[0] * pz[1]]) * h
            el = (px[2] * py[0] * pz[0] + px[0] * py[2] * pz[0] + px[0] * py[0] * pz[2]) * h * h
            scale = max(1.0, abs(ev), np.abs(eg).max(), abs(el))
            worst = max(worst, abs(v[o] - ev) / scale, np.abs(g[:, o] - eg).max() / scale,
                        abs(lap[o] - el) / scale)
    assert worst < 1e-13, worst


def test_heg_coefficients_interpolate_plane_waves(orc):
    wl = qi.heg14(jastrow=False)
    sys = orc.OracleSystem(wl)
    G = wl.grid[0]
    rng = np.random.default_rng(2)
    for _ in range(20):
        knot = rng.integers(0, G, size=3)
        r = knot * wl.L / G
        v, _, _ = sys.spo_vgl(r)
        expect = [np.cos(k @ r) if kd == 0 else np.sin(k @ r) for k, kd in zip(wl.pw_k, wl.pw_kind)]
        np.testing.assert_allclose(v, expect, atol=1e-14)


def test_spline_is_periodic_and_smooth_across_the_seam(orc):
    wl = qi.solid(8, 10, n_walkers=1, n_sweeps=1)
    sys = orc.OracleSystem(wl)
    rng = np.random.default_rng(3)
    for _ in range(10):
        r = rng.uniform(0, wl.L, 3)
        shift = rng.integers(-2, 3, size=3) * wl.L
        a = sys.spo_vgl(r)
        b = sys.spo_vgl(r + shift)
        for x, y in zip(a, b):
            np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-12)
    # C2 continuity: value and derivatives just below and above x = 0 (the seam)
    eps = 1e-9
    lo = sys.spo_vgl(np.array([wl.L - eps, 1.1, 2.2]))
    hi = sys.spo_vgl(np.array([eps, 1.1, 2.2]))
    for x, y in zip(lo, hi):
        np.testing.assert_allclose(x, y, rtol=1e-6, atol=1e-6)


def test_spline_gradient_matches_finite_differences(orc):
    wl = qi.solid(8, 10, n_walkers=1, n_sweeps=1)
    sys = orc.OracleSystem(wl)
    r = np.array([1.234, 2.345, 0.456])
    v, g, lap = sys.spo_vgl(r)
    h = 1e-5
    fd_g = np.zeros_like(g)
    fd_l = np.zeros_like(lap)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        vp = sys.spo_vgl(r + e)[0]
        vm = sys.spo_vgl(r - e)[0]
        fd_g[a] = (vp - vm) / (2 * h)
        fd_l += (vp - 2 * v + vm) / (h * h)
    np.testing.assert_allclose(g, fd_g, rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(lap, fd_l, rtol=1e-4, atol=1e-4)
