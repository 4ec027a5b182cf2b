"""Pins of the oracle's Jastrow radial functions and their use in the local energy."""
import math

import numpy as np

import qmc_inputs as qi


def _wl(j2=None, j1=None, n_up=1, n_dn=1, L=10.0, ions=None, coefs=None, hamiltonian="kinetic"):
    if coefs is None:
        coefs = np.ones((4, 4, 4, max(n_up, n_dn, 1)))   # constant orbital(s)
    ion_pos = np.zeros((0, 3)) if ions is None else np.asarray(ions, dtype=float)
    return qi.Workload(name="t", n_up=n_up, n_dn=n_dn, L=L, n_orb=coefs.shape[3],
                       grid=coefs.shape[:3], coefs=coefs, ion_pos=ion_pos,
                       ion_Z=np.full(len(ion_pos), 1.0), j2=j2, j1=j1, hamiltonian=hamiltonian,
                       sigma=0.3, seed=0, n_walkers=1, n_sweeps=1)


def test_pade_closed_form(orc):
    a, b = 0.5, 1.0
    sys = orc.OracleSystem(_wl(j2={"kind": "pade", "a": a, "b": b}))
    for r in [0.0, 0.1, 0.7, 2.5, 9.0]:
        u, du, d2u = sys.radial(2, r)
        assert abs(u - a * r / (1 + b * r)) < 1e-15
        assert abs(du - a / (1 + b * r) ** 2) < 1e-15
        assert abs(d2u + 2 * a * b / (1 + b * r) ** 3) < 1e-15


def _bspline_j2(M=8, rc=3.0, A=0.4):
    return {"kind": "bspline", "M": M, "rc": rc, "p": qi.bspline_jastrow_params(M, A),
            "cusp_same": 0.25, "cusp_opp": 0.5}


def test_bspline_cusp_and_cutoff(orc):
    j2 = _bspline_j2()
    j1 = {"kind": "bspline", "M": 8, "rc": 3.0, "p": qi.bspline_jastrow_params(8, 0.3), "cusp": 0.0}
    sys = orc.OracleSystem(_wl(j2=j2, j1=j1, ions=[[1.0, 1.0, 1.0]]))
    assert abs(sys.radial(1, 0.0)[1] - 0.25) < 1e-13       # same-spin cusp
    assert abs(sys.radial(2, 0.0)[1] - 0.5) < 1e-13        # opposite-spin cusp
    assert abs(sys.radial(3, 0.0)[1] - 0.0) < 1e-13        # no electron-ion cusp
    for kind in (1, 2, 3):
        below = sys.radial(kind, 3.0 - 1e-7)
        assert np.all(np.abs(below) < 1e-6)                # u, u', u'' -> 0 at rc when p_M = 0
        assert np.all(sys.radial(kind, 3.0) == 0.0)
        assert np.all(sys.radial(kind, 4.0) == 0.0)


def test_bspline_values_at_knots(orc):
    # At r = (m-1) delta the cubic B-spline sum is (p_{m-1} + 4 p_m + p_{m+1}) / 6.
    M, rc = 8, 3.0
    j2 = _bspline_j2(M, rc)
    sys = orc.OracleSystem(_wl(j2=j2))
    delta = rc / M
    p = list(j2["p"]) + [0.0, 0.0]
    p0 = p[1] - 2 * delta * 0.5                              # opposite-spin cusp
    pp = [p0] + p                                           # pp[m] = p_m
    for m in range(1, M):
        r = (m - 1) * delta
        expect = (pp[m - 1] + 4 * pp[m] + pp[m + 1]) / 6.0
        assert abs(sys.radial(2, r)[0] - expect) < 1e-14


def test_bspline_derivatives_match_finite_differences(orc):
    sys = orc.OracleSystem(_wl(j2=_bspline_j2()))
    h = 1e-5
    for r in [0.05, 0.4, 1.1, 1.9, 2.6]:
        u, du, d2u = sys.radial(1, r)
        up, um = sys.radial(1, r + h)[0], sys.radial(1, r - h)[0]
        assert abs(du - (up - um) / (2 * h)) < 1e-8
        assert abs(d2u - (up - 2 * u + um) / h ** 2) < 1e-4


def test_two_electron_kinetic_closed_form(orc):
    # Constant orbitals, one up and one down electron, Pade J2: grad_1 J = u' r_hat,
    # lap_1 J = u'' + 2u'/r, so T_L = -(u'' + 2u'/r + u'^2) (both electrons alike).
    a, b = 0.5, 1.0
    sys = orc.OracleSystem(_wl(j2={"kind": "pade", "a": a, "b": b}))
    for r in [0.3, 1.0, 2.2]:
        pos = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
        T = sys.local_energy(pos)[0]
        du = a / (1 + b * r) ** 2
        d2u = -2 * a * b / (1 + b * r) ** 3
        assert abs(T - (-(d2u + 2 * du / r + du * du))) < 1e-13


def test_local_energy_matches_finite_differences_of_log_psi(orc):
    # T_L = -1/2 sum_i [lap_i ln|Psi| + |grad_i ln|Psi||^2], with ln|Psi| recomputed
    # from scratch (fresh LU and full Jastrow) at displaced positions.
    wl = qi.solid(6, 12, n_walkers=1, n_sweeps=1, ions_per_elec=0.5)
    wl.hamiltonian = "kinetic"
    sys = orc.OracleSystem(wl)
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, wl.L, size=(wl.n_elec, 3))
    T = sys.local_energy(pos)[0]
    h = 1e-4
    lp0 = sys.log_psi(pos)[0]
    acc = 0.0
    for i in range(wl.n_elec):
        for a in range(3):
            p, m = pos.copy(), pos.copy()
            p[i, a] += h
            m[i, a] -= h
            lpp, lpm = sys.log_psi(p)[0], sys.log_psi(m)[0]
            g = (lpp - lpm) / (2 * h)
            lap = (lpp - 2 * lp0 + lpm) / h ** 2
            acc += lap + g * g
    T_fd = -0.5 * acc
    assert abs(T - T_fd) < 1e-5 * max(1.0, abs(T)), (T, T_fd)
