"""Pins of the oracle's three-body electron-electron-ion Jastrow term (section "Jastrow
factors", the form of Drummond et al.): its value against a numpy evaluation of the formula
written here, its gradient and Laplacian (inside the kinetic energy) against finite
differences of that evaluation, and the particle-by-particle ratio against full recomputation."""
import dataclasses

import numpy as np

import oracle
import qmc_inputs as qi


def _mi(d, L):
    return d - L * np.rint(d / L)


def _j3(wl, pos):
    """J3 = sum_I sum_{i<j} sum_lmn g_lmn a^l b^m c^n (a - h)^3 (b - h)^3 over a, b < h."""
    p = wl.j3
    h = p["rc"] / 2.0
    g = p["gamma"]
    N = wl.n_elec
    J = 0.0
    for I in range(wl.n_ions):
        R = wl.ion_pos[I]
        for i in range(N):
            a = np.linalg.norm(_mi(pos[i] - R, wl.L))
            if a >= h:
                continue
            for j in range(i + 1, N):
                b = np.linalg.norm(_mi(pos[j] - R, wl.L))
                if b >= h:
                    continue
                c = np.linalg.norm(_mi(pos[i] - pos[j], wl.L))
                gs = g[0 if (i < wl.n_up) == (j < wl.n_up) else 1]
                poly = sum(gs[l, m, n] * a ** l * b ** m * c ** n
                           for l in range(p["m_ei"] + 1) for m in range(p["m_ei"] + 1) for n in range(p["m_ee"] + 1))
                J += poly * (a - h) ** 3 * (b - h) ** 3
    return J


def _system(j3=True, n=16):
    wl = qi.solid(n, 12, n_walkers=4, n_sweeps=1, j3=j3)
    return wl


def _pos_near_ions(wl, rng):
    """Electrons placed within the cutoff of the ions, so that many triples contribute."""
    h = wl.j3["rc"] / 2.0
    idx = rng.integers(0, wl.n_ions, size=wl.n_elec)
    d = rng.normal(size=(wl.n_elec, 3))
    d *= (rng.uniform(0.2, 0.9, size=(wl.n_elec, 1)) * h) / np.linalg.norm(d, axis=1, keepdims=True)
    return np.mod(wl.ion_pos[idx] + d, wl.L)


def test_value_matches_numpy_formula():
    wl = _system()
    rng = np.random.default_rng(3)
    with_j3, without = oracle.OracleSystem(wl), oracle.OracleSystem(dataclasses.replace(wl, j3=None))
    for _ in range(4):
        pos = _pos_near_ions(wl, rng)
        ref = _j3(wl, pos)
        assert abs(ref) > 1e-3
        got = with_j3.log_psi(pos)[0] - without.log_psi(pos)[0]
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))


def test_kinetic_energy_matches_finite_differences():
    """T_L = -1/2 sum_i (lap_i ln Psi + |grad_i ln Psi|^2) with ln Psi recomputed here (numpy
    determinants of the oracle's orbitals, the two-body terms through the oracle's radial
    functions, the three-body term from the formula) and central differences."""
    wl = dataclasses.replace(_system(n=8), hamiltonian="kinetic")
    osys = oracle.OracleSystem(wl)
    base = oracle.OracleSystem(dataclasses.replace(wl, j3=None))
    rng = np.random.default_rng(9)
    pos = _pos_near_ions(wl, rng)

    def ln_psi(x):
        return base.log_psi(x)[0] + _j3(wl, x)

    h = 1e-4
    T = 0.0
    for i in range(wl.n_elec):
        for a in range(3):
            p, m = pos.copy(), pos.copy()
            p[i, a] += h
            m[i, a] -= h
            f0, fp, fm = ln_psi(pos), ln_psi(p), ln_psi(m)
            T += -0.5 * ((fp - 2 * f0 + fm) / h ** 2 + ((fp - fm) / (2 * h)) ** 2)
    got = osys.local_energy(pos)[0]
    assert abs(_j3(wl, pos)) > 1e-3
    assert abs(got - T) < 1e-5 * max(1.0, abs(T)), (got, T)


def test_particle_by_particle_decisions_with_three_body_term():
    """One sweep replayed by full recomputation of ln|Psi| (numpy determinants, the oracle's
    two-body terms, the three-body formula here): every decision agrees."""
    wl = _system(n=8)
    osys = oracle.OracleSystem(wl)
    base = oracle.OracleSystem(dataclasses.replace(wl, j3=None))
    rng = np.random.default_rng(4)
    W = 4
    init = np.array([_pos_near_ions(wl, rng) for _ in range(W)])
    res = osys.run(range(W), 1, measure_every=0, init_pos=init)
    for w in range(W):
        R = init[w].copy()
        for i in range(wl.n_elec):
            xi = oracle.gauss3(wl.seed, w, 0, i)
            Rp = R.copy()
            Rp[i] = np.mod(R[i] + wl.sigma * xi, wl.L)
            lr = 2 * ((base.log_psi(Rp)[0] + _j3(wl, Rp)) - (base.log_psi(R)[0] + _j3(wl, R)))
            u = oracle.accept_uniform(wl.seed, w, 0, i)
            assert abs(np.log(u) - lr) > 1e-8
            acc = np.log(u) < lr
            assert bool(res["accept"][w, 0, i]) == acc
            if acc:
                R = Rp
        assert np.allclose(res["final_pos"][w], R, atol=1e-12)
