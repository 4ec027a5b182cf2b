"""All-electron moves in the oracle (section "Trial Moves" with every coordinate proposed at
once): pinned against the particle-by-particle chain for one electron, and against decisions
recomputed with numpy determinants and a Jastrow sum written out here."""
import dataclasses

import numpy as np
import pytest

import oracle
import qmc_inputs as qi


def _one_electron(ae: bool):
    wl = qi.solid(2, 12, n_walkers=6, n_sweeps=1)
    wl.n_up, wl.n_dn, wl.n_orb = 1, 0, 1
    wl.coefs = qi.solid_table(1, 12, seed=3, dtype=np.float64)
    return dataclasses.replace(wl, all_electron=ae)


def test_one_electron_all_electron_chain_is_the_particle_by_particle_chain():
    """With one electron both moves propose the same r' from the same counters and use the
    same uniform; the acceptance ratio is the same number (v.B vs a ratio of determinants), so
    the chains coincide decision by decision."""
    ref = oracle.OracleSystem(_one_electron(False)).run(range(6), 120, measure_every=0)
    ae = oracle.OracleSystem(_one_electron(True)).run(range(6), 120, measure_every=0)
    assert np.array_equal(ref["accept"], ae["accept"])
    assert 0.2 < ae["accept"].mean() < 0.95
    assert np.allclose(ref["final_pos"], ae["final_pos"], rtol=0, atol=1e-12)


def _min_image(d, L):
    return d - L * np.rint(d / L)


def _jastrow(osys, wl, pos):
    """J = sum_{i<j} u2(r_ij) + sum_{i,I} u1(r_iI), minimum image, from the radial functions."""
    N = wl.n_elec
    J = 0.0
    for i in range(N):
        for j in range(i + 1, N):
            r = np.linalg.norm(_min_image(pos[i] - pos[j], wl.L))
            same = (i < wl.n_up) == (j < wl.n_up)
            J += osys.radial(1 if same else 2, r)[0]
        for I in range(wl.n_ions):
            r = np.linalg.norm(_min_image(pos[i] - wl.ion_pos[I], wl.L))
            J += osys.radial(3, r)[0]
    return J


def _slater_dets(osys, wl, pos):
    out = []
    for off, n in ((0, wl.n_up), (wl.n_up, wl.n_dn)):
        A = np.array([osys.spo_vgl(pos[off + k])[0][:n] for k in range(n)]).reshape(n, n)
        out.append(np.linalg.det(A) if n else 1.0)
    return out


def test_decisions_match_determinants_and_jastrow_recomputed_here():
    wl = dataclasses.replace(qi.solid(6, 12, n_walkers=8, n_sweeps=1, sigma=0.15), all_electron=True)
    wl.n_up, wl.n_dn, wl.n_orb = 3, 3, 3
    wl.coefs = qi.solid_table(3, 12, seed=7, dtype=np.float64)
    osys = oracle.OracleSystem(wl)
    rng = np.random.default_rng(11)
    W, steps = 8, 6
    init = rng.uniform(0.0, wl.L, size=(W, wl.n_elec, 3))
    res = osys.run(range(W), steps, measure_every=0, init_pos=init, trace=True)
    n_acc = 0
    for w in range(W):
        R = init[w]
        for s in range(steps):
            xi = np.array([oracle.gauss3(wl.seed, w, s, i) for i in range(wl.n_elec)])
            Rp = np.mod(R + wl.sigma * xi, wl.L)
            d0, d1 = _slater_dets(osys, wl, R)
            p0, p1 = _slater_dets(osys, wl, Rp)
            ratio2 = (p0 * p1 / (d0 * d1)) ** 2 * np.exp(2.0 * (_jastrow(osys, wl, Rp) - _jastrow(osys, wl, R)))
            u = oracle.accept_uniform(wl.seed, w, s, 0)
            acc = u < ratio2
            assert abs(u - ratio2) > 1e-9 * max(ratio2, 1.0), "near tie: choose another seed"
            assert bool(res["accept"][w, s, 0]) == acc and np.all(res["accept"][w, s] == acc)
            R = Rp if acc else R
            assert np.allclose(res["trace"][w, s], R, rtol=0, atol=1e-12)
            n_acc += acc
    assert 0 < n_acc < W * steps


def _ln_psi(osys, wl, pos):
    d0, d1 = _slater_dets(osys, wl, pos)
    return np.log(abs(d0 * d1)) + _jastrow(osys, wl, pos)


def _fd_velocity(osys, wl, pos, h=1e-5):
    """grad ln|Psi| by central differences of ln|Psi| (numpy determinants, the Jastrow sum
    written out above): independent of the oracle's analytic gradients."""
    v = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for a in range(3):
            p, m = pos.copy(), pos.copy()
            p[i, a] += h
            m[i, a] -= h
            v[i, a] = (_ln_psi(osys, wl, p) - _ln_psi(osys, wl, m)) / (2 * h)
    return v


def _drift_system(sigma):
    wl = dataclasses.replace(qi.solid(6, 12, n_walkers=6, n_sweeps=1, sigma=sigma),
                             all_electron=True, drift=True)
    wl.n_up, wl.n_dn, wl.n_orb = 3, 3, 3
    wl.coefs = qi.solid_table(3, 12, seed=7, dtype=np.float64)
    return wl


def test_drift_moves_match_a_finite_difference_recompute():
    """Drift-diffusion all-electron moves (eq. trans_prob_alle with F = 2 grad ln Psi, lambda =
    1/2, tau = sigma^2; acceptance eq. accept_reject): proposals, T ratios and decisions
    recomputed here from finite-difference drift velocities and the Gaussian densities
    written out in full (not the oracle's closed form of their ratio)."""
    wl = _drift_system(0.2)
    tau = wl.sigma ** 2
    osys = oracle.OracleSystem(wl)
    rng = np.random.default_rng(5)
    W, steps = 6, 5
    init = rng.uniform(0.0, wl.L, size=(W, wl.n_elec, 3))
    res = osys.run(range(W), steps, measure_every=0, init_pos=init, trace=True)
    n_acc = 0

    def log_t(frm, to, v_frm):
        # ln T(frm -> to) up to the common normalisation; displacements unwrapped
        d = to - frm - tau * v_frm
        return -np.sum(d * d) / (2 * tau)

    for w in range(W):
        R = init[w]
        for s in range(steps):
            xi = np.array([oracle.gauss3(wl.seed, w, s, i) for i in range(wl.n_elec)])
            vR = _fd_velocity(osys, wl, R)
            Rp_unwrapped = R + tau * vR + wl.sigma * xi
            Rp = np.mod(Rp_unwrapped, wl.L)
            vP = _fd_velocity(osys, wl, Rp)
            ln_ratio = (2 * (_ln_psi(osys, wl, Rp) - _ln_psi(osys, wl, R))
                        + log_t(Rp_unwrapped, R, vP) - log_t(R, Rp_unwrapped, vR))
            u = oracle.accept_uniform(wl.seed, w, s, 0)
            assert abs(np.log(u) - ln_ratio) > 1e-5, "near tie: choose another seed"
            acc = np.log(u) < ln_ratio
            assert np.all(res["accept"][w, s] == acc), (w, s)
            R = Rp if acc else R
            assert np.allclose(res["trace"][w, s], R, rtol=0, atol=1e-8)
            n_acc += acc
    assert 0 < n_acc < W * steps


def test_drift_cuts_the_rejections_of_small_steps():
    """The drift-diffusion proposal follows |Psi|^2 more closely than the plain Gaussian of the
    same width, so the drift moves are rejected less often (about half as often on this
    small system with random orbitals, whose many nodes keep both rates well above zero); a
    sign or index mistake in the drift or in the T ratio makes them worse than the plain moves
    instead."""
    ids = range(48)
    for sigma in (0.03, 0.06):
        rej = {}
        for name, drift in (("plain", False), ("drift", True)):
            wl = dataclasses.replace(_drift_system(sigma), drift=drift)
            r = oracle.OracleSystem(wl).run(ids, 40, measure_every=0)
            rej[name] = 1.0 - r["accept"][:, :, 0].mean()
        assert rej["plain"] > 0.05
        assert rej["drift"] < 0.6 * rej["plain"], (sigma, rej)
