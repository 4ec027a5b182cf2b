"""Particle-by-particle drift-diffusion sweeps in the oracle (section "Trial Moves": each
electron's move drawn from the transition probability with the wavefunction force F = 2 grad
ln Psi and lambda = 1/2, tau = sigma^2, accepted by eq. accept_reject with the ratio of the
transition probabilities): pinned against the all-electron drift move for one electron, and
against proposals, transition ratios and decisions recomputed here from finite-difference
drift velocities of numpy determinants and a Jastrow sum written out here."""
import dataclasses

import numpy as np

import oracle
import qmc_inputs as qi


def _min_image(d, L):
    return d - L * np.rint(d / L)


def _ln_psi(osys, wl, pos):
    """ln|D_up D_dn| from numpy determinants of the orbital values plus J = sum_{i<j} u2 +
    sum_{i,I} u1 (minimum image, the oracle's radial functions)."""
    out = 0.0
    for off, n in ((0, wl.n_up), (wl.n_up, wl.n_dn)):
        if n:
            A = np.array([osys.spo_vgl(pos[off + k])[0][:n] for k in range(n)])
            out += np.log(abs(np.linalg.det(A)))
    N = wl.n_elec
    for i in range(N):
        for j in range(i + 1, N):
            r = np.linalg.norm(_min_image(pos[i] - pos[j], wl.L))
            same = (i < wl.n_up) == (j < wl.n_up)
            out += osys.radial(1 if same else 2, r)[0]
        for I in range(wl.n_ions):
            out += osys.radial(3, np.linalg.norm(_min_image(pos[i] - wl.ion_pos[I], wl.L)))[0]
    return out


def _fd_velocity(osys, wl, pos, i, h=1e-5):
    """grad_i ln|Psi| by central differences."""
    v = np.zeros(3)
    for a in range(3):
        p, m = pos.copy(), pos.copy()
        p[i, a] += h
        m[i, a] -= h
        v[a] = (_ln_psi(osys, wl, p) - _ln_psi(osys, wl, m)) / (2 * h)
    return v


def _system(sigma, seed=7):
    wl = dataclasses.replace(qi.solid(6, 12, n_walkers=6, n_sweeps=1, sigma=sigma), drift=True)
    wl.n_up, wl.n_dn, wl.n_orb = 3, 3, 3
    wl.coefs = qi.solid_table(3, 12, seed=seed, dtype=np.float64)
    return wl


def test_one_electron_sweep_is_the_all_electron_drift_move():
    """With one electron the particle-by-particle drift move and the all-electron drift move
    propose the same r' from the same counters with the same velocity, and take the same
    uniform and the same acceptance ratio, so the chains coincide decision by decision."""
    wl = qi.solid(2, 12, n_walkers=6, n_sweeps=1, sigma=0.25)
    wl.n_up, wl.n_dn, wl.n_orb = 1, 0, 1
    wl.coefs = qi.solid_table(1, 12, seed=3, dtype=np.float64)
    pb = oracle.OracleSystem(dataclasses.replace(wl, drift=True)).run(range(6), 120, measure_every=0)
    ae = oracle.OracleSystem(dataclasses.replace(wl, drift=True, all_electron=True)).run(range(6), 120,
                                                                                       measure_every=0)
    assert np.array_equal(pb["accept"], ae["accept"])
    assert 0.2 < pb["accept"].mean() < 0.97
    assert np.allclose(pb["final_pos"], ae["final_pos"], rtol=0, atol=1e-12)


def test_drift_sweeps_match_a_finite_difference_recompute():
    """Every move of a sweep, in order: the velocity at the current configuration (the
    earlier moves of the sweep applied) and at the proposal by central differences, the
    proposal r_i + tau v + sigma xi, |Psi'/Psi|^2 from numpy determinants and the Jastrow sum,
    the Gaussian densities T(r -> r') and T(r' -> r) written out in full, and the decision
    from the ACCEPT draw; then the positions after the sweep."""
    wl = _system(0.3)
    tau = wl.sigma ** 2
    osys = oracle.OracleSystem(wl)
    rng = np.random.default_rng(5)
    W, sweeps = 4, 3
    init = rng.uniform(0.0, wl.L, size=(W, wl.n_elec, 3))
    res = osys.run(range(W), sweeps, measure_every=0, init_pos=init, trace=True)

    def log_t(frm, to, v_frm):
        d = to - frm - tau * v_frm
        return -np.sum(d * d) / (2 * tau)

    n_acc = n_moves = 0
    for w in range(W):
        R = init[w].copy()
        for s in range(sweeps):
            for i in range(wl.n_elec):
                xi = oracle.gauss3(wl.seed, w, s, i)
                v = _fd_velocity(osys, wl, R, i)
                rp_unwrapped = R[i] + tau * v + wl.sigma * xi
                Rp = R.copy()
                Rp[i] = np.mod(rp_unwrapped, wl.L)
                vp = _fd_velocity(osys, wl, Rp, i)
                ln_ratio = (2 * (_ln_psi(osys, wl, Rp) - _ln_psi(osys, wl, R))
                            + log_t(rp_unwrapped, R[i], vp) - log_t(R[i], rp_unwrapped, v))
                u = oracle.accept_uniform(wl.seed, w, s, i)
                assert abs(np.log(u) - ln_ratio) > 1e-5, "near tie: choose another seed"
                acc = np.log(u) < ln_ratio
                assert bool(res["accept"][w, s, i]) == acc, (w, s, i)
                if acc:
                    R = Rp
                n_acc += acc
                n_moves += 1
            assert np.allclose(res["trace"][w, s], R, rtol=0, atol=1e-8)
    assert 0.1 * n_moves < n_acc < 0.97 * n_moves


def test_drift_sweeps_cut_the_rejections_of_small_steps():
    """The drift-diffusion proposal follows |Psi|^2 more closely than the plain Gaussian of the
    same width: fewer rejections, where a sign mistake in the drift or the T ratio makes more."""
    ids = range(32)
    for sigma in (0.06, 0.12):
        rej = {}
        for name, drift in (("plain", False), ("drift", True)):
            wl = dataclasses.replace(_system(sigma), drift=drift)
            r = oracle.OracleSystem(wl).run(ids, 30, measure_every=0)
            rej[name] = 1.0 - r["accept"].mean()
        assert rej["plain"] > 0.02
        assert rej["drift"] < 0.6 * rej["plain"], (sigma, rej)


def test_drift_sweep_logdet_follows_fresh_determinants():
    """Accepted moves update the inverse by Sherman-Morrison; the accumulated log|D| and signs
    after the sweeps equal a fresh LU of the final positions."""
    wl = _system(0.3)
    r = oracle.OracleSystem(wl).run(range(6), 8, measure_every=0)
    np.testing.assert_allclose(r["logdet"], r["logdet_lu"], atol=1e-9)
