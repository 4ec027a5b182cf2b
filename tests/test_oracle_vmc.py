"""Pins of the oracle's full particle-by-particle VMC chain."""
import math

import numpy as np

import qmc_inputs as qi

HEG14_TKIN = 6.0 * (2.0 * math.pi / qi.cell_side(14)) ** 2   # 2 spins x 6 shell orbitals x k^2/2


def test_heg14_kinetic_value():
    assert abs(HEG14_TKIN - 15.69278) < 1e-5


def test_plane_wave_electron_gas_has_zero_variance(orc):
    # Variational principle corollary (equation vmc:var_variance): an eigenstate has
    # zero variance of the local energy.  The closed-shell plane-wave determinant
    # without Jastrow is a kinetic eigenstate with E = sum |k|^2 / 2.
    wl = qi.heg14(jastrow=False, hamiltonian="kinetic")
    r = orc.OracleSystem(wl, spo="planewave").run(range(wl.n_walkers), 30, measure_every=1)
    T = r["energies"][..., 0]
    assert np.abs(T - HEG14_TKIN).max() < 1e-12 * HEG14_TKIN
    assert 0.3 < r["accept"].mean() < 0.95


def test_spline_electron_gas_converges_with_grid(orc):
    # A cubic spline of a plane wave is not a Laplacian eigenfunction, so the
    # spline kinetic energy varies with the configuration.  At fixed random
    # configurations the median deviation from sum |k|^2/2 falls as O(G^-2).
    rng = np.random.default_rng(7)
    pos = rng.uniform(0, qi.cell_side(14), size=(60, 14, 3))
    med = []
    for G in (16, 32, 64):
        sys = orc.OracleSystem(qi.heg14(jastrow=False, grid=G, hamiltonian="kinetic"))
        d = np.array([abs(sys.local_energy(p)[0] - HEG14_TKIN) for p in pos])
        med.append(np.median(d))
    assert med[0] / med[1] > 3.0 and med[1] / med[2] > 3.0, med
    assert med[2] < 1e-3 * HEG14_TKIN


def test_metropolis_samples_psi_squared(orc):
    # One electron, one orbital phi(x) = 2 + cos(2 pi x / L): the sampled x must
    # follow |phi|^2 / int |phi|^2 (equation accept_reject, detailed balance).
    L, G = 1.0, 64
    c1 = qi.heg_coefficients(np.array([[0, 0, 0]]), np.array([0]), L, G)
    c2 = qi.heg_coefficients(np.array([[1, 0, 0]]), np.array([0]), L, G)
    coefs = 2.0 * c1 + c2
    wl = qi.Workload(name="p7", n_up=1, n_dn=0, L=L, n_orb=1, grid=(G, G, G), coefs=coefs,
                     ion_pos=np.zeros((0, 3)), ion_Z=np.zeros(0), j2=None, j1=None,
                     hamiltonian="kinetic", sigma=3.0 * L, seed=11, n_walkers=4, n_sweeps=1)
    n_sweeps = 100000
    r = orc.OracleSystem(wl).run(range(4), n_sweeps, measure_every=0, trace=True, bits=False)
    x = r["trace"][:, ::4, 0, 0].ravel()
    nb = 40
    edges = np.linspace(0, L, nb + 1)
    obs, _ = np.histogram(x, edges)
    tp = 2 * math.pi
    F = lambda t: 4.5 * t + 4 / tp * np.sin(tp * t) + np.sin(2 * tp * t) / (4 * tp)
    p = (F(edges[1:]) - F(edges[:-1])) / 4.5
    exp = p * len(x)
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    from scipy.stats import chi2 as chi2dist
    assert chi2dist.sf(chi2, nb - 1) > 1e-3, chi2


def test_accumulated_logdet_matches_fresh_lu(orc):
    wl = qi.solid(16, 12, n_walkers=3, n_sweeps=1)
    r = orc.OracleSystem(wl).run(range(3), 40, measure_every=0)
    np.testing.assert_allclose(r["logdet"], r["logdet_lu"], atol=1e-9)
    assert 0.2 < r["accept"].mean() < 0.95


def test_walker_streams_are_independent(orc):
    wl = qi.solid(16, 12, n_walkers=3, n_sweeps=1)
    sys = orc.OracleSystem(wl)
    a = sys.run([0, 1, 2], 5, measure_every=1)
    b = sys.run([2], 5, measure_every=1)
    assert np.array_equal(a["accept"][2], b["accept"][0])
    assert np.array_equal(a["energies"][2], b["energies"][0])


def test_sweep_replayed_by_full_recomputation(orc):
    # Replay one sweep move by move with ln|Psi| recomputed from scratch (fresh
    # LU and full Jastrow): the acceptance is u < |Psi'/Psi|^2 (equation
    # accept_reject; the no-drift transition probabilities cancel).
    wl = qi.solid(8, 10, n_walkers=2, n_sweeps=1)
    sys = orc.OracleSystem(wl)
    for wid in (0, 1):
        r = sys.run([wid], 2, measure_every=0, trace=True)
        pos = np.array([orc.init_position(wl.seed, wid, i, wl.L) for i in range(wl.n_elec)])
        for s in range(2):
            for i in range(wl.n_elec):
                rp = (pos[i] + wl.sigma * orc.gauss3(wl.seed, wid, s, i)) % wl.L
                trial = pos.copy()
                trial[i] = rp
                lp0, s0 = sys.log_psi(pos)
                lp1, s1 = sys.log_psi(trial)
                u = orc.accept_uniform(wl.seed, wid, s, i)
                ratio = math.exp(2 * (lp1 - lp0))
                acc = u < ratio
                if abs(u - ratio) > 1e-9 * ratio:
                    assert bool(r["accept"][0, s, i]) == acc
                else:
                    acc = bool(r["accept"][0, s, i])
                if acc:
                    pos = trial
            np.testing.assert_allclose(pos, r["trace"][0, s], atol=1e-12)


def test_uniform_configurations_average_to_jellium_madelung(orc):
    # For independent uniform positions the pair terms of the Ewald energy (with
    # the neutralising background) average to zero, leaving N times the energy
    # of one charge with its own images and background, -alpha / (2 L).
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden", "madelung.txt")
    alpha = [float(l.split()[1]) for l in open(gold) if l.startswith("simple_cubic_jellium")][0]
    N, L = 14, qi.cell_side(14)
    rng = np.random.default_rng(8)
    E = np.array([orc.ewald(rng.uniform(0, L, size=(N, 3)), -np.ones(N), L) for _ in range(3000)])
    expect = -N * alpha / (2 * L)
    assert abs(E.mean() - expect) < 5 * E.std() / np.sqrt(len(E)), (E.mean(), expect)


def test_heg14_energy_components(orc):
    wl = qi.heg14()
    r = orc.OracleSystem(wl).run(range(4), 5, measure_every=1)
    E = r["energies"]
    assert np.all(E[..., 2] == 0) and np.all(E[..., 3] == 0)    # no ions
    assert np.all(E[..., 1] < 0) and np.all(E[..., 0] > 0)


def test_initial_configurations_are_plain_uniform_draws(orc):
    """Without given positions a walker starts from uniform draws in the cell, electron i of
    walker w at L (u0, u1, u2) from the INIT counters (i, 0, w) -- no conditioning filter, so
    walker 114 of the 384-electron system keeps its first draw although its up-spin Slater
    matrix has a condition number near 1e8.  The uniforms are recomputed here from the
    Philox4x32-10 blocks (pinned by the published known-answer vectors)."""
    wl = qi.mixed384()
    osys = orc.OracleSystem(wl)
    out = osys.run([114, 0], 0, measure_every=0)
    key = [wl.seed & 0xFFFFFFFF, wl.seed >> 32]

    def u53(o0, o1):
        return ((int(o0) | (int(o1) << 32)) >> 11) * 2.0 ** -53

    for slot, w in enumerate((114, 0)):
        for i in (0, 1, 191, 383):
            a = orc.philox4x32_10([i, 0, w, (1 << 16) | 0], key)
            b = orc.philox4x32_10([i, 0, w, (1 << 16) | 1], key)
            want = wl.L * np.array([u53(a[0], a[1]), u53(a[2], a[3]), u53(b[0], b[1])])
            assert np.array_equal(out["final_pos"][slot][i], want)
    n = wl.n_up
    A = np.array([osys.spo_vgl(out["final_pos"][0][i])[0] for i in range(n)])
    assert np.linalg.cond(A) > 1e7
