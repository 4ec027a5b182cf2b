"""Pins of the oracle's Ewald sum: Madelung constants and splitting independence."""
import os

import numpy as np

import qmc_inputs as qi

GOLD = os.path.join(os.path.dirname(__file__), "golden", "madelung.txt")


def _gold():
    out = {}
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_rocksalt_madelung(orc):
    M = _gold()["rocksalt"]
    a = 2.0
    na = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * a
    cl = na + np.array([.5, 0, 0]) * a
    pos = np.vstack([na, cl])
    q = np.array([1.0] * 4 + [-1.0] * 4)
    for kl in [3.0, 5.0, 8.0]:
        E = orc.ewald(pos, q, a, kl / a)
        assert abs(-E / 4 * (a / 2) - M) < 1e-9


def test_simple_cubic_jellium_madelung(orc):
    alpha = _gold()["simple_cubic_jellium"]
    for L in [1.0, 3.7]:
        for kl in [3.0, 5.0, 8.0]:
            E = orc.ewald(np.array([[0.3, 0.1, 0.7]]), np.array([1.0]), L, kl / L)
            assert abs(-2 * L * E - alpha) < 1e-8


def test_kappa_independence_and_translation(orc):
    rng = np.random.default_rng(4)
    L = 4.0
    pos = rng.uniform(0, L, size=(10, 3))
    q = rng.choice([-1.0, 1.0, 2.0], size=10)
    Es = [orc.ewald(pos, q, L, kl / L) for kl in (3.0, 5.0, 8.0)]
    assert max(Es) - min(Es) < 1e-10 * max(1.0, abs(Es[0]))
    shifted = (pos + np.array([0.37, -1.2, 5.5])) % L
    assert abs(orc.ewald(shifted, q, L) - Es[1]) < 1e-10 * max(1.0, abs(Es[1]))


def test_two_charges_far_apart_approach_bare_coulomb_difference(orc):
    # In a huge cell the energy difference between two separations of a +1/-1
    # pair is the bare Coulomb difference (the open-boundary form of v_C = 1/r).
    L = 400.0
    def E(d):
        return orc.ewald(np.array([[0, 0, 0], [d, 0, 0]]) + 100.0, np.array([1.0, -1.0]), L)
    assert abs((E(2.0) - E(1.0)) - (-1 / 2.0 + 1 / 1.0)) < 1e-6


def test_potential_components_independent_of_kappa(orc):
    wl = qi.solid(16, 8, n_walkers=1, n_sweeps=1)
    rng = np.random.default_rng(6)
    pos = rng.uniform(0, wl.L, size=(wl.n_elec, 3))
    vals = [orc.OracleSystem(wl, kappa=kl / wl.L).local_energy(pos) for kl in (3.0, 5.0, 8.0)]
    vals = np.array(vals)
    assert np.abs(vals.max(0) - vals.min(0)).max() < 1e-10 * np.abs(vals).max()
