"""Pins of the oracle's diffusion Monte Carlo (section "Diffusion Monte Carlo"): the weight
update, branching, estimator and trial-energy feedback recomputed here from the oracle's own
per-step outputs with the rules written out independently; the exact eigenstate case; and
the fixed-node constraint along every lineage."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import qmc_inputs as qi

HEG14_TKIN = 6.0 * (2.0 * math.pi / qi.cell_side(14)) ** 2


def _dmc_wl(sigma=0.2, all_electron=True):
    """Drift-diffusion moves of all electrons at once, or particle by particle (one sweep per
    step, tau = sigma^2 per electron move; a single electron's move is accepted far more often
    than a move of all 14, so it takes twice the width)."""
    if not all_electron:
        sigma = sigma * 2.0
    return dataclasses.replace(qi.heg14(), all_electron=all_electron, drift=True, sigma=sigma)


def _plan(mult):
    """Free slots (multiplicity 0) in ascending order take the extra copies, sources in
    ascending order, each source's M - 1 copies in a row; the rest are dropped."""
    extra = [j for j, m in enumerate(mult) for _ in range(max(m - 1, 0))]
    free = [f for f, m in enumerate(mult) if m == 0]
    plan = -np.ones(len(mult), dtype=np.int64)
    for f, j in zip(free, extra):
        plan[f] = j
    return plan, max(len(extra) - len(free), 0)


@pytest.mark.parametrize("all_electron", [True, False])
def test_branching_weights_estimator_and_feedback_recomputed(all_electron):
    wl = _dmc_wl(all_electron=all_electron)
    tau = wl.sigma ** 2
    n_slots, n_target, steps, fb = 40, 24, 40, 0.5
    r = oracle.OracleSystem(wl).dmc(n_slots, n_target, steps, feedback=fb)
    st, w, m, pl, en = r["stats"], r["weights"], r["mult"], r["plan"], r["energies"]
    alive = np.arange(n_slots) < n_target
    prev_e = None
    n_copies = n_deaths = 0
    for k in range(steps):
        assert np.array_equal(w[k] > 0, alive)
        et = st[k, 3]
        if prev_e is not None:
            # eqs. pmc:g_growth, pmc:walker_weight from weight 1 after the previous branching
            ref = np.exp(-tau * (prev_e[alive] + en[k][alive] - 2.0 * et) / 2.0)
            assert np.allclose(w[k][alive], ref, rtol=1e-13, atol=0)
        # eq. pmc:weighted_average
        e_mix = np.sum(w[k][alive] * en[k][alive]) / np.sum(w[k][alive])
        assert abs(st[k, 0] - e_mix) < 1e-12 * max(abs(e_mix), 1.0)
        assert abs(st[k, 1] - np.sum(w[k][alive])) < 1e-12 * n_slots
        # M = INT(w + xi)
        xi = np.array([oracle.branch_uniform(wl.seed, j, k) for j in range(n_slots)])
        mult = np.where(alive, np.floor(w[k] + xi), 0).astype(np.int64)
        assert np.array_equal(m[k], mult)
        plan, dropped = _plan(mult)
        assert np.array_equal(pl[k], plan)
        assert st[k, 4] == dropped
        new_alive = (mult >= 1) | (plan >= 0)
        assert st[k, 2] == new_alive.sum()
        n_copies += int((plan >= 0).sum())
        n_deaths += int((alive & (mult == 0)).sum())
        # energies carried into the next step: a copy takes its source's
        prev_e = np.where(plan >= 0, en[k][np.maximum(plan, 0)], en[k])
        if k + 1 < steps:
            assert abs(st[k + 1, 3] - (e_mix - fb * math.log(new_alive.sum() / n_target))) < 1e-12 * max(abs(e_mix), 1)
        alive = new_alive
    assert n_copies > 0 and n_deaths > 0   # both births and deaths


@pytest.mark.parametrize("all_electron", [True, False])
def test_exact_eigenstate_keeps_unit_weights(all_electron):
    """The closed-shell plane-wave determinant without Jastrow is an eigenstate of the kinetic
    Hamiltonian: E_L is the eigenvalue at every configuration, so with E_T = E_L every weight
    stays 1, nothing branches and every estimate is the eigenvalue."""
    wl = dataclasses.replace(qi.heg14(jastrow=False, hamiltonian="kinetic"), all_electron=all_electron,
                             drift=True, sigma=0.3)
    r = oracle.OracleSystem(wl, spo="planewave").dmc(12, 8, 25, feedback=1.0)
    st = r["stats"]
    assert np.abs(st[:, 0] - HEG14_TKIN).max() < 1e-12 * HEG14_TKIN
    assert np.abs(st[:, 3] - HEG14_TKIN).max() < 1e-12 * HEG14_TKIN
    assert np.all(st[:, 2] == 8) and np.all(r["plan"] == -1)
    assert np.abs(r["weights"][:, :8] - 1.0).max() < 1e-12


def _sign_psi(osys, wl, pos):
    """sign(D_up D_dn) from numpy determinants of the orbital values (the Jastrow factor is
    positive)."""
    sgn = 1.0
    for off, n in ((0, wl.n_up), (wl.n_up, wl.n_dn)):
        if n:
            A = np.array([osys.spo_vgl(pos[off + k])[0][:n] for k in range(n)])
            sgn *= np.sign(np.linalg.det(A))
    return int(sgn)


@pytest.mark.parametrize("all_electron", [True, False])
def test_fixed_node_keeps_the_sign_of_every_lineage(all_electron):
    """Moves across a node are proposed (and rejected) and a copy carries its source's sign,
    so every final walker has its initial ancestor's sign of Psi, checked here with numpy
    determinants at the final positions."""
    wl = _dmc_wl(0.35, all_electron)
    n_slots, n_target, steps = 40, 24, 30
    osys = oracle.OracleSystem(wl)
    r = osys.dmc(n_slots, n_target, steps, feedback=0.5)
    assert r["stats"][:, 5].sum() > 0
    init = osys.run(range(n_target), 0, measure_every=0)["final_pos"]
    s0 = np.array([_sign_psi(osys, wl, p) for p in init])
    ancestor = np.arange(n_slots)
    for k in range(steps):
        plan = r["plan"][k]
        ancestor = np.where(plan >= 0, ancestor[np.maximum(plan, 0)], ancestor)
    alive = np.flatnonzero(r["final_sign"] != 0)
    assert len(alive) == r["stats"][-1, 2]
    for j in alive:
        assert _sign_psi(osys, wl, r["final_pos"][j]) == s0[ancestor[j]] == r["final_sign"][j]


def test_multiplicities_are_capped_at_the_capacity():
    """A first trial energy far above the local energies makes every weight huge (about 1e12
    after one step): every multiplicity is capped at the number of slots, the free slots take
    the copies of the lowest alive slots, and every extra copy asked for and not placed counts
    as dropped, sum(INT(w + xi) - 1) - placed, computed here from the weights and draws."""
    wl = _dmc_wl(0.2)
    tau = wl.sigma ** 2
    n_slots, n_target = 16, 8
    osys = oracle.OracleSystem(wl)
    e_mean = osys.dmc(n_slots, n_target, 1)["stats"][0, 3]   # the first E_T: the mean local energy
    r = osys.dmc(n_slots, n_target, 1, e_trial=e_mean + 28.0 / tau, feedback=0.0)
    w, m, pl, st = r["weights"][0], r["mult"][0], r["plan"][0], r["stats"][0]
    alive = np.arange(n_slots) < n_target
    xi = np.array([oracle.branch_uniform(wl.seed, j, 0) for j in range(n_slots)])
    raw = np.where(alive, np.floor(w + xi), 0.0)
    assert raw[alive].min() > 1e10
    assert np.array_equal(m, np.where(alive, np.minimum(raw, n_slots), 0).astype(np.int64))
    plan, _ = _plan(m)
    assert np.array_equal(pl, plan)
    assert np.array_equal(plan[n_target:], np.zeros(n_slots - n_target, dtype=np.int64))   # all from slot 0
    assert st[4] == np.sum(raw[alive] - 1.0) - (plan >= 0).sum()
    assert st[2] == n_slots
