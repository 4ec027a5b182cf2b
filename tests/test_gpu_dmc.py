"""GPU parity of diffusion Monte Carlo (section "Diffusion Monte Carlo") against the oracle's
DMC, through the C ABI: per step the mixed estimate, the sum of weights and E_T within 1e-10
relative (FP64; 1e-5 mixed), the population, dropped copies and node-crossing rejections
exactly; at the end the set of alive slots exactly, their positions within 1e-10 bohr and
their signs exactly.  Branching decisions M = INT(w + xi) are integers decided in FP64 on
both sides from weights that agree to rounding."""
import dataclasses

import numpy as np
import pytest

import qmc_inputs as qi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_06922_amd import qmc
    qmc.load_library()
    return qmc


def _drift(wl, sigma):
    return dataclasses.replace(wl, all_electron=True, drift=True, sigma=sigma)


def _compare(gpu, orc, wl, n_slots, n_target, steps, feedback, rel=1e-10, pos_tol=1e-10, e_trial=float("nan")):
    import torch
    print(f"[dmc] {wl.name} {wl.precision} sigma={wl.sigma}: {n_target} of {n_slots} slots, {steps} steps",
          flush=True)
    s = gpu.System(wl, n_walkers=n_slots)
    s.dmc_init(n_target, e_trial=e_trial, feedback=feedback)
    out = torch.zeros((steps, 6), dtype=torch.float64, device="cuda")
    s.dmc_steps(steps, out)
    st = out.cpu().numpy()
    w, _, et, pop = s.dmc_state()
    pos, _, sg = s.get_walkers()
    s.close()
    ref = orc.OracleSystem(wl).dmc(n_slots, n_target, steps, e_trial=e_trial, feedback=feedback)
    rs = ref["stats"]
    print(f"[dmc] population {st[:, 2].min():.0f}..{st[:, 2].max():.0f}, copies dropped {st[:, 4].sum():.0f}, "
          f"node crossings {st[:, 5].sum():.0f}, E {st[-1, 0]:.6f}", flush=True)
    for c in (2, 4, 5):
        assert np.array_equal(st[:, c], rs[:, c]), (c, np.flatnonzero(st[:, c] != rs[:, c])[:3])
    for c in (0, 1, 3):
        err = np.abs(st[:, c] - rs[:, c]) / np.maximum(np.abs(rs[:, c]), 1.0)
        assert err.max() < rel, (c, err.max())
    alive = ref["final_sign"] != 0
    assert np.array_equal(w > 0, alive)
    assert pop == alive.sum()
    np.testing.assert_allclose(pos[alive], ref["final_pos"][alive], rtol=0, atol=pos_tol)
    assert np.array_equal(sg[alive].prod(axis=1), ref["final_sign"][alive])
    return st


def _per_slot(gpu, orc, wl, n_slots, n_target, steps, feedback, rel=1e-10, e_trial=float("nan")):
    """Steps one at a time; after each, every slot's weight and energy before branching, its
    multiplicity and copy source (qmc_dmc_get_branching), and its weight and energy after
    branching (qmc_dmc_get) against the oracle's step."""
    import torch
    print(f"[dmc-slots] {wl.name} {wl.precision}: {n_target} of {n_slots} slots, {steps} steps", flush=True)
    s = gpu.System(wl, n_walkers=n_slots)
    s.dmc_init(n_target, e_trial=e_trial, feedback=feedback)
    with pytest.raises(gpu.QMCError):
        s.dmc_branching()   # no step yet
    out = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
    got = []
    for _ in range(steps):
        s.dmc_steps(1, out)
        got.append((out.cpu().numpy()[0].copy(), *s.dmc_branching(), *s.dmc_state()))
    s.close()
    ref = orc.OracleSystem(wl).dmc(n_slots, n_target, steps, e_trial=e_trial, feedback=feedback)
    copies = 0
    for k, (st, wb, eb, m, pl, w, E, et, pop) in enumerate(got):
        rw, re, rm, rp = ref["weights"][k], ref["energies"][k], ref["mult"][k], ref["plan"][k]
        assert np.array_equal(m, rm), (k, np.flatnonzero(m != rm)[:4])
        assert np.array_equal(pl, rp), (k, np.flatnonzero(pl != rp)[:4])
        was_alive = ~np.isnan(re)
        assert np.array_equal(~np.isnan(eb), was_alive), k
        assert np.all(wb[~was_alive] == 0.0) and np.all(m[~was_alive] == 0)
        assert (np.abs(wb - rw) / np.maximum(np.abs(rw), 1.0)).max() < rel, k
        assert (np.abs(eb[was_alive] - re[was_alive]) / np.maximum(np.abs(re[was_alive]), 1.0)).max() < rel, k
        # after branching: weight 1 where a walker stayed or arrived, and copies carry the
        # energy of their source
        alive = (m >= 1) | (pl >= 0)
        assert np.array_equal(w, alive.astype(np.float64)) and pop == alive.sum() == ref["stats"][k, 2]
        src = np.where(pl >= 0, pl, np.arange(n_slots))
        assert np.all(was_alive[src[alive]])
        np.testing.assert_allclose(E[alive], re[src[alive]], rtol=rel, atol=rel)
        assert (np.abs(st[:2] - ref["stats"][k, :2]) / np.maximum(np.abs(ref["stats"][k, :2]), 1.0)).max() < rel
        assert np.array_equal(st[[2, 4, 5]], ref["stats"][k, [2, 4, 5]])
        copies += int((pl >= 0).sum())
    print(f"[dmc-slots] {copies} copies over {steps} steps, final population {got[-1][-1]}", flush=True)
    return copies


def test_dmc_per_slot_branching_heg14(gpu, orc):
    """Large steps and a high first E_T: copies, deaths, node crossings and dropped copies."""
    assert _per_slot(gpu, orc, _drift(qi.heg14(), 0.3), 32, 20, 16, 0.3, e_trial=5.0) > 0


def test_dmc_multiplicities_capped_at_the_capacity(gpu, orc):
    """A first E_T far above the local energies (weights about 1e12 after the first step):
    multiplicities capped at the slot count, the copy plan, and the dropped copies counted
    from the uncapped multiplicities, as the oracle has them."""
    wl = _drift(qi.heg14(), 0.2)
    e_mean = orc.OracleSystem(wl).dmc(16, 8, 1)["stats"][0, 3]
    _per_slot(gpu, orc, wl, 16, 8, 3, 0.0, e_trial=e_mean + 28.0 / wl.sigma ** 2)


def test_dmc_per_slot_branching_solid128(gpu, orc):
    """The 128-electron solid, 64 slots with 48 alive at the start, 12 steps."""
    assert _per_slot(gpu, orc, _drift(qi.solid128(), 0.03), 64, 48, 12, 1.0) > 0


def test_dmc_per_slot_branching_mixed_precision(gpu, orc):
    wl = qi.solid(48, 16, n_walkers=1, n_sweeps=1, precision="mixed", table_dtype=np.float32)
    _per_slot(gpu, orc, _drift(wl, 0.08), 48, 32, 10, 0.5, rel=1e-5)


def test_dmc_heg14(gpu, orc):
    st = _compare(gpu, orc, _drift(qi.heg14(), 0.2), 40, 24, 40, 0.5)
    assert st[:, 2].min() != st[:, 2].max()   # the population moved


def test_dmc_ragged_solid_with_ions(gpu, orc):
    wl = qi.solid(18, 14, n_walkers=1, n_sweeps=1)
    wl.n_up, wl.n_dn, wl.n_orb = 9, 7, 9
    wl.coefs = qi.solid_table(9, 14, seed=3, dtype=np.float64)
    _compare(gpu, orc, _drift(wl, 0.15), 48, 32, 25, 0.5)


def test_dmc_node_crossings_and_full_population(gpu, orc):
    """Large steps (many proposals cross a node) and a first trial energy far above the
    estimate: the weights grow, the population reaches the capacity and copies are dropped."""
    st = _compare(gpu, orc, _drift(qi.heg14(), 0.35), 32, 24, 20, 0.0, e_trial=30.0)
    assert st[:, 5].sum() > 0 and st[:, 4].sum() > 0


def test_dmc_solid128(gpu, orc):
    """The 128-electron solid: 512 slots, 256 walkers, 2 steps."""
    _compare(gpu, orc, _drift(qi.solid128(), 0.03), 512, 256, 2, 1.0)


def test_dmc_mixed_precision(gpu, orc):
    """FP32 table and rows; the drift velocities are FP64 (FP64 gradient rows and inverses), so
    the positions follow the oracle's to the FP64 bar and only the energies carry FP32
    rounding."""
    wl = qi.solid(48, 16, n_walkers=1, n_sweeps=1, precision="mixed", table_dtype=np.float32)
    _compare(gpu, orc, _drift(wl, 0.08), 48, 32, 12, 0.5, rel=1e-5)


def test_dmc_mixed_precision_long_run(gpu, orc):
    """96 slots, 64 walkers at the start, 40 steps."""
    wl = qi.solid(48, 16, n_walkers=1, n_sweeps=1, precision="mixed", table_dtype=np.float32, seed=6)
    _compare(gpu, orc, _drift(wl, 0.08), 96, 64, 40, 0.5, rel=1e-5)


def test_dmc_with_three_body_jastrow(gpu, orc):
    """The three-body term enters the drift velocities, the Jastrow change and the local
    energies that weight the walkers."""
    wl = qi.solid(24, 12, n_walkers=1, n_sweeps=1, j3=True, j3_strength=50.0)
    _compare(gpu, orc, _drift(wl, 0.12), 32, 24, 12, 0.5)


def _pdrift(wl, sigma):
    return dataclasses.replace(wl, all_electron=False, drift=True, sigma=sigma)


def test_dmc_pbyp_drift_heg14(gpu, orc):
    """DMC on particle-by-particle drift-diffusion sweeps (one sweep per step, a move with
    R < 0 rejected), with copies, deaths and node-crossing rejections."""
    st = _compare(gpu, orc, _pdrift(qi.heg14(), 0.4), 40, 24, 30, 0.5)
    assert st[:, 5].sum() > 0 and st[:, 2].min() != st[:, 2].max()


def test_dmc_pbyp_drift_per_slot_ragged_solid(gpu, orc):
    wl = qi.solid(18, 14, n_walkers=1, n_sweeps=1)
    wl.n_up, wl.n_dn, wl.n_orb = 9, 7, 9
    wl.coefs = qi.solid_table(9, 14, seed=3, dtype=np.float64)
    assert _per_slot(gpu, orc, _pdrift(wl, 0.05), 32, 24, 12, 0.5) > 0


def test_dmc_pbyp_drift_solid128(gpu, orc):
    """The 128-electron solid: 64 slots, 48 walkers, 6 steps."""
    _compare(gpu, orc, _pdrift(qi.solid128(), 0.03), 64, 48, 6, 1.0)


def test_dmc_in_a_caller_arena(gpu):
    """The population buffers fit an arena sized by qmc_estimate_device_bytes, and the run is
    bit for bit the one with the library's own allocations."""
    import torch
    wl = _drift(qi.heg14(), 0.2)
    out = []
    for arena in (False, True):
        s = gpu.System(wl, n_walkers=32, use_torch_arena=arena)
        s.dmc_init(24, feedback=0.5)
        st = torch.zeros((10, 6), dtype=torch.float64, device="cuda")
        s.dmc_steps(10, st)
        out.append((st.cpu().numpy(), s.get_walkers()[0], s.dmc_state()[0]))
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_dmc_needs_drift_moves_and_init(gpu):
    s = gpu.System(dataclasses.replace(qi.heg14(), all_electron=True, sigma=0.1))
    with pytest.raises(gpu.QMCError):
        s.dmc_init(4)
    s.close()
    import torch
    s = gpu.System(_drift(qi.heg14(), 0.1))
    with pytest.raises(gpu.QMCError):
        s.dmc_steps(1, torch.zeros((1, 6), dtype=torch.float64, device="cuda"))
    with pytest.raises(gpu.QMCError):
        s.dmc_init(s.W + 1)
    s.close()
