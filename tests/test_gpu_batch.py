"""GPU: batched systems (fused launches, graph replay) and the delay-rank autotuner."""
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


def _systems():
    """Uneven mixed-precision systems (the last one too large to keep its inverse in LDS)."""
    spec = [(16, 10, 8, 8), (40, 14, 12, 16), (72, 16, 6, 32), (400, 24, 2, 32)]
    out = []
    for i, (n, g, w, K) in enumerate(spec):
        out.append(qi.solid(n, g, n_walkers=w, n_sweeps=1, precision="mixed", table_dtype=np.float32,
                            delay_rank=K, recompute_period=3, seed=i, name=f"batch{n}"))
    return out


def _alone(gpu, wl, sweeps):
    s = gpu.System(wl)
    bits, e = [], []
    for _ in range(sweeps):
        s.sweep(1)
        bits.append(s.accept_log())
        e.append(s.measure())
    s.close()
    return np.stack(bits), np.stack(e)


def test_batch_equals_each_system_alone(gpu):
    sweeps = 5
    wls = _systems()
    ref = [_alone(gpu, wl, sweeps) for wl in wls]
    systems = [gpu.System(wl) for wl in wls]
    batch = gpu.Batch(systems)
    for it in range(sweeps):
        batch.sweep(1, measure=True)
        for k, s in enumerate(systems):
            print(f"[batch] sweep {it} system {k}", flush=True)
            assert np.array_equal(s.accept_log(), ref[k][0][it])
            assert np.array_equal(s.last_energies(), ref[k][1][it])
    batch.close()
    for s in systems:
        s.close()


def test_batch_graph_replay_equals_eager(gpu):
    sweeps = 6
    wls = _systems()[:3]
    outs = []
    for graph in (False, True):
        systems = [gpu.System(wl) for wl in wls]
        batch = gpu.Batch(systems, graph=graph)
        res = []
        for it in range(sweeps):
            batch.sweep(1, measure=True)
            res.append([(s.accept_log(), s.last_energies()) for s in systems])
        batch.close()
        for s in systems:
            s.close()
        outs.append(res)
    for it in range(sweeps):
        for k in range(len(wls)):
            assert np.array_equal(outs[0][it][k][0], outs[1][it][k][0])
            assert np.array_equal(outs[0][it][k][1], outs[1][it][k][1])


def test_autotune_keeps_the_chain_exact(gpu, orc):
    wl = qi.solid(48, 16, n_walkers=8, n_sweeps=1, delay_rank=8)
    s = gpu.System(wl)
    best, ms = s.autotune_delay(ranks=(4, 8, 16, 64), trial_sweeps=2)
    assert best in (4, 8, 16, 64) and ms > 0
    s.sweep(1)
    pos, ld, _ = s.get_walkers()
    bits = s.accept_log()
    s.close()
    ref = orc.OracleSystem(wl).run(range(8), 9, measure_every=0)
    assert np.array_equal(bits, ref["accept"][:, -1])
    np.testing.assert_allclose(pos, ref["final_pos"], rtol=0, atol=1e-11)
    np.testing.assert_allclose(ld, ref["logdet"], rtol=0, atol=1e-9)


def test_gather_autotune_keeps_rows_bitwise(gpu):
    """Every gather width gives the same orbital rows: a tuned run and an untuned run of the
    same number of sweeps coincide bit for bit."""
    wl = qi.solid(40, 14, n_walkers=16, n_sweeps=1, precision="mixed", table_dtype=np.float32,
                  delay_rank=8, recompute_period=0)
    s = gpu.System(wl)
    tl, ms = s.autotune_gather(trial_sweeps=2)
    assert 0 <= tl <= 6 and ms > 0
    s.sweep(2)
    _, n_sweeps = s.counters()
    tuned = (s.get_walkers()[0], s.measure())
    s.close()
    s = gpu.System(wl)
    s.sweep(int(n_sweeps))
    ref = (s.get_walkers()[0], s.measure())
    s.close()
    assert np.array_equal(tuned[0], ref[0]) and np.array_equal(tuned[1], ref[1])


def test_batch_with_a_three_body_member_equals_alone(gpu):
    """The three-body term travels in each member's parameter block, so a batch with a
    member that has it and one that has not advances each as alone, bit for bit."""
    sweeps = 4
    j3 = qi.solid(32, 12, n_walkers=24, n_sweeps=1, precision="mixed", delay_rank=8, recompute_period=3,
                  seed=5, j3=True, j3_strength=50.0)
    plain = _systems()[0]
    wls = [j3, plain]
    ref = [_alone(gpu, wl, sweeps) for wl in wls]
    systems = [gpu.System(wl) for wl in wls]
    batch = gpu.Batch(systems)
    for it in range(sweeps):
        batch.sweep(1, measure=True)
        for k, s in enumerate(systems):
            assert np.array_equal(s.accept_log(), ref[k][0][it])
            assert np.array_equal(s.last_energies(), ref[k][1][it])
    batch.close()
    for s in systems:
        s.close()


def test_batched_members_match_the_oracle(gpu, orc):
    """The four uneven FP32 systems of the batched workload (32, 96, 192 and 512 electrons on
    24^3 to 64^3 tables, rank-16 delay, 256 walkers each) advanced together by replayed graphs
    for 20 sweeps: two sampled walkers of every member take every decision of the FP64 oracle,
    their energies of every sweep within 1e-5 relative."""
    sweeps = 20
    wls = qi.batched_systems(256)
    samples = [np.array([3 * k, 255 - 5 * k]) for k in range(len(wls))]
    systems = [gpu.System(wl) for wl in wls]
    batch = gpu.Batch(systems, graph=True)
    bits = [[] for _ in wls]
    energies = [[] for _ in wls]
    for it in range(sweeps):
        batch.sweep(1, measure=True)
        for k, s in enumerate(systems):
            bits[k].append(s.accept_log()[samples[k]])
            energies[k].append(s.last_energies()[samples[k]])
    batch.close()
    for s in systems:
        s.close()
    for k, wl in enumerate(wls):
        print(f"[batch-oracle] {wl.name}: walkers {list(samples[k])}, {sweeps} sweeps", flush=True)
        b, e = np.stack(bits[k], 1), np.stack(energies[k], 1)
        ref = orc.OracleSystem(wl).run(samples[k], sweeps, measure_every=1)
        assert np.array_equal(b, ref["accept"]), f"decisions differ at {np.argwhere(b != ref['accept'])[:3]}"
        rel = np.abs(e.sum(-1) - ref["energies"].sum(-1)) / np.maximum(np.abs(ref["energies"].sum(-1)), 1.0)
        assert rel.max() < 1e-5, rel.max()
