"""GPU: the serving loop (continuous batching under a memory budget) gives each request the
results it gets alone."""
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


def test_served_requests_match_alone(gpu):
    from paper_1802_06922_amd import serve
    spec = [(24, 12, 6, 4), (48, 14, 10, 7), (16, 10, 4, 3), (96, 16, 8, 5)]   # (N, grid, W, sweeps)
    reqs = []
    for i, (n, g, w, sw) in enumerate(spec):
        wl = qi.solid(n, g, n_walkers=w, n_sweeps=1, precision="mixed", table_dtype=np.float32,
                      recompute_period=2, seed=10 + i, name=f"req{i}")
        wl.delay_rank = serve.delay_rank_for(wl, cap=16)
        r = serve.Request(rid=i, arrival_s=0.0, wl=wl, n_sweeps=sw)
        r.est_bytes = gpu.estimate_device_bytes(wl, w)
        reqs.append(r)
    # a budget holding about two requests at once: later ones join mid-run as others finish
    budget = int(sorted(r.est_bytes for r in reqs)[-1] + sorted(r.est_bytes for r in reqs)[-2] + 1)
    srv = serve.Server(hbm_budget_bytes=budget, reserve_bytes=0)
    st = srv.run(reqs, time_scale=0.0, log=lambda m: print(m, flush=True))
    assert st["requests"] == len(spec)
    assert st["sweep_iterations"] < sum(s[3] for s in spec)   # requests shared sweeps
    for r in st["finished"]:
        print(f"[serve] compare request {r.rid}", flush=True)
        s = gpu.System(r.wl)
        for _ in range(r.n_sweeps):
            s.sweep(1)
            e = s.measure()
        pos = s.get_walkers()[0]
        s.close()
        assert np.array_equal(e, r.energy)
        assert np.array_equal(pos, r.final_pos)
        assert len(r.latencies_ms) == r.n_sweeps and min(r.latencies_ms) > 0


def test_served_dmc_requests_match_alone(gpu):
    """DMC requests served beside VMC requests (their steps on their own streams, overlapping the
    fused VMC sweeps): each request's results are the ones it gets alone, bit for bit."""
    import dataclasses

    import torch
    from paper_1802_06922_amd import serve
    spec = [(24, 12, 6, 4, "vmc"), (16, 12, 16, 6, "dmc"), (48, 14, 10, 5, "vmc"), (32, 12, 24, 5, "dmc")]
    reqs = []
    for i, (n, g, w, sw, kind) in enumerate(spec):
        wl = qi.solid(n, g, n_walkers=w, n_sweeps=1, precision="mixed", table_dtype=np.float32,
                      recompute_period=2, seed=20 + i, name=f"req{i}")
        wl.delay_rank = serve.delay_rank_for(wl, cap=16)
        if kind == "dmc":
            wl = dataclasses.replace(wl, all_electron=True, drift=True, sigma=0.3 / np.sqrt(n))
        r = serve.Request(rid=i, arrival_s=0.0, wl=wl, n_sweeps=sw, kind=kind,
                          dmc_target=w * 3 // 4 if kind == "dmc" else 0, dmc_feedback=0.5)
        r.est_bytes = gpu.estimate_device_bytes(wl, w)
        reqs.append(r)
    srv = serve.Server(reserve_bytes=0)
    st = srv.run(reqs, time_scale=0.0, log=lambda m: print(m, flush=True))
    assert st["requests"] == len(spec) and st["dmc_requests"] == 2
    for r in st["finished"]:
        print(f"[serve] compare request {r.rid} ({r.kind})", flush=True)
        s = gpu.System(r.wl)
        if r.kind == "dmc":
            s.dmc_init(r.dmc_target, feedback=r.dmc_feedback)
            out = torch.zeros((r.n_sweeps, 6), dtype=torch.float64, device="cuda")
            s.dmc_steps(r.n_sweeps, out)
            e = out.cpu().numpy()
        else:
            for _ in range(r.n_sweeps):
                s.sweep(1)
                e = s.measure()
        pos = s.get_walkers()[0]
        s.close()
        assert np.array_equal(e, r.energy)
        assert np.array_equal(pos, r.final_pos)


def test_served_requests_match_the_oracle(gpu, orc):
    """One VMC and one DMC request (mixed precision) served together: the VMC request's last
    energies within 1e-5 of the FP64 oracle and its positions to rounding (every decision
    taken as the oracle takes it); the DMC request's per-step population, dropped copies and
    node-crossing rejections exactly, its estimates within 1e-5, and its alive walkers where
    the oracle's are."""
    import dataclasses
    from paper_1802_06922_amd import serve
    spec = [(24, 12, 6, 4, "vmc"), (16, 12, 16, 6, "dmc")]
    reqs = []
    for i, (n, g, w, sw, kind) in enumerate(spec):
        wl = qi.solid(n, g, n_walkers=w, n_sweeps=1, precision="mixed", table_dtype=np.float32,
                      recompute_period=2, seed=30 + i, name=f"req{i}")
        wl.delay_rank = serve.delay_rank_for(wl, cap=16)
        if kind == "dmc":
            wl = dataclasses.replace(wl, all_electron=True, drift=True, sigma=0.3 / np.sqrt(n))
        r = serve.Request(rid=i, arrival_s=0.0, wl=wl, n_sweeps=sw, kind=kind,
                          dmc_target=w * 3 // 4 if kind == "dmc" else 0, dmc_feedback=0.5)
        r.est_bytes = gpu.estimate_device_bytes(wl, w)
        reqs.append(r)
    st = serve.Server(reserve_bytes=0).run(reqs, time_scale=0.0, log=lambda m: print(m, flush=True))
    assert st["requests"] == 2 and st["dmc_requests"] == 1
    for r in st["finished"]:
        print(f"[serve-oracle] request {r.rid} ({r.kind})", flush=True)
        o = orc.OracleSystem(r.wl)
        if r.kind == "vmc":
            ref = o.run(range(r.wl.n_walkers), r.n_sweeps, measure_every=1)
            e, re = r.energy.sum(-1), ref["energies"][:, -1].sum(-1)
            assert (np.abs(e - re) / np.maximum(np.abs(re), 1.0)).max() < 1e-5
            np.testing.assert_allclose(r.final_pos, ref["final_pos"], rtol=0, atol=1e-10)
        else:
            ref = o.dmc(r.wl.n_walkers, r.dmc_target, r.n_sweeps, feedback=r.dmc_feedback)
            for c in (2, 4, 5):
                assert np.array_equal(r.energy[:, c], ref["stats"][:, c]), c
            for c in (0, 1, 3):
                err = np.abs(r.energy[:, c] - ref["stats"][:, c]) / np.maximum(np.abs(ref["stats"][:, c]), 1.0)
                assert err.max() < 1e-5, (c, err.max())
            alive = ref["final_sign"] != 0
            np.testing.assert_allclose(r.final_pos[alive], ref["final_pos"][alive], rtol=0, atol=1e-7)
