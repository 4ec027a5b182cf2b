"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import dataclasses
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmc.h")


@pytest.fixture(scope="module")
def libqmc():
    from paper_1802_06922_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    return ctypes.CDLL(hipbuild.LIB)


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["qmc_create_system", "qmc_load_spline_table", "qmc_init_walkers", "qmc_sweep",
                     "qmc_measure_local_energy"]:
        assert required in names


def test_library_exports_every_declared_symbol(libqmc):
    missing = [n for n in _declared() if not hasattr(libqmc, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1802_06922_amd import qmc
    assert sorted(qmc.EXPORTS) == _declared()


def test_estimate_device_bytes_without_gpu(libqmc):
    import numpy as np

    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc
    qmc.load_library()
    wl = qi.heg14()
    small = qmc.estimate_device_bytes(wl, 8)
    big = qmc.estimate_device_bytes(wl, 800)
    assert 0 < small < big
    # table + walker buffers dominate: at least the FP64 table and two value buffers
    S = 8
    assert small >= 16 ** 3 * S * 8 + 2 * 8 * 14 * 5 * S * 8
    keep = []
    d = qmc.make_desc(wl, keep)
    d.n_up = 0
    assert libqmc.qmc_estimate_device_bytes(ctypes.byref(d), 8, 16, 16, 16) == 0
    assert np.isfinite(small)


def test_create_rejects_bad_descriptors_before_touching_the_device(libqmc):
    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc
    L = qmc.load_library()
    wl = qi.solid128()
    keep = []
    bad = qmc.make_desc(wl, keep)
    bad.j2_rcut = wl.L  # beyond the Wigner-Seitz radius L/2
    h = ctypes.c_void_p()
    assert L.qmc_create_system(ctypes.byref(bad), None, ctypes.byref(h)) == qmc.QMC_ERR_ARG
    assert b"cutoff" in L.qmc_last_error(None)
    bad = qmc.make_desc(wl, keep)
    bad.sigma = 0.0
    assert L.qmc_create_system(ctypes.byref(bad), None, ctypes.byref(h)) == qmc.QMC_ERR_ARG
    assert L.qmc_create_system(None, None, ctypes.byref(h)) == qmc.QMC_ERR_ARG


def test_max_delay_rank_is_host_only_and_monotone(libqmc):
    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc
    qmc.load_library()
    ranks = []
    for n in (16, 64, 128, 256, 512, 1024):
        wl = qi.solid(n, 8, n_walkers=1, n_sweeps=1, precision="mixed", table_dtype=qi.np.float32)
        k = qmc.max_delay_rank(wl)
        assert k in (1, 4, 8, 16, 32, 64)
        ranks.append(k)
    # the window grows with N: the largest feasible rank never grows with the system
    assert ranks == sorted(ranks, reverse=True)
    assert ranks[0] == 64 and ranks[-1] < 64
    # FP64 windows take twice the LDS of FP32 ones
    wl64 = qi.solid(512, 8, n_walkers=1, n_sweeps=1, precision="fp64")
    assert qmc.max_delay_rank(wl64) <= ranks[4]
    keep = []
    d = qmc.make_desc(qi.heg14(), keep)
    d.n_up = 0
    assert libqmc.qmc_max_delay_rank(ctypes.byref(d)) == 0


def test_estimate_counts_move_kind_buffers(libqmc):
    """All-electron moves add the proposal's inverses and log-determinants; drift moves add the
    velocities, the transition-ratio partials and the DMC population on top."""
    import dataclasses

    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc
    qmc.load_library()
    wl = qi.solid(32, 12, n_walkers=64, n_sweeps=1)
    W, N, n = 64, 32, 16
    pbyp = qmc.estimate_device_bytes(wl, W)
    ae = qmc.estimate_device_bytes(dataclasses.replace(wl, all_electron=True), W)
    drift = qmc.estimate_device_bytes(dataclasses.replace(wl, all_electron=True, drift=True), W)
    assert ae - pbyp >= W * 2 * n * n * 8            # inverses at R'
    assert drift - ae >= 2 * W * N * 3 * 8 + W * 6 * 8   # velocities at R and R', DMC weights and energies


def test_served_request_mix_without_gpu(libqmc):
    """Every k-th served request becomes a DMC run of drift-diffusion all-electron moves whose
    device-memory estimate includes its population buffers; the others stay VMC runs."""
    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc, serve
    qmc.load_library()
    trace = qi.served_trace(n_requests=6, rate_per_s=20.0, seed=0)
    for e in trace:   # keep the host-side table generation small
        e["n_elec"], e["grid"], e["n_walkers"] = 16, 8, 8
    reqs = serve.build_requests(trace, sweep_scale=0.01, dmc_every=3)
    kinds = [r.kind for r in sorted(reqs, key=lambda r: r.rid)]
    assert kinds == ["vmc", "vmc", "dmc", "vmc", "vmc", "dmc"]
    for r in reqs:
        if r.kind == "dmc":
            assert r.wl.all_electron and r.wl.drift and 1 <= r.dmc_target <= r.wl.n_walkers
            vmc_like = qmc.estimate_device_bytes(dataclasses.replace(r.wl, all_electron=False, drift=False),
                                                 r.wl.n_walkers)
            assert r.est_bytes > vmc_like
        else:
            assert not r.wl.all_electron


def test_server_refuses_a_request_that_can_never_fit(libqmc):
    """A request larger than the whole device-memory budget is refused and recorded; the loop
    goes on with the rest (here: nothing else, so no GPU work at all)."""
    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc, serve
    qmc.load_library()
    trace = qi.served_trace(n_requests=3, rate_per_s=1000.0, seed=0)
    for e in trace:
        e["n_elec"], e["grid"], e["n_walkers"] = 16, 8, 8
    reqs = serve.build_requests(trace, sweep_scale=0.01, table_pool=True)
    srv = serve.Server(hbm_budget_bytes=min(r.est_bytes for r in reqs) - 1)
    st = srv.run(reqs)
    assert st["requests"] == 0 and st["rejected"] == 3 and st["failed"] == 0
    assert all(r.status == "rejected" and "budget" in r.error for r in st["refused"])


def test_server_records_a_failed_preparation(libqmc, monkeypatch):
    """A request whose preparation raises finishes as failed and gives its memory back."""
    import qmc_inputs as qi
    from paper_1802_06922_amd import qmc, serve
    qmc.load_library()
    trace = qi.served_trace(n_requests=2, rate_per_s=1000.0, seed=0)
    for e in trace:
        e["n_elec"], e["grid"], e["n_walkers"] = 16, 8, 8
    reqs = serve.build_requests(trace, sweep_scale=0.01)

    def boom(*a, **k):
        raise qmc.QMCError(qmc.QMC_ERR_SINGULAR, "singular start")

    monkeypatch.setattr(qmc, "System", boom)
    srv = serve.Server(hbm_budget_bytes=sum(r.est_bytes for r in reqs))
    st = srv.run(reqs)
    assert st["requests"] == 0 and st["failed"] == 2 and st["rejected"] == 0
    assert all("singular" in r.error for r in st["refused"])


def test_request_tables_are_translated_windows_of_the_bank():
    """A served request's own table: a seeded cyclic window of the bank's orbitals, translated on
    the periodic grid, with seeded signs (checked entry by entry against np.roll)."""
    import numpy as np

    import qmc_inputs as qi
    bank = qi.solid_table(12, 8, seed=8)
    t = qi.request_table(bank, 5, seed=3)
    assert t.shape == (8, 8, 8, 5) and t.dtype == np.float32
    # recover the common shift and the window start from the seeded draw, then compare exactly
    rng = np.random.default_rng([3, 0x7AB1E])
    start = int(rng.integers(0, 12))
    shift = rng.integers(0, 8, size=3)
    sign = np.where(rng.random(5) < 0.5, -1.0, 1.0)
    idx = (start + np.arange(5)) % 12
    want = np.roll(bank[..., idx], shift=tuple(int(x) for x in shift), axis=(0, 1, 2)) * sign.astype(np.float32)
    assert np.array_equal(t, want)
    assert not np.array_equal(t, qi.request_table(bank, 5, seed=4))
