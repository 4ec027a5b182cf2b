"""GPU: the sweep's proposals evaluated in table order give the same bits as (walker, electron) order.

The ordered gather draws every proposal, buckets it by the table tile that holds it, sorts the
items by bucket and evaluates them in that order (each XCD a contiguous slice).  Each item's
arithmetic is unchanged, so every accept decision, position, log-determinant and local energy
must be bitwise equal to the run with QMC_GATHER_ORDER=0 (the items in (walker, electron)
order), over several sweeps, for both precisions, all-electron moves and item counts that are
not a multiple of the workgroup's items.
"""
import dataclasses
import os

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


def _run(gpu, wl, sweeps, ordered):
    old = os.environ.get("QMC_GATHER_ORDER")
    os.environ["QMC_GATHER_ORDER"] = "1" if ordered else "0"
    try:
        s = gpu.System(wl)
    finally:
        if old is None:
            del os.environ["QMC_GATHER_ORDER"]
        else:
            os.environ["QMC_GATHER_ORDER"] = old
    out = []
    for _ in range(sweeps):
        s.sweep(1)
        e = s.measure()
        pos, ld, sg = s.get_walkers()
        out.append((s.accept_log(), pos, ld, sg, e))
    s.close()
    return out


CASES = [
    # (name, workload factory, sweeps)
    ("solid48_fp64_ragged", lambda: qi.solid(48, 20, n_walkers=7, n_sweeps=1, seed=3, name="ord48"), 4),
    ("solid72_mixed_K16", lambda: qi.solid(72, 24, n_walkers=13, n_sweeps=1, precision="mixed",
                                           delay_rank=16, recompute_period=3, seed=5, name="ord72"), 4),
    ("solid24_all_electron_drift", lambda: dataclasses.replace(
        qi.solid(24, 16, n_walkers=9, n_sweeps=1, seed=2, name="ord24ae"), all_electron=True, sigma=0.05,
        drift=True), 4),
    ("solid384_mixed_K16", lambda: qi.solid(384, 64, n_walkers=64, n_sweeps=1, precision="mixed",
                                            table_dtype=np.float32, delay_rank=16, recompute_period=64,
                                            name="ord384"), 3),
]


@pytest.mark.parametrize("name,make,sweeps", CASES, ids=[c[0] for c in CASES])
def test_table_order_gives_the_same_bits(gpu, name, make, sweeps):
    wl = make()
    a = _run(gpu, wl, sweeps, ordered=True)
    b = _run(gpu, wl, sweeps, ordered=False)
    for it, (x, y) in enumerate(zip(a, b)):
        print(f"[gather-order] {name} sweep {it}: accepted {int(x[0].sum())}", flush=True)
        for k, what in enumerate(("accept log", "positions", "log|D|", "sign", "energies")):
            assert np.array_equal(x[k], y[k]), f"{what} differ at sweep {it}"
