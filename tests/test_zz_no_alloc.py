"""The entry point for callers that cannot allocate device memory: qmc_eval_spo_vgl_noalloc
against qmc_eval_spo_vgl, through the C ABI."""
import numpy as np
import pytest

import qmc_inputs as qi

pytestmark = pytest.mark.gpu


def test_noalloc_eval_matches_the_allocating_call():
    """Two calls in a row (the second smaller, so the shared staging array still holds the first
    call's results past its end) give bit for bit the results of qmc_eval_spo_vgl, in FP64 and in
    mixed precision; a call whose staging would not fit the fixed array is refused with ARG."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_06922_amd import qmc
    qmc.load_library()
    rng = np.random.default_rng(7)
    for wl in (qi.solid(40, 12, n_walkers=1, n_sweeps=1),
               qi.solid(38, 10, n_walkers=1, n_sweeps=1, precision="mixed", table_dtype=np.float32)):
        print(f"[noalloc] {wl.name}", flush=True)
        s = qmc.System(wl, n_walkers=1)
        for n in (301, 17):
            pts = rng.uniform(-wl.L, 2 * wl.L, size=(n, 3))
            assert np.array_equal(s.eval_spo_vgl_noalloc(pts), s.eval_spo_vgl(pts))
        too_many = qmc.NOALLOC_DOUBLES // (3 + 5 * wl.n_orb) + 1
        with pytest.raises(qmc.QMCError) as ei:
            s.eval_spo_vgl_noalloc(np.zeros((too_many, 3)))
        assert ei.value.status == qmc.QMC_ERR_ARG
        s.close()
