"""Failure handling of the multi-pass sort's decoupled look-back, forced from
the host: with every look-back wait told to give up at once
(agn_ctx_set_lookback_polls(ctx, -1)) the call must finish without a fault
and report the curve as not valid (iters_done = -2); with the default limit
restored, the same call must again give the exact result (FP64: the oracle's
permutation)."""
import numpy as np
import pytest

import oracle
from paper_1909_06374_amd import synth

from test_gpu_parity import PSD, agn, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _generate(ctx, n, prec, iters, erdf, amp_seed=31):
    m = agn()
    p = m.psd_params(**PSD)
    x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    d = torch.full((iters,), -1.0, dtype=torch.float64, device="cuda:0")
    done = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
    ws = torch.empty(m.agn_workspace_size(n, prec), dtype=torch.uint8, device="cuda:0")
    m.agn_lc_generate(ctx, p, dev(erdf), n, 1.0, iters, -1.0, amp_seed, 0, prec, x, d, done, ws)
    return host(x), host(d), int(host(done)[0])


# multi-pass lengths: FP64 above 8192, FP32 above 16384
@pytest.mark.parametrize("n,prec", [(2**14, 0), (2**15, 1), (3 * 2**14, 0)], ids=["fp64-2p14", "fp32-2p15", "fp64-3x2p14"])
def test_forced_lookback_give_up_is_reported(gpu_ctx, n, prec):
    erdf = synth.erdf_draw(n, seed=61)
    iters = 3
    ref_x, ref_d, ref_done = _generate(gpu_ctx, n, prec, iters, erdf)
    assert ref_done == iters
    try:
        gpu_ctx.set_lookback_polls(-1)
        _, _, done = _generate(gpu_ctx, n, prec, iters, erdf)
        assert done == -2
    finally:
        gpu_ctx.set_lookback_polls(0)
    x, dl, done = _generate(gpu_ctx, n, prec, iters, erdf)
    assert done == iters
    assert np.array_equal(x, ref_x) and np.array_equal(dl, ref_d)
    if prec == 0:
        p = oracle.psd_params(**PSD)
        xo, _, _, _ = oracle.generate(p, erdf, 1.0, iters, 31, 0)
        assert np.array_equal(x, xo)
