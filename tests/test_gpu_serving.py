"""The request server on the GPU: every request completes, the HBM budget
holds, and a request served inside mixed concurrent batches is bit-identical
to the same request served alone (and, in FP64, to the oracle run on the
same device-drawn PDF sample)."""
import numpy as np
import pytest

import oracle
from paper_1909_06374_amd.serving import GpuBackend, Request, Server, make_requests

from test_gpu_parity import agn

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _alone(ctx, r, prec):
    be = GpuBackend(ctx, n_slots=1, prec=prec, keep_outputs=True)
    solo = Request(rid=r.rid, n=r.n, iters=r.iters, f_br=r.f_br, a_low=r.a_low, a_high=r.a_high,
                   seed=r.seed, arrival=0.0)
    Server(be, budget_bytes=2**36).run([solo])
    return be.outputs[r.rid]


@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_equals_alone(gpu_ctx, prec):
    reqs = make_requests(rate_hz=400.0, duration_s=0.1, seed=8, k_lo=10, k_hi=16, iters_lo=4, iters_hi=12)
    assert len(reqs) >= 20
    # the first half is queued at time zero, so that the first launch takes
    # several of them together whatever the speed of the device; the rest
    # arrive while batches are in flight
    for r in reqs[:len(reqs) // 2]:
        r.arrival = 0.0
    be = GpuBackend(gpu_ctx, n_slots=3, prec=prec, keep_outputs=True)
    srv = Server(be, budget_bytes=2**33, max_batch_samples=2**17)
    st = srv.run(reqs)
    assert st.completed == len(reqs) and st.max_footprint <= srv.budget
    assert st.batches < len(reqs), "requests should share batches"
    assert all(r.done >= r.arrival for r in reqs)
    for r in reqs[::4]:
        x = be.outputs[r.rid]
        assert np.array_equal(x, _alone(gpu_ctx, r, prec)), r.rid
    if prec == 0:
        m = agn()
        for r in reqs[:3]:
            d = torch.empty(r.n, dtype=torch.float64, device="cuda:0")
            m.agn_erdf_draw(gpu_ctx, m.erdf_params(), r.n, r.seed, r.rid, d)
            erdf = d.cpu().numpy()
            xo, _, _, _ = oracle.generate(oracle.psd_params(0.0, r.f_br, r.a_low, r.a_high), erdf, 1.0,
                                          r.iters, r.seed, r.rid)
            assert np.array_equal(be.outputs[r.rid], xo)


def test_budget_serialises_large_requests(gpu_ctx):
    be = GpuBackend(gpu_ctx, n_slots=4, prec=1)
    reqs = [Request(rid=i, n=2**18, iters=3, f_br=0.01, a_low=1.0, a_high=2.0, seed=i, arrival=0.0)
            for i in range(6)]
    budget = 2 * be.footprint(reqs[0]) + 1
    st = Server(be, budget_bytes=budget).run(reqs)
    assert st.completed == 6 and st.max_footprint <= budget


@pytest.mark.parametrize("prec", [0, 1])
def test_segmented_serving_equals_alone(gpu_ctx, prec):
    """Iteration-level serving: each launch runs at most 5 iterations of a
    request, which then goes back to the queue; outputs and Eq. 4 histories
    equal those of the same request served alone in one launch, bit for bit
    (the series is the iteration's only state), and in FP64 the oracle's."""
    reqs = make_requests(rate_hz=400.0, duration_s=0.08, seed=18, k_lo=10, k_hi=17, iters_lo=4, iters_hi=16)
    assert len(reqs) >= 15
    for r in reqs[:len(reqs) // 2]:
        r.arrival = 0.0
    be = GpuBackend(gpu_ctx, n_slots=3, prec=prec, keep_outputs=True)
    srv = Server(be, budget_bytes=2**33, max_batch_samples=2**17, segment_iters=5)
    st = srv.run(reqs)
    assert st.completed == len(reqs) and st.max_footprint <= srv.budget
    assert any(r.segments > 1 for r in reqs)
    assert not be.state, "every request's series is freed when it completes"
    for r in reqs[::3]:
        solo_be = GpuBackend(gpu_ctx, n_slots=1, prec=prec, keep_outputs=True)
        solo = Request(rid=r.rid, n=r.n, iters=r.iters, f_br=r.f_br, a_low=r.a_low, a_high=r.a_high,
                       seed=r.seed, arrival=0.0)
        Server(solo_be, budget_bytes=2**36).run([solo])
        assert np.array_equal(be.outputs[r.rid], solo_be.outputs[r.rid]), r.rid
        assert np.array_equal(be.histories[r.rid], solo_be.histories[r.rid]), r.rid
    if prec == 0:
        m = agn()
        for r in reqs[:2]:
            d = torch.empty(r.n, dtype=torch.float64, device="cuda:0")
            m.agn_erdf_draw(gpu_ctx, m.erdf_params(), r.n, r.seed, r.rid, d)
            xo, _, _, _ = oracle.generate(oracle.psd_params(0.0, r.f_br, r.a_low, r.a_high), d.cpu().numpy(), 1.0,
                                          r.iters, r.seed, r.rid)
            assert np.array_equal(be.outputs[r.rid], xo)
