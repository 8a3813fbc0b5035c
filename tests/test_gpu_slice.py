"""GPU parity of the slice sampler (Sec. 3.1's draw; Neal 2003) against the
oracle's chains.

Both sides follow the same chain with the same uniforms; the device kernel
does not fuse multiply-adds, so every proposal is the same double on both
sides, and only a density value within a few ulps of its slice level could
be decided differently (about 1e-15 of the decisions).
The bar is therefore bit-identical draws.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "eq1_table2_log": dict(kind=1, measure=0),
    "eq1_table2_linear": dict(kind=1, measure=1),
    "eq2_log": dict(kind=2, measure=0, u_min=-6.0, u_max=1.0, u_star=-3.25),
    "sharp_linear": dict(kind=0, measure=1, u_min=-4.0, u_max=0.0, u_star=-1.5, d1=0.4, d2=2.5),
    "star_outside": dict(kind=1, measure=0, u_min=-3.0, u_max=-2.0, u_star=-1.0),
}


def agn():
    import paper_1909_06374_amd as m
    return m


def gpu_slice(m, ctx, case, n, chains, burn, seed, curve):
    keys = ("kind", "measure", "u_min", "u_max", "u_star", "d1", "d2", "sigma")
    po = oracle.pdf_params(**case)
    pg = m.pdf_params(*[getattr(po, k) for k in keys])
    out = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device="cuda:0")
    m.agn_pdf_slice(ctx, pg, n, chains, burn, seed, curve, out)
    torch.cuda.synchronize()
    return po, out.cpu().numpy()[:n]


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("n,chains,burn", [(1, 1, 0), (100, 1000, 5), (4099, 257, 50)])
def test_slice_matches_oracle(gpu_ctx, name, n, chains, burn):
    m = agn()
    po, got = gpu_slice(m, gpu_ctx, CASES[name], n, chains, burn, 21, 3)
    ref = oracle.pdf_slice(po, n, chains, burn, 21, 3)
    assert np.array_equal(got, ref), np.nonzero(got != ref)[0][:5]


def test_slice_many_chains(gpu_ctx):
    """2^18 draws from 16384 chains (16 steps each after 100 of burn-in)."""
    m = agn()
    po, got = gpu_slice(m, gpu_ctx, CASES["eq1_table2_linear"], 1 << 18, 16384, 100, 8, 0)
    ref = oracle.pdf_slice(po, 1 << 18, 16384, 100, 8, 0)
    assert np.array_equal(got, ref)


def test_slice_errors(gpu_ctx):
    m = agn()
    out = torch.empty(16, dtype=torch.float64, device="cuda:0")
    p = m.pdf_params(m.AGN_PDF_EQ1)
    for args in [(16, 0, 0), (16, 4, -1), (-1, 4, 0)]:
        with pytest.raises(m.AgnError):
            m.agn_pdf_slice(gpu_ctx, p, args[0], args[1], args[2], 0, 0, out)
    with pytest.raises(m.AgnError):
        m.agn_pdf_slice(gpu_ctx, m.pdf_params(2, sigma=0.0), 16, 4, 0, 0, 0, out)
    m.agn_pdf_slice(gpu_ctx, p, 0, 4, 0, 0, 0, out)  # n = 0: nothing to do
