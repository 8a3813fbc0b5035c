"""The allocation-free spectrum entry point (agn_psd_spectrum_noalloc) against
agn_psd_spectrum, through the C ABI: the same kernels on the library's own
device array instead of a caller's workspace, so the moduli must be
bit-identical.  Two calls in a row, the second on a smaller curve, check that
nothing left in the shared array by the first call leaks into the second."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_spectrum_equals_workspace_entry(gpu_ctx, prec):
    import paper_1909_06374_amd as m
    el = torch.float64 if prec == m.AGN_FP64 else torch.float32
    p = m.psd_params(0.0, 1.0 / 3652.5, 1.0, 2.0)
    for n, seed, dt in [(2**22, 11, 7.0), (3 * 2**9, 12, 1.0)]:
        h = n // 2 + 1
        ws = torch.empty(m.agn_spectrum_workspace_size(n), dtype=torch.uint8, device="cuda:0")
        ref = torch.full((h,), float("nan"), dtype=el, device="cuda:0")
        m.agn_psd_spectrum(gpu_ctx, p, n, dt, seed, 3, prec, ref, ws)
        got = torch.full((h,), float("nan"), dtype=el, device="cuda:0")
        m.agn_psd_spectrum_noalloc(gpu_ctx, p, n, dt, seed, 3, prec, got)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(a)) and a[0] == 0.0
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (n, prec)


def test_noalloc_spectrum_rejects_bad_arguments(gpu_ctx):
    import paper_1909_06374_amd as m
    p = m.psd_params(0.0, 0.01, 1.0, 2.0)
    out = torch.empty(8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(m.AgnError) as e:
        m.agn_psd_spectrum_noalloc(gpu_ctx, p, 10, 1.0, 0, 0, m.AGN_FP64, out)
    assert e.value.code == m.AGN_EUNSUPPORTED_N
    with pytest.raises(m.AgnError):
        m.agn_psd_spectrum_noalloc(gpu_ctx, m.psd_params(0.0, -1.0, 1.0, 2.0), 8, 1.0, 0, 0, m.AGN_FP64, out)
