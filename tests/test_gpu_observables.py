"""Periodogram of Eq. A2 and its log-binned means on the GPU against the
oracle (a plain DFT-based periodogram and numpy binning), for curves on both
the LDS and the multi-pass transform paths in one batch.

Tolerance: both sides compute X_j with a fast transform whose error obeys
|dX_j| <= c eps log2(N) sqrt(N) ||x||_2 (Parseval bound on the 2-norm of the
error vector); with c = 2 for the two implementations together,
|dP_j| <= (2 / N^2) (2 |X_j| e + e^2), e = 4 eps log2(N) sqrt(N) ||x||_2."""
import math

import numpy as np
import pytest

import oracle
from paper_1909_06374_amd import synth

from test_gpu_parity import agn, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS = 2.0**-52


def _bound(x, Pref):
    n = len(x)
    e = 4 * EPS * math.log2(n) * math.sqrt(n) * np.sqrt(np.sum(x * x))
    X = np.sqrt(Pref * n * n / 2.0)
    return 2.0 / (n * n) * (2 * X * e + e * e)


def test_periodogram_and_bins_match_oracle(gpu_ctx):
    m = agn()
    ns = [4, 64, 1536, 12288, 2**14, 3 * 2**13, 2**15, 2**16, 1024]
    xs = []
    for i, n in enumerate(ns):
        amp = oracle.psd_spectrum(oracle.psd_params(0.0, 1 / 100.0, 1.0, 2.5), n, 1.0, seed=i)
        x0 = synth.erdf_draw(n, seed=100 + i)
        xs.append(oracle.iterate(amp, x0, 2)[0] if n <= 2**14 else x0)
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    poffs = np.concatenate([[0], np.cumsum([n // 2 + 1 for n in ns])[:-1]]).astype(np.int64)
    dex = 0.1
    nb = [m.agn_log_bin_count(n, dex) for n in ns]
    boffs = np.concatenate([[0], np.cumsum(nb)[:-1]]).astype(np.int64)
    x = dev(np.concatenate(xs))
    P = torch.full((int(sum(n // 2 + 1 for n in ns)),), float("nan"), dtype=torch.float64, device="cuda:0")
    B = torch.full((int(sum(nb)),), float("nan"), dtype=torch.float64, device="cuda:0")
    ws = torch.empty(m.agn_periodogram_workspace_size(ns, dex), dtype=torch.uint8, device="cuda:0")
    m.agn_periodogram_batch(gpu_ctx, ns, offs, x, poffs, P, dex, boffs, B, ws)
    Pg, Bg = host(P), host(B)
    for c, n in enumerate(ns):
        pr = oracle.periodogram(xs[c])
        pg = Pg[poffs[c]:poffs[c] + n // 2 + 1]
        tol = _bound(xs[c], pr)
        assert np.all(np.abs(pg - pr) <= tol), (n, np.max(np.abs(pg - pr) / tol))
        _, br = oracle.log_binned(pr, n, 1.0, dex)
        bg = Bg[boffs[c]:boffs[c] + nb[c]]
        assert len(br) == nb[c]
        assert np.all(np.abs(bg - br) <= tol.max()), n


def test_periodogram_of_generated_curve(gpu_ctx):
    """On the generator's output (2^15, multi-pass transform): Parseval's
    identity P_0 + 2 sum_{0<j<N/2} P_j + P_{N/2} = (2/N) sum_t x_t^2 to
    round-off, and a spectrum steeper above the input break than below it
    (Sec. 3.2.2: the output follows the shape of the target PSD)."""
    m = agn()
    n = 2**15
    p = m.psd_params(0.0, 1 / 300.0, 1.0, 2.5)
    erdf = dev(synth.erdf_draw(n, seed=5))
    ws = torch.empty(m.agn_workspace_size(n, 0), dtype=torch.uint8, device="cuda:0")
    x = torch.empty(n, dtype=torch.float64, device="cuda:0")
    m.agn_lc_generate(gpu_ctx, p, erdf, n, 1.0, 50, -1.0, 3, 0, 0, x, None, None, ws)
    P = torch.empty(n // 2 + 1, dtype=torch.float64, device="cuda:0")
    nb = m.agn_log_bin_count(n, 0.2)
    B = torch.empty(nb, dtype=torch.float64, device="cuda:0")
    pws = torch.empty(m.agn_periodogram_workspace_size([n], 0.2), dtype=torch.uint8, device="cuda:0")
    m.agn_periodogram_batch(gpu_ctx, [n], [0], x, [0], P, 0.2, [0], B, pws)
    Pg, xg, b = host(P), host(x), host(B)
    lhs = Pg[0] + 2 * Pg[1:n // 2].sum() + Pg[n // 2]
    assert abs(lhs - 2.0 / n * np.sum(xg * xg)) <= 1e-12 * lhs
    j = np.arange(1, n // 2 + 1)
    cen = np.array([np.mean(np.log10(j[(np.floor(np.log10(j) / 0.2 + 1e-9)) == k])) for k in range(nb)])
    f = 10**cen / n
    lo = (f > 2 / n) & (f < (1 / 300.0) / 3)
    hi = (f > 3 / 300.0) & (f < 0.05)
    slope_lo = np.polyfit(np.log10(f[lo]), np.log10(b[lo]), 1)[0]
    slope_hi = np.polyfit(np.log10(f[hi]), np.log10(b[hi]), 1)[0]
    assert slope_hi < slope_lo < 0, (slope_lo, slope_hi)


def test_periodogram_argument_errors(gpu_ctx):
    m = agn()
    x = torch.zeros(64, dtype=torch.float64, device="cuda:0")
    P = torch.zeros(33, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(m.agn_periodogram_workspace_size([32], 0.0) + 4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(m.AgnError):
        m.agn_periodogram_batch(gpu_ctx, [32], [1], x, [0], P, 0.0, None, None, ws)
    with pytest.raises(m.AgnError):
        m.agn_periodogram_batch(gpu_ctx, [30], [0], x, [0], P, 0.0, None, None, ws)
    with pytest.raises(m.AgnError):
        m.agn_log_bin_count(64, 0.0)
