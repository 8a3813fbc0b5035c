"""Pins of the oracle's lag statistics: the structure function of Eq. A6
(in L/L_Edd and, per Sec. 3.2.10, in magnitudes) and the counts of pairs
with |dm| above a threshold (Fig. 16), with a detection cut (Fig. 17).

Checks against closed forms (ramps, alternating and geometric series), the
autocorrelation identity sum (x_i - x_{i+k})^2 = S_head + S_tail - 2 ac(k)
with ac from numpy's FFT of the zero-padded series, and the literal |dm|
from log10 on data that keep every pair away from a threshold.
"""
import math

import numpy as np
import pytest

import oracle


def test_sf_closed_forms():
    n = 1000
    ramp = 1.0 + np.arange(n, dtype=np.float64)
    lags = [1, 2, 7, 500, 999]
    sf2, _, _ = oracle.lag_stats(ramp, lags)
    assert np.array_equal(sf2, np.array(lags, dtype=np.float64) ** 2)
    alt = np.where(np.arange(n) % 2 == 0, 3.0, 1.0)
    sf2, _, _ = oracle.lag_stats(alt, [1, 2, 3, 4, 999])
    assert np.array_equal(sf2, [4.0, 0.0, 4.0, 0.0, 4.0])
    # magnitudes of a geometric series form a ramp: m_i = -2.5 log10 x_i = c i
    c = 0.013
    geo = 10.0 ** (-0.4 * c * np.arange(n))
    sf2m, _, _ = oracle.lag_stats(geo, lags, units=1)
    assert np.allclose(sf2m, (c * np.array(lags, dtype=np.float64)) ** 2, rtol=1e-11, atol=0)


def test_sf_autocorrelation_identity():
    """sum over pairs of (x_i - x_{i+k})^2 = sum_{i<n-k} x_i^2 + sum_{i>=k} x_i^2 - 2 ac(k),
    ac(k) = sum_i x_i x_{i+k} from numpy's FFT of x zero-padded to 2n."""
    rng = np.random.default_rng(4)
    n = 3 * 2 ** 9
    x = np.exp(np.cumsum(rng.normal(0, 0.05, n)))          # positive red-noise-like series
    X = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(np.abs(X) ** 2, 2 * n)[:n]
    s = np.concatenate([[0.0], np.cumsum(x * x)])
    lags = np.array([1, 2, 3, 10, 100, 777, n - 1])
    sf2, _, _ = oracle.lag_stats(x, lags)
    for l, k in enumerate(lags):
        expect = (s[n - k] + (s[n] - s[k]) - 2 * ac[k]) / (n - k)
        assert sf2[l] == pytest.approx(expect, rel=1e-9)
    # magnitudes: the same identity on m = -2.5 log10 x
    m = -2.5 * np.log10(x)
    M = np.fft.rfft(m, 2 * n)
    acm = np.fft.irfft(np.abs(M) ** 2, 2 * n)[:n]
    sm = np.concatenate([[0.0], np.cumsum(m * m)])
    sf2m, _, _ = oracle.lag_stats(x, lags, units=1)
    for l, k in enumerate(lags):
        expect = (sm[n - k] + (sm[n] - sm[k]) - 2 * acm[k]) / (n - k)
        assert sf2m[l] == pytest.approx(expect, rel=1e-8, abs=1e-12 * sm[n] / n)


def test_exceedance_counts_geometric_series():
    """x_i = 10^(s i): every pair at lag k has |dm| = 2.5 s k exactly, so each
    threshold is exceeded by all n - k pairs or by none.  With a cut at
    x_c = 10^(s i_c), pairs (i, i + k) with i + k < i_c are dropped and the
    others have |dm| = 2.5 s (i + k - max(i, i_c))."""
    n, s = 400, 0.01
    x = 10.0 ** (s * np.arange(n))
    lags = np.array([1, 5, 40, 120])
    dm = np.array([0.0, 0.11, 0.34, 1.11, 2.96])     # off the grid 0.025 m of |dm| values
    _, ex, pairs = oracle.lag_stats(x, lags, dm_ref=dm)
    for l, k in enumerate(lags):
        assert pairs[l] == n - k
        for j, d in enumerate(dm):
            assert ex[l, j] == (n - k if 2.5 * s * k > d else 0)
    ic = 100
    _, ex, pairs = oracle.lag_stats(x, lags, dm_ref=dm, lam_cut=10.0 ** (s * ic))
    for l, k in enumerate(lags):
        i = np.arange(n - k)
        det = i + k >= ic
        assert pairs[l] == det.sum()
        dmp = 2.5 * s * (i + k - np.maximum(i, ic))
        for j, d in enumerate(dm):
            # stay clear of exact ties: thresholds sit between the discrete values
            assert ex[l, j] == np.sum(det & (dmp > d + 1e-9))


def test_exceedance_matches_literal_log_definition():
    """On a random positive series, |dm| = 2.5 |log10(x_j / x_i)| > D counted
    literally equals the oracle's ratio test wherever no pair lies within
    1e-9 mag of a threshold (checked)."""
    rng = np.random.default_rng(8)
    n = 3000
    x = 10.0 ** rng.uniform(-3.75, 0.5, n)
    lags = np.array([1, 3, 64, 1000])
    dm = np.array([0.5, 1.0, 2.5, 5.0, 10.0])
    cut = 10.0 ** -1.2
    _, ex, pairs = oracle.lag_stats(x, lags, dm_ref=dm, lam_cut=cut)
    _, ex0, pairs0 = oracle.lag_stats(x, lags, dm_ref=dm)
    for l, k in enumerate(lags):
        a, b = x[:-k], x[k:]
        d0 = 2.5 * np.abs(np.log10(b / a))
        assert pairs0[l] == n - k
        det = np.maximum(a, b) >= cut
        ac, bc = np.maximum(a, cut), np.maximum(b, cut)
        d1 = 2.5 * np.abs(np.log10(bc / ac))
        assert pairs[l] == det.sum()
        for j, D in enumerate(dm):
            assert np.min(np.abs(d0 - D)) > 1e-9
            assert ex0[l, j] == np.sum(d0 > D)
            near = det & (np.abs(d1 - D) <= 1e-9)
            assert not np.any(near & (d1 != 0))
            assert ex[l, j] == np.sum(det & (d1 > D))


def test_lag_stats_rejects_bad_input():
    x = np.ones(16)
    for kw in [dict(lags=[0]), dict(lags=[16]), dict(lags=[1], units=2), dict(lags=[1], dm_ref=[-1.0])]:
        with pytest.raises(oracle.OracleError):
            oracle.lag_stats(x, **kw)
    with pytest.raises(oracle.OracleError):
        oracle.lag_stats(np.array([1.0, 0.0, 2.0, 3.0]), [1])
