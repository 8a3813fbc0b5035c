"""Pins of the oracle's fit of Eq. 3 to a binned periodogram (the convergence
test that Sec. 3.2.2 describes: fit the periodogram with the input PSD's
functional form and compare the fitted parameters with the input ones).

Checks: exact recovery from noise-free Eq. 3 data, agreement with scipy's
least_squares (an independent optimiser) on noisy data, the shift of log10 A
under a scale factor, skipped empty bins, and the fitted slopes of the
periodograms of Timmer-Koenig series built with numpy's inverse FFT.
"""
import numpy as np
import pytest
from scipy import optimize

import oracle


def eq3_log(f, a, fb, al, ah):
    return a - np.log10((f / fb) ** al + (f / fb) ** ah)


@pytest.mark.parametrize("a,al,ah", [(0.7, 1.3, 2.6), (-3.0, 1.0, 1.0), (2.0, 0.2, 3.5), (0.0, 1.8, 1.2)])
def test_fit_recovers_exact_eq3(a, al, ah):
    f = np.logspace(-4, -0.5, 37)
    fb = 3e-3
    p = oracle.psd_fit(f, 10 ** eq3_log(f, a, fb, al, ah), fb, 1.0, 2.0)
    # with equal slopes the two slope columns of the Jacobian coincide, so the
    # slopes' difference is fixed only at second order: to about sqrt(eps)
    tol = 1e-7 if al == ah else 1e-11
    # Eq. 3 is symmetric in the slopes: the smaller is reported as a_low
    assert np.allclose(p[:3], [a, min(al, ah), max(al, ah)], rtol=0, atol=tol)
    assert p[3] < 1e-12


def test_fit_matches_scipy_least_squares():
    rng = np.random.default_rng(5)
    f = np.logspace(-5, -0.3, 45)
    fb = 1e-3
    for trial in range(5):
        y = eq3_log(f, 0.3, fb, 1.1, 2.4) + rng.normal(0, 0.2, len(f))
        p = oracle.psd_fit(f, 10 ** y, fb, 1.0, 2.0)
        res = optimize.least_squares(lambda t: eq3_log(f, t[0], fb, t[1], t[2]) - y, [0.0, 1.0, 2.0],
                                     xtol=1e-15, ftol=1e-15, gtol=1e-15)
        ref = [res.x[0], min(res.x[1:]), max(res.x[1:])]
        assert np.allclose(p[:3], ref, rtol=0, atol=1e-8), (p, res.x)
        assert p[3] == pytest.approx(np.sqrt(np.mean(res.fun ** 2)), rel=1e-8)


def test_fit_scale_and_empty_bins():
    rng = np.random.default_rng(6)
    f = np.logspace(-4, -1, 30)
    fb = 5e-3
    y = 10 ** (eq3_log(f, 0.0, fb, 1.0, 2.0) + rng.normal(0, 0.1, len(f)))
    p = oracle.psd_fit(f, y, fb)
    q = oracle.psd_fit(f, 1000.0 * y, fb)
    assert q[0] == pytest.approx(p[0] + 3.0, abs=1e-10)
    assert np.allclose(q[1:], p[1:], atol=1e-10)
    y0 = y.copy()
    y0[[3, 17]] = 0.0
    keep = np.ones(len(f), bool)
    keep[[3, 17]] = False
    assert np.allclose(oracle.psd_fit(f, y0, fb), oracle.psd_fit(f[keep], y[keep], fb), atol=1e-12)


def test_fit_of_timmer_koenig_periodograms():
    """Periodograms (Eq. A2) of TK95 series with the oracle's moduli and
    numpy's inverse FFT, averaged over 40 realisations and log-binned:
    the fitted slopes are the input ones within 0.1."""
    n, dt = 2 ** 14, 1.0
    p = oracle.psd_params(0.0, 1 / 300.0, 1.2, 2.7)
    acc = 0.0
    rng = np.random.default_rng(7)
    for s in range(40):
        amp = oracle.psd_spectrum(p, n, dt, seed=s, curve_id=0)
        ph = rng.uniform(0, 2 * np.pi, len(amp))
        X = amp * np.exp(1j * ph)
        X[0] = 0.0
        X[-1] = amp[-1]
        x = np.fft.irfft(X, n)
        acc = acc + oracle.periodogram(x)
    fm, pm = oracle.log_binned_mean_f(acc / 40, n, dt, 0.1)
    fit = oracle.psd_fit(fm, pm, p.f_br, 1.0, 2.0)
    assert abs(fit[1] - 1.2) < 0.1 and abs(fit[2] - 2.7) < 0.1, fit


def test_fit_rejects_bad_input():
    f = np.logspace(-3, -1, 10)
    y = np.ones(10)
    with pytest.raises(oracle.OracleError):
        oracle.psd_fit(f, y, 1e-4)           # every bin above the break
    with pytest.raises(oracle.OracleError):
        oracle.psd_fit(f[:2], y[:2], 2e-3)   # fewer than 3 bins
    with pytest.raises(oracle.OracleError):
        oracle.psd_fit(f, y, -1.0)


def test_fit_single_power_law_reaches_the_minimum():
    """Noisy data from one power law (equal slopes): there the two slope
    columns of the Jacobian coincide; the fit still reaches the least-squares
    minimum found by scipy from several starts (rms to 1e-9, log10 A and the
    mean slope to 1e-6)."""
    rng = np.random.default_rng(11)
    n, fb = 2 ** 14, 1 / 300.0
    fm, _ = oracle.log_binned_mean_f(np.ones(n // 2 + 1), n, 1.0, 0.1)
    y = eq3_log(fm, 0.5, fb, 1.6, 1.6) + rng.normal(0, 0.15, len(fm))
    p = oracle.psd_fit(fm, 10 ** y, fb, 1.0, 2.0)
    best = None
    for x0 in ([0.0, 1.0, 2.0], [0.0, 1.6, 1.6001], [0.0, 0.5, 3.0]):
        res = optimize.least_squares(lambda t: eq3_log(fm, t[0], fb, t[1], t[2]) - y, x0,
                                     xtol=1e-15, ftol=1e-15, gtol=1e-15)
        r = np.sqrt(np.mean(res.fun ** 2))
        if best is None or r < best[0]:
            best = (r, res.x)
    assert p[3] == pytest.approx(best[0], rel=1e-9)
    assert p[0] == pytest.approx(best[1][0], abs=1e-6)
    assert 0.5 * (p[1] + p[2]) == pytest.approx(0.5 * (best[1][1] + best[1][2]), abs=1e-6)
