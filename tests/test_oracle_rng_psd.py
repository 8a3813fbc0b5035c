"""Pins of the oracle's random numbers, Eq. 3 and the Timmer-Koenig moduli.

Each check compares the oracle with something other than itself: numpy's
independent Philox4x64-10, closed forms of Eq. 3, the variance of series
built with numpy's inverse FFT, and the Exp(1) / chi^2_1 laws of the moduli.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from pdf_reference import quad_cdf as _quad_cdf


def numpy_philox_block(key, block):
    """Block `block` of Philox4x64-10 under `key` from numpy's implementation.
    numpy increments the counter before each block, so start one below."""
    ctr = (block - 1) % (2**256)
    words = [(ctr >> (64 * i)) & (2**64 - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("key", [(0, 0), (12345, 678), (2**64 - 1, 2**63 + 5), (0xDEADBEEF, 3 << 32 | 17)])
def test_philox_matches_numpy(key):
    for block in [0, 1, 2, 7, 1000, 2**40 + 3]:
        assert oracle.philox4x64([block, 0, 0, 0], key) == numpy_philox_block(key, block)


def test_uniform_stream_layout_and_mapping():
    for seed, stream, curve in [(0, 0, 0), (7, 1, 3), (2**63 + 11, 0, 1023)]:
        key = (seed, (stream << 32) | curve)
        for k in [0, 1, 2, 3, 4, 5, 1023, 4097]:
            w = numpy_philox_block(key, k // 4)[k % 4]
            expect = ((w >> 12) + 0.5) * 2.0**-52
            assert oracle.uniform(seed, stream, curve, k) == expect
            assert 0.0 < expect < 1.0


def test_uniforms_are_uniform():
    u = np.array([oracle.uniform(3, 0, 5, k) for k in range(20000)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_eq3_closed_forms():
    A, fb = 3.7, 0.01
    # At the break both terms are 1.
    assert oracle.psd_eq3(fb, A, fb, 1.0, 2.5) == pytest.approx(A / 2, rel=1e-15)
    # Equal slopes: a single power law of half the amplitude.
    for f in [1e-4, 3e-3, 0.2]:
        assert oracle.psd_eq3(f, A, fb, 1.7, 1.7) == pytest.approx(0.5 * A * (f / fb) ** -1.7, rel=1e-14)
    # Asymptotes.
    assert oracle.psd_eq3(fb * 1e-6, A, fb, 1.0, 2.0) / (A * 1e6) == pytest.approx(1.0, rel=2e-6)
    assert oracle.psd_eq3(fb * 1e6, A, fb, 1.0, 2.0) / (A * 1e-12) == pytest.approx(1.0, rel=2e-6)
    # The bending form A f^-1 / (1 + (f/f_b)^1.5) is Eq. 3 with slopes (1, 2.5).
    for f in [1e-4, 5e-3, 0.1, 0.5]:
        bend = A * (fb / f) / (1.0 + (f / fb) ** 1.5)
        assert oracle.psd_eq3(f, A, fb, 1.0, 2.5) == pytest.approx(bend, rel=1e-13)


def test_norm_gives_unit_variance_series():
    """TK95 series built with numpy (complex Gaussians of variance P/2 per
    component, real Nyquist, zero DC, numpy's inverse FFT) have unit mean
    variance under the oracle's normalisation."""
    n, dt = 512, 1.0
    p = oracle.psd_params(0.0, 1 / 50.0, 1.0, 2.0)
    A = oracle.psd_norm(p, n, dt)
    j = np.arange(1, n // 2 + 1)
    P = np.array([oracle.psd_eq3(jj / (n * dt), A, p.f_br, p.a_low, p.a_high) for jj in j])
    rng = np.random.default_rng(0)
    R = 4000
    X = np.zeros((R, n // 2 + 1), dtype=complex)
    X[:, 1:] = np.sqrt(P / 2) * (rng.standard_normal((R, n // 2)) + 1j * rng.standard_normal((R, n // 2)))
    X[:, -1] = np.sqrt(P[-1] / 2) * rng.standard_normal(R)
    x = np.fft.irfft(X, n, axis=1)
    v = (x ** 2).mean(axis=1)
    assert abs(v.mean() - 1.0) < 4 * v.std() / math.sqrt(R)


def test_tk95_moduli_laws():
    n, dt = 2**16, 1.0
    p = oracle.psd_params(0.0, 1 / 300.0, 1.2, 2.7)
    A = oracle.psd_norm(p, n, dt)
    amp = oracle.psd_spectrum(p, n, dt, seed=11, curve_id=2)
    assert amp[0] == 0.0
    j = np.arange(1, n // 2)
    P = np.array([oracle.psd_eq3(jj / (n * dt), A, p.f_br, p.a_low, p.a_high) for jj in j])
    e = amp[1:n // 2] ** 2 / P
    assert stats.kstest(e, "expon").pvalue > 1e-3
    assert abs(e.mean() - 1.0) < 4 / math.sqrt(len(e))
    # Nyquist bin: amp^2 / (P/2) ~ chi^2 with one degree of freedom.
    m = 6
    Pn = oracle.psd_eq3(0.5 / dt, oracle.psd_norm(p, m, dt), p.f_br, p.a_low, p.a_high)
    ny = np.array([oracle.psd_spectrum(p, m, dt, seed=s, curve_id=0)[m // 2] for s in range(3000)])
    assert stats.kstest(ny ** 2 / (Pn / 2), "chi2", args=(1,)).pvalue > 1e-3
    # Expected sum of squared moduli gives unit variance (normalisation).
    tot = []
    for s in range(200):
        a = oracle.psd_spectrum(p, 256, dt, seed=s, curve_id=0)
        tot.append((2 * (a[1:128] ** 2).sum() + a[128] ** 2) / 256**2)
    tot = np.array(tot)
    assert abs(tot.mean() - 1.0) < 4 * tot.std() / math.sqrt(len(tot))


def test_tk95_seed_and_curve_streams_differ():
    p = oracle.psd_params(0.0, 0.01, 1.0, 2.0)
    a = oracle.psd_spectrum(p, 64, 1.0, seed=1, curve_id=0)
    b = oracle.psd_spectrum(p, 64, 1.0, seed=1, curve_id=1)
    c = oracle.psd_spectrum(p, 64, 1.0, seed=2, curve_id=0)
    d = oracle.psd_spectrum(p, 64, 1.0, seed=1, curve_id=0)
    assert np.array_equal(a, d)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_spectrum_rejects_bad_input():
    p = oracle.psd_params(0.0, 0.01, 1.0, 2.0)
    for n in [0, 3, 10, 14]:
        with pytest.raises(oracle.OracleError):
            oracle.psd_spectrum(p, n, 1.0, 0)
    with pytest.raises(oracle.OracleError):
        oracle.psd_spectrum(oracle.psd_params(0.0, -1.0, 1.0, 2.0), 8, 1.0, 0)


def test_erdf_sampler_closed_form_cdf():
    """PDF draw (Sec. 2.1 step ii): KS against the closed-form CDF of the
    sharp broken power law, mass below the break, support, seeding."""
    from paper_1909_06374_amd import synth
    p = oracle.erdf_params()
    lam = oracle.erdf_bpl(p, 100000, seed=9, curve_id=4)
    u = np.log10(lam)
    assert np.all((u >= -4.0) & (u <= 0.0))
    assert stats.kstest(u, synth.erdf_bpl_cdf).pvalue > 1e-3
    frac = np.mean(u < -1.5)
    assert abs(frac - 0.98254) < 5 * math.sqrt(0.98254 * 0.01746 / len(u))
    # uniform #k of stream 1 drives draw k through the inverse CDF
    U = np.array([oracle.uniform(9, 1, 4, k) for k in range(50)])
    assert np.allclose(np.log10(lam[:50]), synth.erdf_bpl_u_from_uniform(U), rtol=0, atol=1e-13)
    assert not np.array_equal(oracle.erdf_bpl(p, 64, 9, 4), oracle.erdf_bpl(p, 64, 9, 5))
    # other parameters: a single slope (d1 = d2) is an exponential law in u
    q = oracle.erdf_params(-3.0, 0.0, -1.0, 1.0, 1.0)
    u2 = np.log10(oracle.erdf_bpl(q, 50000, 1, 0))
    lam_rate = np.log(10.0)
    cdf = lambda x: (1 - np.exp(-lam_rate * (x + 3.0))) / (1 - np.exp(-lam_rate * 3.0))
    assert stats.kstest(u2, cdf).pvalue > 1e-3


PDF_CASES = [
    # Table 2: Eq. 1 with lambda* = 0.11, slopes 0.47 / 2.53, log lambda in [-3.75, 0.5]
    dict(kind=1, measure=0), dict(kind=1, measure=1),
    # Eq. 2 with log lambda* = -3.25, sigma = 0.64 on a wide support
    dict(kind=2, measure=0, u_min=-6.0, u_max=1.0, u_star=-3.25),
    dict(kind=2, measure=1, u_min=-6.0, u_max=1.0, u_star=-3.25),
    # support entirely in the upper tail of the normal
    dict(kind=2, measure=0, u_min=-1.5, u_max=0.5, u_star=-3.25),
    # sharp broken power law, both measures, and a slope of exactly 1 (flat in u for dN/dlambda)
    dict(kind=0, measure=0), dict(kind=0, measure=1), dict(kind=0, measure=1, d1=1.0),
]


@pytest.mark.parametrize("case", PDF_CASES)
def test_pdf_draw_inverts_the_cdf(case):
    """Draw k is the inverse CDF of uniform #k of stream 1: the CDF from
    quadrature of the restated density, at the drawn value, returns that uniform."""
    p = oracle.pdf_params(**case)
    lam = oracle.pdf_draw(p, 40, seed=5, curve_id=2)
    u = np.log10(lam)
    assert np.all((u >= p.u_min) & (u <= p.u_max))
    F = _quad_cdf(p)
    for k in range(40):
        assert abs(F(u[k]) - oracle.uniform(5, 1, 2, k)) < 1e-12, (case, k)


def test_pdf_lognormal_matches_scipy_truncnorm():
    """Eq. 2 is a normal in log10(lambda); read as dN/dlambda its mean moves up
    by sigma^2 ln 10.  KS against scipy's truncated normal."""
    for measure, mean in [(0, -3.25), (1, -3.25 + 0.64 ** 2 * math.log(10.0))]:
        p = oracle.pdf_params(2, measure, u_min=-6.0, u_max=1.0, u_star=-3.25, sigma=0.64)
        u = np.log10(oracle.pdf_draw(p, 20000, seed=3, curve_id=measure))
        a, b = (-6.0 - mean) / 0.64, (1.0 - mean) / 0.64
        assert stats.kstest(u, stats.truncnorm(a, b, loc=mean, scale=0.64).cdf).pvalue > 1e-3
        assert abs(u.mean() - stats.truncnorm(a, b, loc=mean, scale=0.64).mean()) < 5 * u.std() / math.sqrt(len(u))


def test_pdf_eq1_special_cases_in_closed_form():
    """Eq. 1 with equal slopes d is half a single power law: u has the
    truncated exponential law, inverted in closed form per uniform.  With
    d = 1 and the linear measure the density in u is flat."""
    d, lo, hi = 1.7, -3.0, 0.5
    p = oracle.pdf_params(1, 0, u_min=lo, u_max=hi, u_star=-1.0, d1=d, d2=d)
    u = np.log10(oracle.pdf_draw(p, 300, seed=8, curve_id=1))
    U = np.array([oracle.uniform(8, 1, 1, k) for k in range(300)])
    expect = lo - np.log10(1.0 - U * (1.0 - 10.0 ** (-d * (hi - lo)))) / d
    assert np.max(np.abs(u - expect)) < 1e-12
    q = oracle.pdf_params(1, 1, u_min=lo, u_max=hi, u_star=-1.0, d1=1.0, d2=1.0)
    u = np.log10(oracle.pdf_draw(q, 300, seed=8, curve_id=1))
    assert np.max(np.abs(u - (lo + U * (hi - lo)))) < 1e-12


def test_pdf_sharp_kind_equals_the_erdf_sampler_and_draw_at():
    """Kind 0 in dN/dlog10(lambda) is the sharp broken power law of erdf_bpl;
    draws at chosen indices equal the same draws of the full sequence."""
    p = oracle.pdf_params(0, 0, u_min=-4.0, u_max=0.0, u_star=-1.5, d1=0.4, d2=2.5)
    a = oracle.pdf_draw(p, 500, seed=9, curve_id=4)
    b = oracle.erdf_bpl(oracle.erdf_params(), 500, seed=9, curve_id=4)
    assert np.max(np.abs(np.log10(a) - np.log10(b))) < 1e-13
    for case in [dict(kind=1, measure=1), dict(kind=2, measure=0, u_star=-2.0)]:
        q = oracle.pdf_params(**case)
        full = oracle.pdf_draw(q, 400, seed=2, curve_id=7)
        idx = np.array([399, 0, 17, 17, 250])
        assert np.array_equal(oracle.pdf_draw_at(q, idx, seed=2, curve_id=7), full[idx])


def test_pdf_eq1_table2_mass_split():
    """Table 2's Eq. 1: the fraction of draws below the cut log lambda = -1.2
    of Table 2 matches the quadrature mass (binomial bound)."""
    p = oracle.pdf_params(1, 0)
    u = np.log10(oracle.pdf_draw(p, 20000, seed=1, curve_id=0))
    m = _quad_cdf(p)(-1.2)
    assert abs(np.mean(u < -1.2) - m) < 5 * math.sqrt(m * (1 - m) / len(u))


def test_pdf_rejects_bad_parameters():
    bad = [dict(kind=3), dict(kind=0, measure=2), dict(kind=1, u_min=1.0, u_max=0.0),
           dict(kind=2, sigma=0.0), dict(kind=0, u_star=1.0), dict(kind=1, d1=float("nan"))]
    for case in bad:
        with pytest.raises(oracle.OracleError):
            oracle.pdf_draw(oracle.pdf_params(**case), 4, seed=0)
