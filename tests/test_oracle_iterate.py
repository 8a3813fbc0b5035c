"""Pins of the oracle's iteration (Sec. 2.1, Sec. 3.2.2, Eq. 4).

Invariants the paper states (values fixed, only reordered), a fixed point,
symmetries that hold in exact arithmetic (scale, cyclic shift, time reversal),
the N = 2 case worked by hand, chained runs, the same loop written with
numpy's FFT and sort, and the method's purpose: the output spectrum follows
the target moduli.
"""
import numpy as np
import pytest

import oracle
from paper_1909_06374_amd import synth


def spectrum(n, seed=0, f_br=0.05, a_low=1.0, a_high=2.0):
    return oracle.psd_spectrum(oracle.psd_params(0.0, f_br, a_low, a_high), n, 1.0, seed)


def test_replace_special_cases():
    n = 8
    X = np.array([3 + 0j, 1 + 1j, 0j, -2 + 0.5j, -4 + 0j])
    amp = np.array([9.0, 2.0, 3.0, 4.0, 5.0])
    Y = oracle.replace(X, amp, n)
    assert Y[0] == 0  # DC removed
    assert Y[2] == 3.0  # zero modulus: phase 0
    assert Y[4] == -5.0  # Nyquist keeps the sign of Re X
    assert np.allclose(np.abs(Y[1:4]), amp[1:4])
    assert np.allclose(np.angle(Y[[1, 3]]), np.angle(X[[1, 3]]))
    Y = oracle.replace(np.array([1 + 0j, 0j, 0j, 0j, 0j]), amp, n)
    assert Y[4] == 5.0  # sign(0) = +1


@pytest.mark.parametrize("n", [2, 4, 6, 8, 12, 64, 96, 256, 768, 1024])
def test_values_fixed_only_reordered(n):
    x0 = synth.erdf_draw(n, seed=n)
    x, delta, done, rank = oracle.iterate(spectrum(n, seed=n), x0, 7)
    s = np.sort(x0)
    assert np.array_equal(np.sort(x), s)
    assert np.array_equal(s[rank], x)
    assert done == 7 and np.all(delta >= 0)


def test_fixed_point_from_own_moduli():
    n = 256
    x0 = synth.erdf_draw(n, seed=3)
    amp = np.abs(oracle.rfft(x0))
    amp[0] = 0.0
    x, delta, done, _ = oracle.iterate(amp, x0, 5)
    assert np.array_equal(x, x0)
    assert np.all(delta == 0.0)
    x, delta, done, _ = oracle.iterate(amp, x0, 5, tol=0.0)
    assert done == 1 and delta[0] == 0.0


@pytest.mark.parametrize("n", [64, 96, 512])
def test_symmetries(n):
    x0 = synth.erdf_draw(n, seed=10 + n)
    amp = spectrum(n, seed=n)
    x, _, _, _ = oracle.iterate(amp, x0, 6)
    # Positive scale of the target moduli.
    xs, _, _, _ = oracle.iterate(amp * 8.0, x0, 6)
    assert np.array_equal(xs, x)
    # Cyclic shift in time.
    m = n // 3
    xc, _, _, _ = oracle.iterate(amp, np.roll(x0, m), 6)
    assert np.array_equal(xc, np.roll(x, m))
    # Time reversal t -> -t mod N.
    rev = lambda v: np.concatenate([v[:1], v[:0:-1]])
    xr, _, _, _ = oracle.iterate(amp, rev(x0), 6)
    assert np.array_equal(xr, rev(x))


def test_two_point_case_by_hand():
    # N = 2: y = (Y1, -Y1) with Y1 = amp1 * sign(x0 - x1); the order is kept.
    for x0 in ([0.3, 0.1], [0.1, 0.3], [0.2, 0.2]):
        x, delta, _, _ = oracle.iterate(np.array([0.0, 1.0]), np.array(x0), 3)
        assert list(x) == x0 and np.all(delta == 0)
    # No power at all: y = 0 ties, broken by index -> ascending order.
    x, _, _, _ = oracle.iterate(np.array([0.0, 0.0]), np.array([0.3, 0.1]), 1)
    assert list(x) == [0.1, 0.3]


def test_delta_is_eq4_on_consecutive_series_and_runs_chain():
    n = 128
    x0 = synth.erdf_draw(n, seed=5)
    amp = spectrum(n, seed=5, f_br=0.02, a_high=2.5)
    x_all, d_all, _, _ = oracle.iterate(amp, x0, 6)
    prev = x0
    for i in range(6):
        cur, d1, _, _ = oracle.iterate(amp, prev, 1)
        expect = np.sqrt(np.mean(np.log10(cur / prev) ** 2))
        assert d1[0] == pytest.approx(expect, rel=1e-14, abs=1e-300)
        assert d_all[i] == pytest.approx(d1[0], rel=1e-15, abs=1e-300)
        assert (d1[0] == 0.0) == np.array_equal(cur, prev)
        prev = cur
    assert np.array_equal(prev, x_all)


def test_stopping_rules():
    n = 1024
    w = synth.single_curve(n=n, seed=0)
    amp = oracle.psd_spectrum(oracle.psd_params(**w["params"]), n, 1.0, 0)
    x_full, d_full, done_full, _ = oracle.iterate(amp, w["erdf"], 60)
    assert done_full == 60
    x0, d0, done0, _ = oracle.iterate(amp, w["erdf"], 60, tol=0.0)
    # The run reaches an exact fixed point; stopping there does not change x.
    assert done0 < 60 and np.array_equal(x0, x_full) and d0[done0 - 1] == 0.0
    assert np.all(d0[done0:] == 0.0) and np.array_equal(d0[:done0], d_full[:done0])
    tol = d_full[5] * 1.0000001
    _, dt_, done_t, _ = oracle.iterate(amp, w["erdf"], 60, tol=tol)
    assert done_t == int(np.argmax(d_full <= tol)) + 1


def numpy_loop(amp, x0, iters):
    s = np.sort(x0)
    x = x0.copy()
    n = len(x0)
    for _ in range(iters):
        X = np.fft.rfft(x)
        m = np.abs(X)
        Y = np.where(m > 0, amp * X / np.where(m > 0, m, 1.0), amp + 0j)
        Y[0] = 0.0
        Y[-1] = amp[-1] * (1.0 if X[-1].real >= 0 else -1.0)
        y = np.fft.irfft(Y, n)
        nx = np.empty_like(x)
        nx[np.argsort(y, kind="stable")] = s
        x = nx
    return x


@pytest.mark.parametrize("n,seed", [(64, 1), (96, 2), (1024, 3), (1536, 4), (4096, 5)])
def test_matches_numpy_fft_and_sort_loop(n, seed):
    x0 = synth.erdf_draw(n, seed=seed)
    amp = spectrum(n, seed=seed, f_br=1 / 200.0, a_low=1.0, a_high=2.5)
    x, _, _, _ = oracle.iterate(amp, x0, 20)
    assert np.array_equal(x, numpy_loop(amp, x0, 20))


def test_output_spectrum_follows_target():
    """With a narrow-range PDF the iteration matches the target moduli closely:
    the log-binned periodogram of the output tracks amp^2 bin by bin."""
    n = 4096
    rng = np.random.default_rng(9)
    ratios = []
    for r in range(20):
        x0 = 10.0 + rng.standard_normal(n)
        amp = spectrum(n, seed=100 + r, f_br=1 / 100.0, a_low=1.0, a_high=2.0)
        x, _, _, _ = oracle.iterate(amp, x0, 100)
        X = oracle.rfft(x - x.mean())
        P_out = np.abs(X[1:]) ** 2
        _, a = oracle.log_binned(np.concatenate([[0], amp[1:] ** 2]), n, 1.0)
        _, b = oracle.log_binned(np.concatenate([[0], P_out]), n, 1.0)
        ratios.append(b / a)
    ratios = np.array(ratios)
    scale = np.median(ratios)
    rel = np.mean(ratios, axis=0) / scale
    # bin-by-bin agreement of the shape (spanning ~3.3 decades of frequency and
    # ~8 decades of power)
    assert np.all(np.abs(np.log10(rel)) < 0.15), rel


def test_tk95_ensemble_periodogram_is_psd():
    """Mean periodogram (Eq. A2) of TK95 realisations equals the input PSD in
    expectation (>= 50 realisations; Sec. 3.2.5)."""
    n, dt = 1024, 1.0
    p = oracle.psd_params(0.0, 1 / 200.0, 1.0, 2.5)
    A = oracle.psd_norm(p, n, dt)
    P = np.array([oracle.psd_eq3(j / (n * dt), A, p.f_br, p.a_low, p.a_high) for j in range(1, n // 2)])
    acc = np.zeros(n // 2 - 1)
    R = 200
    for s in range(R):
        amp = oracle.psd_spectrum(p, n, dt, seed=s)
        acc += amp[1:n // 2] ** 2
    ratio = acc / R / P
    # each bin: mean of R Exp(1) draws; binned over 0.1 dex
    _, rb = oracle.log_binned(np.concatenate([[0], ratio, [1.0]]), n, dt)
    assert np.all(np.abs(rb - 1.0) < 5 / np.sqrt(R))


def test_invalid_draw_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.iterate(np.ones(5), np.array([1.0, -1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0]), 1)
    with pytest.raises(oracle.OracleError):
        oracle.iterate(np.ones(5), np.array([1.0, np.inf, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0]), 1)


def test_oracle_regression_fixture():
    import hashlib, json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_single_curve.json")))
    w = synth.single_curve(n=1024, seed=0)
    assert hashlib.sha256(w["erdf"].tobytes()).hexdigest() == g["erdf_sha256"]
    p = oracle.psd_params(**w["params"])
    x, delta, done, rank = oracle.generate(p, w["erdf"], w["dt"], 50, seed=0)
    assert hashlib.sha256(x.tobytes()).hexdigest() == g["x_out_sha256"]
    assert list(delta) == g["delta"] and done == g["iters_done"]
