"""Pins of the oracle's DFT (Appendix A, Eq. A1 up to the sign convention) and
of its stable argsort: a naive O(N^2) long-double DFT, Parseval, impulse and
cosine closed forms, the round trip, numpy's FFT, and brute-force ranks."""
import itertools
import math

import numpy as np
import pytest

import oracle


def sizes(limit):
    out = []
    for a in range(0, 12):
        for b in range(0, 3):
            n = 2**a * 3**b
            if n <= limit:
                out.append(n)
    return sorted(out)


PI_LD = np.longdouble("3.14159265358979323846264338327950288")


def naive_dft(z, sign):
    """O(n^2) DFT in long double; the phase index jk is reduced mod n exactly."""
    n = len(z)
    k = np.arange(n, dtype=np.int64)
    jk = (np.outer(k, k) % n).astype(np.longdouble)
    ang = sign * 2 * PI_LD * jk / n
    W = np.cos(ang) + 1j * np.sin(ang)  # complex256
    zz = z.astype(np.clongdouble)
    return W @ zz


@pytest.mark.parametrize("n", sizes(432))
def test_dft_matches_naive_longdouble(n):
    rng = np.random.default_rng(n)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, 1):
        got = oracle.dft(z, sign)
        ref = naive_dft(z, sign)
        err = np.abs(got.astype(np.clongdouble) - ref).max()
        bound = 5 * 2.0**-53 * max(1.0, math.log2(n)) * np.linalg.norm(z) * math.sqrt(n)
        assert float(err) <= bound


@pytest.mark.parametrize("n", [2, 4, 6, 8, 12, 48, 96, 1024, 1536, 3072])
def test_rfft_parseval_roundtrip_numpy(n):
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal(n)
    X = oracle.rfft(x)
    lhs = abs(X[0]) ** 2 + 2 * (np.abs(X[1:n // 2]) ** 2).sum() + abs(X[n // 2]) ** 2
    assert lhs == pytest.approx(n * (x ** 2).sum(), rel=1e-13)
    assert np.allclose(oracle.irfft(X, n), n * x, rtol=0, atol=1e-12 * n * np.abs(x).max())
    assert np.allclose(X, np.fft.rfft(x), rtol=0, atol=1e-12 * np.abs(x).sum())


@pytest.mark.parametrize("n", [8, 24, 64, 96])
def test_impulse_and_cosine(n):
    j = np.arange(n // 2 + 1)
    for n0 in [0, 1, 5 % n, n - 1]:
        x = np.zeros(n)
        x[n0] = 1.0
        X = oracle.rfft(x)
        assert np.allclose(X, np.exp(-2j * np.pi * j * n0 / n), atol=1e-14)
    for m in [1, 3, n // 2 - 1]:
        x = np.cos(2 * np.pi * m * np.arange(n) / n)
        X = oracle.rfft(x)
        expect = np.zeros(n // 2 + 1, dtype=complex)
        expect[m] = n / 2
        assert np.allclose(X, expect, atol=1e-12 * n)
    # Nyquist cosine: all weight in the real Nyquist bin.
    x = np.cos(np.pi * np.arange(n))
    X = oracle.rfft(x)
    assert X[n // 2] == pytest.approx(n, abs=1e-12) and np.abs(X[:-1]).max() < 1e-12


def test_irfft_is_unnormalised_hermitian_inverse():
    n = 48
    rng = np.random.default_rng(5)
    Y = rng.standard_normal(n // 2 + 1) + 1j * rng.standard_normal(n // 2 + 1)
    Y[0] = Y[0].real
    Y[-1] = Y[-1].real
    full = np.concatenate([Y, np.conj(Y[-2:0:-1])])
    ref = np.array([(full * np.exp(2j * np.pi * np.arange(n) * t / n)).sum().real for t in range(n)])
    assert np.allclose(oracle.irfft(Y, n), ref, atol=1e-12)


def brute_ranks(y):
    n = len(y)
    return np.array([sum((y[m] < y[i]) or (y[m] == y[i] and m < i) for m in range(n)) for i in range(n)])


def test_argsort_brute_force_with_ties():
    rng = np.random.default_rng(0)
    for n in [1, 2, 3, 7, 16, 33]:
        for _ in range(20):
            y = rng.integers(0, 4, n).astype(float) * 0.5 - 1.0
            perm = oracle.argsort(y)
            rank = brute_ranks(y)
            assert np.array_equal(perm[rank], np.arange(n))


def test_argsort_exhaustive_small():
    for n in range(1, 7):
        for p in itertools.permutations(range(n)):
            y = np.array(p, dtype=float)
            assert np.array_equal(oracle.argsort(y), np.argsort(y, kind="stable"))


def test_argsort_numpy_stable_and_signed_zero():
    rng = np.random.default_rng(1)
    y = rng.standard_normal(5000)
    y[::7] = y[3]
    assert np.array_equal(oracle.argsort(y), np.argsort(y, kind="stable"))
    z = np.array([0.0, -0.0, 1.0, -0.0, 0.0, -1.0])
    assert list(oracle.argsort(z)) == [5, 0, 1, 3, 4, 2]


def test_argsort_rejects_nan():
    with pytest.raises(oracle.OracleError):
        oracle.argsort(np.array([1.0, np.nan, 0.0]))
