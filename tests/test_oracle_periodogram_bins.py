"""Pins of the oracle's periodogram (Eq. A2 of Appendix A) and of its
logarithmic frequency bins, against things other than the oracle itself:

- numpy's FFT (an independent transform) for P_j = 2 / N^2 |X_j|^2;
- Parseval's identity written for the one-sided periodogram,
  P_0 + 2 sum_{0<j<N/2} P_j + P_{N/2} = (2 / N) sum_t x_t^2;
- closed forms: a cosine at Fourier frequency m puts 2 (N/2)^2 / N^2 = 1/2
  into P_m and nothing elsewhere, a constant c puts 2 c^2 into P_0;
- the 0.1-dex bins of N = 64 listed by hand (which j falls into which bin).

A planted 1/N^2 (for 2/N^2) fails the numpy, Parseval and cosine checks; a
bin edge moved by one Fourier frequency fails the hand-listed bins.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n", [2, 4, 6, 8, 12, 64, 96, 1024, 1536, 4096, 3 * 2**11])
def test_periodogram_equals_numpy_fft(n):
    x = np.random.default_rng(n).standard_normal(n) * 3.0 + 0.5
    P = oracle.periodogram(x)
    X = np.fft.rfft(x)
    ref = 2.0 / n**2 * np.abs(X) ** 2
    assert P.shape == (n // 2 + 1,)
    scale = 2.0 / n**2 * n * np.sum(x * x)  # bound on any single 2 / N^2 |X_j|^2
    assert np.all(np.abs(P - ref) <= 1e-13 * scale + 1e-300)


@pytest.mark.parametrize("n", [2, 6, 64, 3 * 2**9, 2**14])
def test_periodogram_parseval(n):
    x = np.random.default_rng(7 + n).lognormal(size=n)
    P = oracle.periodogram(x)
    lhs = P[0] + 2.0 * np.sum(P[1:n // 2]) + P[n // 2]
    rhs = 2.0 / n * np.sum(x * x)
    assert abs(lhs - rhs) <= 1e-12 * rhs


@pytest.mark.parametrize("n,m", [(64, 5), (96, 1), (1024, 200), (48, 24)])
def test_periodogram_cosine_and_constant(n, m):
    t = np.arange(n)
    P = oracle.periodogram(np.cos(2 * np.pi * m * t / n))
    # X_m = N/2 (interior) or N (Nyquist bin, where the cosine is (-1)^t)
    want = 2.0 / n**2 * (n / 2.0) ** 2 if m < n // 2 else 2.0
    others = np.delete(P, m)
    assert abs(P[m] - want) <= 1e-13
    assert np.all(others <= 1e-24)
    c = 0.75
    Pc = oracle.periodogram(np.full(n, c))
    assert abs(Pc[0] - 2.0 * c * c) <= 1e-14 and np.all(Pc[1:] <= 1e-26)


# N = 64, dex = 0.1: bin b holds the j (1 <= j <= 32) with
# floor(10 log10 j) = b (no j sits within 1e-9 of an edge except the decade
# j = 10, whose log10 is exactly 1, so it opens bin 10).  Listed by hand.
BINS_64 = {
    0: [1],
    3: [2],
    4: [3],
    6: [4, 5],
    7: [6],
    8: [7],
    9: [8, 9],
    10: [10, 11, 12],
    11: [13, 14, 15],
    12: [16, 17, 18, 19],
    13: [20, 21, 22, 23, 24, 25],
    14: [26, 27, 28, 29, 30, 31],
    15: [32],
}


def test_log_bins_listed_by_hand():
    n, dt, dex = 64, 2.0, 0.1
    P = np.random.default_rng(1).uniform(1.0, 2.0, n // 2 + 1)
    fc, mean = oracle.log_binned(P, n, dt, dex)
    fm, mean2 = oracle.log_binned_mean_f(P, n, dt, dex)
    f1 = 1.0 / (n * dt)
    assert len(mean) == len(BINS_64) == len(mean2)
    for i, (b, js) in enumerate(sorted(BINS_64.items())):
        assert mean[i] == pytest.approx(np.mean([P[j] for j in js]), rel=1e-15)
        assert mean2[i] == mean[i]
        assert fm[i] == pytest.approx(np.mean([j * f1 for j in js]), rel=1e-15)
        assert fc[i] == pytest.approx(f1 * 10 ** ((b + 0.5) * dex), rel=1e-14)
    # every j in exactly one listed bin
    assert sorted(j for js in BINS_64.values() for j in js) == list(range(1, n // 2 + 1))


def test_log_bins_ignore_dc_and_hold_each_frequency_once():
    """P_0 (the mean) never enters a bin.  A periodogram that is 1 at a single
    j and 0 elsewhere has exactly one non-zero bin mean, 1 / (count of that
    bin); the bin index never decreases with j, and the counts read back this
    way add up to N/2 (every j in exactly one bin)."""
    for n in (96, 1024, 3 * 2**10):
        P = np.ones(n // 2 + 1)
        P[0] = 1e300
        _, mean = oracle.log_binned(P, n, 1.0, 0.1)
        assert np.all(mean == 1.0)
        last, counts = -1, {}
        for j in range(1, n // 2 + 1):
            e = np.zeros(n // 2 + 1)
            e[j] = 1.0
            _, m = oracle.log_binned(e, n, 1.0, 0.1)
            nz = np.flatnonzero(m)
            assert len(nz) == 1 and nz[0] >= last
            last = nz[0]
            counts[last] = 1.0 / m[last]
        assert sum(counts.values()) == pytest.approx(n // 2, rel=1e-12)
        assert len(counts) == len(mean)


def test_library_bin_count_matches_hand_listing():
    """The library's host-side bin count (used to size the device bins): the
    hand-listed case, and the oracle's bins at other lengths."""
    import paper_1909_06374_amd as agn
    try:
        agn.lib()
    except (RuntimeError, OSError):
        pytest.skip("libagn.so not built")
    assert agn.agn_log_bin_count(64, 0.1) == len(BINS_64)
    for n in (96, 1024, 3 * 2**12, 2**20):
        for dex in (0.1, 0.25):
            _, mean = oracle.log_binned(np.ones(n // 2 + 1), n, 1.0, dex)
            assert agn.agn_log_bin_count(n, dex) == len(mean)
