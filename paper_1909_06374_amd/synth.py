"""Seeded synthetic inputs for the light-curve generator.

This module holds input generators only -- none of the method's arithmetic.
Both the GPU path and the CPU oracle receive the arrays made here.

The workloads stand in for the paper's PTF/iPTF-like and LSST-like use cases
(Sec. 4.1, Sec. 4.2); no survey data is used.

ERDF draw.  The method takes a sample of L/L_Edd values (the PDF draw of
Sec. 2.1, step ii) as an input.  The sample used here is a sharp broken power
law in dN/dlog(lambda), with Eq. 1's slope convention (dN/dlog lambda falls as
(lambda/lambda*)^-delta1 below the break and ^-delta2 above it), on
u = log10(lambda) in [u_min, u_max], drawn by its closed-form inverse CDF and
returned as linear lambda = 10^u (the simulated quantity is L/L_Edd itself,
Sec. 2, and Eq. 4 needs positive values).
"""
from __future__ import annotations

import math

import numpy as np

LN10 = math.log(10.0)


def _rng(seed: int, stream: int, index: int) -> np.random.Generator:
    """Independent numpy Philox generator per (seed, stream, index)."""
    key = np.array([seed & (2**64 - 1), ((stream & 0xFFFFFFFF) << 32) | (index & 0xFFFFFFFF)],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def erdf_bpl_masses(u_min=-4.0, u_max=0.0, u_br=-1.5, d1=0.4, d2=2.5):
    """Unnormalised probability mass below and above the break."""
    m1 = (10.0 ** (d1 * (u_br - u_min)) - 1.0) / (d1 * LN10)
    m2 = (1.0 - 10.0 ** (-d2 * (u_max - u_br))) / (d2 * LN10)
    return m1, m2


def erdf_bpl_u_from_uniform(U, u_min=-4.0, u_max=0.0, u_br=-1.5, d1=0.4, d2=2.5):
    """Inverse CDF of the sharp broken power law in u = log10(lambda)."""
    U = np.asarray(U, dtype=np.float64)
    m1, m2 = erdf_bpl_masses(u_min, u_max, u_br, d1, d2)
    t = U * (m1 + m2)
    lo = t < m1
    u = np.empty_like(t)
    u[lo] = u_br - np.log10(10.0 ** (d1 * (u_br - u_min)) - t[lo] * d1 * LN10) / d1
    th = t[~lo] - m1
    u[~lo] = u_br - np.log10(np.maximum(1.0 - th * d2 * LN10, 10.0 ** (-d2 * (u_max - u_br)))) / d2
    return np.clip(u, u_min, u_max)


def erdf_bpl_cdf(u, u_min=-4.0, u_max=0.0, u_br=-1.5, d1=0.4, d2=2.5):
    """Closed-form CDF in u (for tests)."""
    u = np.asarray(u, dtype=np.float64)
    m1, m2 = erdf_bpl_masses(u_min, u_max, u_br, d1, d2)
    below = (10.0 ** (d1 * (u_br - u_min)) - 10.0 ** (-d1 * (u - u_br))) / (d1 * LN10)
    above = m1 + (1.0 - 10.0 ** (-d2 * (u - u_br))) / (d2 * LN10)
    return np.where(u < u_br, below, above) / (m1 + m2)


def erdf_draw(n: int, seed: int, curve_id: int = 0, **kw) -> np.ndarray:
    """n i.i.d. L/L_Edd values (linear), in draw order."""
    U = _rng(seed, 1, curve_id).random(n)
    return 10.0 ** erdf_bpl_u_from_uniform(U, **kw)


# ---------------------------------------------------------------------------
# Per-curve PSD parameters (PTF-like batches): a_low ~ U(0.8, 1.2),
# a_high ~ U(2, 3), log10 f_b ~ U(log10(1/1000), log10(1/50)) per day.
# ---------------------------------------------------------------------------
def curve_params(n_curves: int, seed: int):
    r = _rng(seed, 3, 0)
    a_low = r.uniform(0.8, 1.2, n_curves)
    a_high = r.uniform(2.0, 3.0, n_curves)
    log_fb = r.uniform(math.log10(1.0 / 1000.0), math.log10(1.0 / 50.0), n_curves)
    return a_low, a_high, 10.0 ** log_fb


def size_grid(k_lo: int, k_hi: int):
    """Lengths {2^k, k_lo..k_hi} U {3 * 2^k, 3 * 2^k <= 2^k_hi, 3 * 2^k >= 2^k_lo}."""
    g = [2**k for k in range(k_lo, k_hi + 1)]
    g += [3 * 2**k for k in range(k_lo - 1, k_hi) if 2**k_lo <= 3 * 2**k <= 2**k_hi]
    return sorted(g)


def uneven_sizes(n_curves: int, seed: int, k_lo=10, k_hi=20):
    """Uniform choice over the size grid (log-uniform over the 2^a 3^b lengths)."""
    g = np.array(size_grid(k_lo, k_hi), dtype=np.int64)
    return g[_rng(seed, 5, 0).integers(0, len(g), n_curves)]


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int):
    r = _rng(seed, 4, 0)
    t, out = 0.0, []
    while True:
        t += r.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append(t)
    return np.array(out)


def request_iters(n_req: int, seed: int, lo=50, hi=200):
    return _rng(seed, 6, 0).integers(lo, hi + 1, n_req).astype(np.int32)


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------
DAY = 1.0
YEAR = 365.25


def single_curve(n=1024, seed=0, dt=1.0, f_b=1.0 / 200.0, a_low=1.0, a_high=2.5):
    """One curve, bending power law, unit variance, ERDF of n draws."""
    return dict(n=n, dt=dt, params=dict(norm=0.0, f_br=f_b, a_low=a_low, a_high=a_high),
                erdf=erdf_draw(n, seed, 0), seed=seed)


def ptf_batch(n_curves=1024, n=2**14, seed=1, dt=1.0):
    """PTF-like batch: per-curve PSD slopes and break, ERDF of n draws per curve."""
    a_low, a_high, f_b = curve_params(n_curves, seed)
    erdf = np.stack([erdf_draw(n, seed, c) for c in range(n_curves)])
    return dict(n=n, dt=dt, a_low=a_low, a_high=a_high, f_br=f_b, erdf=erdf, seed=seed)
