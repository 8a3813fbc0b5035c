"""Pins of the oracle's slice sampler (Sec. 3.1: the paper draws the PDF by
slice sampling, Neal 2003, in linear lambda).

Checks: the chain counter layout against numpy's independent Philox; the
stationary law of the draws against the CDF from quadrature (KS) for Eq. 1,
Eq. 2 and the sharp law in both measures; a flat target, where every first
proposal is accepted, so that each draw is a closed form of two uniforms; a
step target, where shrinkage must confine the chain to the step; and that a
chain's draws do not depend on n.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from pdf_reference import quad_cdf


def numpy_philox(key, ctr):
    """Block with counter words ctr (4 x 64 bit) from numpy's Philox4x64,
    which increments its 256-bit counter before each block."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & (2**64 - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def test_chain_uniforms_match_numpy_philox():
    for seed, curve, chain in [(5, 0, 0), (5, 3, 1), (2**63 + 9, 11, 65535), (0, 0, 2**40)]:
        key = (seed, (6 << 32) | curve)
        for k in [0, 1, 3, 4, 7, 1001]:
            w = numpy_philox(key, [k // 4, chain, 0, 0])[k % 4]
            assert oracle.uniform_chain(seed, 6, curve, chain, k) == ((w >> 12) + 0.5) * 2.0**-52
    assert oracle.uniform_chain(7, 1, 2, 0, 13) == oracle.uniform(7, 1, 2, 13)


CASES = [dict(kind=1, measure=0), dict(kind=1, measure=1),
         dict(kind=2, measure=0, u_min=-6.0, u_max=1.0, u_star=-3.25),
         dict(kind=2, measure=1, u_min=-6.0, u_max=1.0, u_star=-3.25),
         dict(kind=0, measure=0, u_min=-4.0, u_max=0.0, u_star=-1.5, d1=0.4, d2=2.5),
         dict(kind=0, measure=1, u_min=-4.0, u_max=0.0, u_star=-1.5, d1=0.4, d2=2.5)]


@pytest.mark.parametrize("case", CASES)
def test_slice_draws_follow_the_pdf(case):
    """Proposals uniform in lambda mix slowly over several decades (lag-one
    correlation 0.6-0.8 within a chain, gone by lag 20), so the chains burn in
    for 300 steps and each gives one draw (the KS bound assumes independence)."""
    p = oracle.pdf_params(**case)
    lam = oracle.pdf_slice(p, 20000, 20000, 300, seed=4, curve_id=1)
    u = np.log10(lam)
    assert np.all((u >= p.u_min - 1e-12) & (u <= p.u_max + 1e-12))
    assert stats.kstest(u, np.vectorize(quad_cdf(p))).pvalue > 1e-3


def test_flat_target_closed_form():
    """Slope 0 on both sides read as dN/dlambda: the density is flat in lambda,
    the first proposal is always accepted, and step t of chain c uses the level
    uniform #2t and the proposal uniform #2t+1."""
    p = oracle.pdf_params(0, 1, u_min=-3.0, u_max=0.5, u_star=-1.0, d1=0.0, d2=0.0)
    C, burn, n = 7, 3, 50
    lam = oracle.pdf_slice(p, n, C, burn, seed=9, curve_id=2)
    lo, hi = 10.0 ** -3.0, 10.0 ** 0.5
    for j in range(n):
        t, c = j // C + burn, j % C
        U = oracle.uniform_chain(9, 6, 2, c, 2 * t + 1)
        assert lam[j] == lo + U * (hi - lo)


def test_step_target_is_confined_by_shrinkage():
    """Flat below lambda* and falling by 60 dex per dex above it (dN/dlambda):
    the draws stay within 0.1 dex of lambda* (density 1e-6 there) and are
    uniform in lambda below it; about 1.9% of the mass lies above lambda*."""
    p = oracle.pdf_params(0, 1, u_min=-2.0, u_max=0.0, u_star=-1.0, d1=0.0, d2=60.0)
    lam = oracle.pdf_slice(p, 20000, 1000, 100, seed=3, curve_id=0)
    assert np.all(np.log10(lam) < -1.0 + 0.1)
    above = np.mean(lam > 0.1)
    assert abs(above - 0.1 / 59 / (0.09 + 0.1 / 59)) < 0.005
    lo, hi = 10.0 ** -2.0, 10.0 ** -1.0
    assert stats.kstest(lam[lam < hi], "uniform", args=(lo, hi - lo)).pvalue > 1e-3


def test_chains_do_not_depend_on_n():
    p = oracle.pdf_params(1, 0)
    a = oracle.pdf_slice(p, 1000, 64, 10, seed=1)
    b = oracle.pdf_slice(p, 333, 64, 10, seed=1)
    assert np.array_equal(a[:333], b)
    c = oracle.pdf_slice(p, 333, 64, 10, seed=2)
    assert not np.array_equal(b, c)


def test_slice_rejects_bad_input():
    p = oracle.pdf_params(1, 0)
    for kw in [dict(n_chains=0, burn=0), dict(n_chains=4, burn=-1)]:
        with pytest.raises(oracle.OracleError):
            oracle.pdf_slice(p, 10, kw["n_chains"], kw["burn"], 0)
    with pytest.raises(oracle.OracleError):
        oracle.pdf_slice(oracle.pdf_params(2, sigma=0.0), 10, 4, 0, 0)
