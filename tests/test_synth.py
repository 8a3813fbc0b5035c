"""Checks of the seeded input generators (harness side, not the method)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_1909_06374_amd import synth


def test_erdf_masses_match_numerical_integral():
    pdf = lambda u: 10 ** (-0.4 * (u + 1.5)) if u < -1.5 else 10 ** (-2.5 * (u + 1.5))
    m1 = integrate.quad(pdf, -4, -1.5)[0]
    m2 = integrate.quad(pdf, -1.5, 0)[0]
    a, b = synth.erdf_bpl_masses()
    assert a == pytest.approx(m1, rel=1e-12) and b == pytest.approx(m2, rel=1e-12)
    assert a / (a + b) == pytest.approx(0.98254, abs=5e-6)


def test_erdf_inverse_cdf():
    assert synth.erdf_bpl_u_from_uniform(np.array([0.0]))[0] == pytest.approx(-4.0)
    assert synth.erdf_bpl_u_from_uniform(np.array([1.0]))[0] == pytest.approx(0.0, abs=1e-12)
    m1, m2 = synth.erdf_bpl_masses()
    assert synth.erdf_bpl_u_from_uniform(np.array([m1 / (m1 + m2)]))[0] == pytest.approx(-1.5)
    lam = synth.erdf_draw(200000, seed=4)
    u = np.log10(lam)
    assert stats.kstest(u, synth.erdf_bpl_cdf).pvalue > 1e-3
    assert np.all(lam > 0) and np.all(np.isfinite(lam))
    assert abs(np.mean(u < -1.5) - 0.98254) < 5 * math.sqrt(0.98254 * 0.01746 / len(u))


def test_draws_are_seeded():
    assert np.array_equal(synth.erdf_draw(100, 1, 2), synth.erdf_draw(100, 1, 2))
    assert not np.array_equal(synth.erdf_draw(100, 1, 2), synth.erdf_draw(100, 1, 3))


def test_size_grid():
    g = synth.size_grid(10, 20)
    assert len(g) == 21 and min(g) == 1024 and max(g) == 2**20
    assert sum(g) / 21 == pytest.approx(174641.5, abs=1)
    g4 = synth.size_grid(12, 22)
    assert len(g4) == 21 and sum(g4) / 21 == pytest.approx(698563, abs=1)


def test_golden_constants_file():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "erdf_bpl_constants.txt")
    vals = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    m1, m2 = synth.erdf_bpl_masses()
    assert m1 == pytest.approx(vals["M1"], abs=1e-6)
    assert m2 == pytest.approx(vals["M2"], abs=1e-6)
    assert m1 / (m1 + m2) == pytest.approx(vals["P_below_break"], abs=5e-6)
