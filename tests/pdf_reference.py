"""Densities of the PDF draw restated from the paper for the tests, with
quadrature CDFs from scipy (QUADPACK): independent of both the oracle and the
HIP library.  Parameter objects are anything with the fields kind, measure,
u_min, u_max, u_star, d1, d2, sigma."""
import math

from scipy import integrate


def shape_u(p, u):
    """Density of u = log10(lambda) up to a constant: the sharp broken power
    law (kind 0), Eq. 1 (kind 1), Eq. 2 (kind 2); read as dN/dlambda
    (measure 1) the density in u gains a factor lambda."""
    x = u - p.u_star
    if p.kind == 0:
        f = 10.0 ** (-(p.d1 if x < 0 else p.d2) * x)
    elif p.kind == 1:
        f = 1.0 / ((10.0 ** x) ** p.d1 + (10.0 ** x) ** p.d2)
    else:
        f = math.exp(-x * x / (2.0 * p.sigma ** 2))
    return f * (10.0 ** x if p.measure == 1 else 1.0)


def _mass(p, a, b):
    pts = [p.u_star] if a < p.u_star < b else None
    return integrate.quad(lambda t: shape_u(p, t), a, b, epsabs=0, epsrel=1e-13, limit=400, points=pts)[0]


def quad_cdf(p):
    """u -> CDF(u) on [u_min, u_max]."""
    tot = _mass(p, p.u_min, p.u_max)
    return lambda u: _mass(p, p.u_min, u) / tot


def density(p):
    """u -> normalised density of u (per dex)."""
    tot = _mass(p, p.u_min, p.u_max)
    return lambda u: shape_u(p, u) / tot
