"""Oracle cross section and hit-or-miss unweighting against closed forms
and exact statistics (CPU).

* e+e- -> mu+mu- at sqrt(s) = 1500 GeV: the Monte Carlo cross section from
  oracle events (RAMBO weights x matrix elements) agrees with the integral
  of the textbook |M|^2(cos theta) (Gauss-Legendre, exact for a quadratic)
  within four standard errors;
* the flux and phase-space factors: for |M|^2 = 1 the two-body estimate is
  the exact (hbar c)^2 / (2 s) / (8 pi);
* unweighting keeps exactly the events with u_i fmax < f_i, the number kept
  agrees with sum f / fmax within four binomial standard deviations, and the
  unweighting uniforms are uniform and uncorrelated with the sampler's.
"""
import math

import numpy as np
import pytest
import torch

import closed_forms as cf
from oracle import integrate, me, philox
from oracle.params import DEFAULT


def _sigma_eemumu_exact():
    s = DEFAULT.sqrts ** 2
    x, wq = np.polynomial.legendre.leggauss(8)
    E = DEFAULT.sqrts / 2
    p = np.zeros((x.size, 4, 4))
    p[:, 0] = [E, 0, 0, E]
    p[:, 1] = [E, 0, 0, -E]
    st = np.sqrt(1 - x * x)
    p[:, 3] = np.stack([np.full_like(x, E), E * st, 0 * x, E * x], -1)
    p[:, 2] = np.stack([np.full_like(x, E), -E * st, 0 * x, -E * x], -1)
    m2 = cf.eemumu(p, DEFAULT.alpha_inv, DEFAULT.mZ, DEFAULT.wZ, DEFAULT.sw2)
    # dsigma/dcos = (hbar c)^2 / (2 s) * |M|^2 / (16 pi) (two-body massless, phi integrated)
    return integrate.HBARC2_PB / (2 * s) / (16 * math.pi) * float((wq * m2).sum())


def test_eemumu_cross_section_matches_closed_form():
    n = 4096
    _, p, w = me.sample('eemumu', 0, 0, n)
    f = (me.matrix_element('eemumu', p) * w).numpy()
    sig, err = integrate.xsec(integrate.stats(f), n, DEFAULT.sqrts, 2)
    exact = _sigma_eemumu_exact()
    assert err / sig < 0.02
    assert abs(sig - exact) <= 4 * err


def test_flux_and_phase_space_factors():
    n = 64
    _, _, w = me.sample('eemumu', 0, 0, n)
    sig, err = integrate.xsec(integrate.stats(w.numpy()), n, DEFAULT.sqrts, 2)
    s = DEFAULT.sqrts ** 2
    assert sig == pytest.approx(integrate.HBARC2_PB / (2 * s) / (8 * math.pi), rel=1e-14)
    # one-pass variance of equal weights: cancellation leaves ~sqrt(eps) of the mean
    assert err <= 1e-7 * sig


def test_stats_skip_nonfinite():
    f = np.array([1.0, np.nan, 3.0, np.inf, -np.inf, 2.0])
    assert integrate.stats(f) == (6.0, 14.0, 3.0, 3.0)
    assert integrate.stats(np.array([np.nan])) == (0.0, 0.0, 0.0, 0.0)


def test_unweighting_rule_and_acceptance():
    rng = np.random.default_rng(11)
    n = 20000
    f = rng.random(n) ** 3
    fmax = 1.0
    kept = integrate.unweight(f, fmax, seed=5, evt_offset=100)
    u = integrate.unweight_uniforms(5, 100, n)
    mask = np.zeros(n, bool)
    mask[kept] = True
    assert np.all(np.diff(kept) > 0)
    assert np.all(u[mask] * fmax < f[mask]) and np.all(u[~mask] * fmax >= f[~mask])
    expect = f.sum() / fmax
    sd = math.sqrt((f / fmax * (1 - f / fmax)).sum())
    assert abs(kept.size - expect) <= 4 * sd
    # NaN is never kept; fmax = 0 keeps every positive f
    g = np.array([np.nan, 0.5, 0.0, -1.0])
    assert list(integrate.unweight(g, 0.0, 1)) == [1]


def test_unweighting_uniforms():
    n = 50000
    u = integrate.unweight_uniforms(3, 0, n)
    assert (u > 0).all() and (u < 1).all()
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
    ks = np.abs(np.sort(u) - (np.arange(n) + 0.5) / n).max()
    assert ks < 1.63 / math.sqrt(n)
    # distinct from every sampler slot drawn with the same seed
    r = philox.uniforms(3, 0, n, 16)
    for k in range(16):
        assert abs(np.corrcoef(u, r[:, k])[0, 1]) < 4 / math.sqrt(n)
    # depends only on the global event index
    assert np.array_equal(integrate.unweight_uniforms(3, 17, 5), u[17:22])
