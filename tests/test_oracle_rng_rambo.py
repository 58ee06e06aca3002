"""Pins for the oracle's random numbers and RAMBO sampler (CPU only)."""
import math
import os

import numpy as np
import pytest
import torch
from scipy import stats

import closed_forms as cf
from oracle import philox, rambo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[:4], v[4:6], v[6:]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        got = philox.philox4x32_10(np.array(ctr), np.array(key))
        assert [int(x) for x in got] == out


def test_bits_to_uniform_edges():
    assert philox.bits_to_uniform(0) == 2.0 ** -54
    assert philox.bits_to_uniform(2 ** 64 - 1) == 1.0 - 2.0 ** -54
    u = philox.bits_to_uniform(np.array([2 ** 63], dtype=np.uint64))
    assert u[0] == 0.5 + 2.0 ** -54


def test_uniforms_counter_based_and_open_interval():
    a = philox.uniforms(7, 0, 300, 12)
    b = philox.uniforms(7, 100, 200, 12)
    assert np.array_equal(a[100:], b)
    assert (a > 0).all() and (a < 1).all()
    # seeds differing only in the high word give different streams
    c = philox.uniforms(7 + (1 << 32), 0, 300, 12)
    assert not np.array_equal(a, c)


def test_uniforms_statistics():
    u = philox.uniforms(1, 0, 1 << 16, 16).ravel()
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / n)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # lag-1 correlation between successive slots of one event
    v = philox.uniforms(2, 0, 1 << 16, 16)
    rho = np.corrcoef(v[:, :-1].ravel(), v[:, 1:].ravel())[0, 1]
    assert abs(rho) < 5 / math.sqrt(v[:, 1:].size)


def _boost_gamma(r, n):
    """gamma = Q^0 / M of the boost RAMBO applies (recomputed from r)."""
    q0 = -torch.log(r[:, 2::4] * r[:, 3::4])
    c = 2 * r[:, 0::4] - 1
    ph = 2 * math.pi * r[:, 1::4]
    st = torch.sqrt(1 - c * c)
    q = torch.stack([q0, q0 * st * torch.cos(ph), q0 * st * torch.sin(ph), q0 * c], -1)
    Q = q.sum(1)
    return Q[:, 0] / torch.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(-1))


@pytest.mark.parametrize("n", [2, 3, 4])
def test_rambo_massless_conservation_and_weight(n):
    """Conservation and masslessness hold to rounding.  The boost to the
    rest frame of sum q cancels terms of size gamma = Q^0/M down to the
    result, so the bound is stated in units of eps gamma (the published
    evaluation of M and the boost would need eps gamma^2)."""
    sqrts = 1500.0
    eps = 2.0 ** -52
    r = torch.from_numpy(philox.uniforms(3, 0, 1 << 14, 4 * n))
    p, w0 = rambo.rambo_massless(r, sqrts, n)
    g = _boost_gamma(r, n)
    tot = p.sum(1)
    assert ((tot[:, 0] - sqrts).abs() / sqrts <= 8 * eps * g).all()
    assert (tot[:, 1:].abs().max(1).values / sqrts <= 8 * eps * g).all()
    m2 = p[..., 0] ** 2 - (p[..., 1:] ** 2).sum(-1)
    assert ((m2.abs() / (p[..., 0] ** 2)).max(1).values <= 16 * eps * g).all()
    # most events are not boosted much: there the error is a few ulps
    assert float((m2.abs() / (p[..., 0] ** 2)).median()) < 1e-15
    assert w0 == pytest.approx(cf.Rn_massless(n, sqrts ** 2), rel=1e-15)


def test_rambo_two_body_flat():
    r = torch.from_numpy(philox.uniforms(4, 0, 1 << 15, 8))
    p, _ = rambo.rambo_massless(r, 1500.0, 2)
    c = (p[:, 0, 3] / p[:, 0, 0]).numpy()
    ph = torch.atan2(p[:, 0, 2], p[:, 0, 1]).numpy()
    assert stats.kstest(c, stats.uniform(-1, 2).cdf).pvalue > 1e-4
    assert stats.kstest(ph, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 1e-4
    # back to back, each with sqrt(s)/2
    assert torch.allclose(p[:, 0, 0], torch.full_like(p[:, 0, 0], 750.0), atol=1e-10)


def test_rambo_three_body_dalitz_flat():
    # massless 3-body phase space is flat in (x1, x2): marginal of x1 is 2 x1
    r = torch.from_numpy(philox.uniforms(5, 0, 1 << 15, 12))
    p, _ = rambo.rambo_massless(r, 1500.0, 3)
    x1 = (2 * p[:, 0, 0] / 1500.0).numpy()
    assert stats.kstest(x1, lambda x: np.clip(x, 0, 1) ** 2).pvalue > 1e-4


def test_rambo_massive_two_body_weight():
    m = 173.0
    sqrts = 1500.0
    r = torch.from_numpy(philox.uniforms(6, 0, 512, 8))
    k, w = rambo.rambo_massive(r, sqrts, [m, m])
    beta = math.sqrt(1 - 4 * m * m / sqrts ** 2)
    g = _boost_gamma(r, 2)
    eps = 2.0 ** -52
    assert ((w / (math.pi / 2 * beta) - 1).abs() <= 8 * eps * g).all()
    assert float((w / (math.pi / 2 * beta) - 1).abs().median()) < 1e-15
    m2 = k[..., 0] ** 2 - (k[..., 1:] ** 2).sum(-1)
    assert ((m2 / (m * m) - 1).abs().max(1).values <= 8 * eps * g * (sqrts / m) ** 2).all()


@pytest.mark.parametrize("masses", [[173.0, 173.0, 0.0], [173.0, 173.0, 0.0, 0.0]])
def test_rambo_massive_on_shell_and_mean_weight(masses):
    n = len(masses)
    sqrts = 1500.0
    N = 1 << 17
    r = torch.from_numpy(philox.uniforms(11, 0, N, 4 * n))
    k, w = rambo.rambo_massive(r, sqrts, masses)
    m2 = k[..., 0] ** 2 - (k[..., 1:] ** 2).sum(-1)
    want = torch.tensor([m * m for m in masses], dtype=torch.float64)
    g = _boost_gamma(r, n)
    eps = 2.0 ** -52
    assert ((m2 - want).abs().max(1).values <= 16 * eps * g * k[..., 0].max(1).values ** 2).all()
    tot = k.sum(1)
    assert ((tot[:, 0] - sqrts).abs() <= 8 * eps * g * sqrts).all()
    assert (tot[:, 1:].abs().max(1).values <= 8 * eps * g * sqrts).all()
    # the RAMBO weight is an unbiased estimate of the phase-space volume
    R = cf.Rn(sqrts ** 2, masses)
    err = float(w.std()) / math.sqrt(N)
    assert abs(float(w.mean()) - R) < 5 * err


def test_rambo_no_phase_space():
    r = torch.from_numpy(philox.uniforms(1, 0, 4, 8))
    with pytest.raises(rambo.NoPhaseSpace):
        rambo.rambo_massive(r, 300.0, [173.0, 173.0])


def _published_boost_longdouble(r, n, sqrts):
    """RAMBO's massless step as published -- M = sqrt(Q^2), b = -Q/M,
    gamma = Q^0/M, a = 1/(1+gamma), x = sqrt(s)/M, p^0 = x(gamma q^0 + b.q),
    p = x(q + b q^0 + a (b.q) b) -- evaluated in 80-bit extended precision
    (64-bit significand), where its loss of ~gamma^2 in accuracy stays far
    below double rounding."""
    LD = np.longdouble
    pi = LD('3.14159265358979323846264338327950288')
    r = r.numpy().astype(LD)
    q = []
    for i in range(n):
        c = LD(2) * r[:, 4 * i] - LD(1)
        st = np.sqrt(LD(1) - c * c)
        ph = LD(2) * pi * r[:, 4 * i + 1]
        q0 = -np.log(r[:, 4 * i + 2] * r[:, 4 * i + 3])
        q.append(np.stack([q0, q0 * st * np.cos(ph), q0 * st * np.sin(ph), q0 * c], -1))
    q = np.stack(q, 1)
    Q = q.sum(1)
    M = np.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(-1))
    b = -Q[:, 1:] / M[:, None]
    gam = Q[:, 0] / M
    a = LD(1) / (LD(1) + gam)
    x = LD(sqrts) / M
    bq = (b[:, None, :] * q[:, :, 1:]).sum(-1)
    p0 = x[:, None] * (gam[:, None] * q[:, :, 0] + bq)
    pv = x[:, None, None] * (q[:, :, 1:] + b[:, None, :] * q[:, :, :1]
                             + a[:, None, None] * bq[:, :, None] * b[:, None, :])
    return np.concatenate([p0[:, :, None], pv], -1)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_rambo_boost_equals_published_form(n):
    """The oracle's boost (pairwise Minkowski products) is the published
    RAMBO boost: against that formula in extended precision it agrees to
    32 eps gamma sqrt(s) in every component (one rounding of the uniforms'
    angles and logarithms, amplified once by the boost), far inside the
    published form's own double-precision error (eps gamma^2)."""
    if np.finfo(np.longdouble).nmant < 60:
        pytest.skip("no extended-precision long double on this host")
    sqrts = 1500.0
    eps = 2.0 ** -52
    r = torch.from_numpy(philox.uniforms(12, 0, 1 << 14, 4 * n))
    p, _ = rambo.rambo_massless(r, sqrts, n)
    ref = torch.from_numpy(_published_boost_longdouble(r, n, sqrts).astype(np.float64))
    g = _boost_gamma(r, n)
    err = (p - ref).abs().amax(dim=(1, 2)) / sqrts
    assert (err <= 32 * eps * g).all()
    if n == 2:  # the sample holds strongly boosted events
        assert float(g.max()) > 100
