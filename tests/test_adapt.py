"""The phase-space adaptation map and its training loop (CPU, torch).

* the warp is the identity for zero logits, monotone, maps (0,1) into (0,1),
  and its Jacobian equals the product of the finite-difference derivatives;
* for a separable peaked integrand with a known integral, training reduces
  the relative second moment by a large factor and the adapted estimate of
  the integral stays within four standard errors of the exact value;
* the coupling flow starts as the identity, its Jacobian equals the
  determinant of the autograd Jacobian matrix, and on a ridge along the
  diagonal (not separable: the separable warp gains nothing there) it
  reduces the relative second moment by a large factor, unbiased;
* both maps invert to rounding, with the same Jacobian, and the defensive
  mixture with the flat density keeps the estimate unbiased, still reduces
  the variance, and bounds every weight by f / mix.
"""
import math

import pytest
import torch

from paper_2106_12631_amd import adapt


def test_identity_and_jacobian():
    torch.manual_seed(0)
    m = adapt.WarpMap(3, 8)
    u = torch.rand(100, 3, dtype=torch.float64)
    x, jac = m(u)
    assert torch.allclose(x, u, rtol=0, atol=1e-15) and torch.allclose(jac, torch.ones(100, dtype=torch.float64))
    with torch.no_grad():
        m.logits.copy_(torch.randn(3, 8, dtype=torch.float64))
    x, jac = m(u)
    assert ((x > 0) & (x < 1)).all()
    us, _ = torch.sort(u[:, 0])
    xs, _ = m(torch.stack([us, us, us], -1))
    assert (xs[1:, 0] >= xs[:-1, 0]).all()
    h = 1e-7
    d = torch.ones(100, dtype=torch.float64)
    for k in range(3):
        up, um = u.clone(), u.clone()
        up[:, k] += h
        um[:, k] -= h
        d *= (m(up)[0][:, k] - m(um)[0][:, k]) / (2 * h)
    inside = ((u * 8 - (u * 8).round()).abs() > 1e-5).all(-1)   # away from bin edges
    assert torch.allclose(jac[inside], d[inside], rtol=1e-6)


def test_training_reduces_variance_and_stays_unbiased():
    torch.manual_seed(1)
    ndim, s0, c = 2, 0.05, 0.01
    norm1 = s0 * math.sqrt(2 * math.pi) * (0.5 * (math.erf(0.7 / (s0 * math.sqrt(2)))
                                                  + math.erf(0.3 / (s0 * math.sqrt(2))))) + c
    exact = norm1 ** ndim

    def fn(x):
        return (torch.exp(-(x - 0.3) ** 2 / (2 * s0 * s0)) + c).prod(-1)

    gen = torch.Generator().manual_seed(5)

    def uniforms(i, n):
        return torch.rand(n, ndim, dtype=torch.float64, generator=gen)

    m, hist = adapt.train(fn, ndim, uniforms, iters=150, batch=4096, nbins=32, lr=0.1)
    u = torch.rand(1 << 16, ndim, dtype=torch.float64, generator=gen)
    flat = adapt.estimate(fn(u))
    with torch.no_grad():
        x, jac = m(u)
    ad = adapt.estimate(fn(x) * jac)
    assert flat[2] / ad[2] > 20
    assert abs(ad[0] - exact) <= 4 * ad[1]
    assert abs(flat[0] - exact) <= 4 * flat[1]
    assert hist[-1] < 0.2 * hist[0]


def test_coupling_flow_identity_and_jacobian():
    torch.manual_seed(2)
    f = adapt.CouplingFlow(5, 8, hidden=16)
    u = torch.rand(20, 5, dtype=torch.float64)
    x, jac = f(u)
    assert torch.equal(x, u.clamp(torch.finfo(u.dtype).eps, 1 - torch.finfo(u.dtype).eps))
    assert torch.equal(jac, torch.ones(20, dtype=torch.float64))
    ib_all = sorted({d for _, ib in f.masks for d in ib})
    assert ib_all == list(range(5))
    with torch.no_grad():
        for p in f.parameters():
            p.add_(0.3 * torch.randn_like(p))
    x, jac = f(u)
    assert ((x > 0) & (x < 1)).all()
    for i in range(5):
        J = torch.autograd.functional.jacobian(lambda v: f(v.unsqueeze(0))[0].squeeze(0), u[i])
        assert abs(float(torch.det(J)) / float(jac[i].detach()) - 1) < 1e-10


def test_coupling_flow_follows_a_correlated_integrand():
    torch.manual_seed(1)
    s0, c = 0.05, 0.01
    # int_0^1 int_0^1 exp(-(x - y)^2 / (2 s0^2)) dx dy = int_{-1}^{1} (1 - |d|) exp(-d^2/(2 s0^2)) dd
    exact = (s0 * math.sqrt(2 * math.pi) * math.erf(1 / (s0 * math.sqrt(2)))
             - 2 * s0 * s0 * (1 - math.exp(-1 / (2 * s0 * s0)))) + c

    def fn(x):
        return torch.exp(-(x[:, 0] - x[:, 1]) ** 2 / (2 * s0 * s0)) + c

    gen = torch.Generator().manual_seed(5)

    def uniforms(i, n):
        return torch.rand(n, 2, dtype=torch.float64, generator=gen)

    u = torch.rand(1 << 16, 2, dtype=torch.float64, generator=gen)
    flat = adapt.estimate(fn(u))
    res = {}
    for flow in ('warp', 'coupling'):
        m, _ = adapt.train(fn, 2, uniforms, iters=80, batch=2048, nbins=16, lr=0.03, flow=flow,
                           clip=1.0)
        with torch.no_grad():
            x, jac = m(u)
        res[flow] = adapt.estimate(fn(x) * jac)
    assert flat[2] / res['warp'][2] < 1.5
    assert flat[2] / res['coupling'][2] > 8
    assert abs(res['coupling'][0] - exact) <= 4 * res['coupling'][1]
    assert abs(flat[0] - exact) <= 4 * flat[1]


def test_inverse_and_defensive_mixture():
    torch.manual_seed(3)
    for m in (adapt.WarpMap(4, 8, floor=0.1), adapt.CouplingFlow(4, 8, hidden=16, floor=0.05)):
        with torch.no_grad():
            for p in m.parameters():
                p.add_(0.5 * torch.randn_like(p))
        u = torch.rand(500, 4, dtype=torch.float64)
        x, jac = m(u)
        u2, jac2 = m.inverse(x)
        assert torch.allclose(u2, u, rtol=0, atol=1e-11)
        assert torch.allclose(jac2, jac, rtol=1e-11, atol=0)

    s0, c, mix = 0.05, 0.01, 0.2
    exact = (s0 * math.sqrt(2 * math.pi) * math.erf(1 / (s0 * math.sqrt(2)))
             - 2 * s0 * s0 * (1 - math.exp(-1 / (2 * s0 * s0)))) + c

    def fn(x):
        return torch.exp(-(x[:, 0] - x[:, 1]) ** 2 / (2 * s0 * s0)) + c

    gen = torch.Generator().manual_seed(5)

    def uniforms(i, n):
        return torch.rand(n, 2, dtype=torch.float64, generator=gen)

    u = torch.rand(1 << 16, 2, dtype=torch.float64, generator=gen)
    flat = adapt.estimate(fn(u))
    m, _ = adapt.train(fn, 2, uniforms, iters=80, batch=2048, nbins=16, lr=0.03, flow='coupling',
                       clip=1.0, mix=mix)
    with torch.no_grad():
        F = adapt.sample_weights(m, fn, u, mix)
    ad = adapt.estimate(F)
    assert flat[2] / ad[2] > 4
    assert abs(ad[0] - exact) <= 4 * ad[1]
    assert float(F.max()) <= (1 + c) / mix * (1 + 1e-12)
