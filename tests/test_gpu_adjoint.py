"""Gradient kernel (mg_adjoint) against the oracle's reverse-mode gradient
and central finite differences (GPU).

f(r) = w(r) |M|^2(p(r)) per event, differentiated with respect to the 12
uniforms of g g -> t t~ g (the gradient workload: seed 4, 2^18 events, the
finite-difference check on the first 1024 events, h = 1e-6).
Tolerances:
* f = w |M|^2 vs the oracle: each side computes its own momenta, so the
  end-to-end bound of the parity tests applies (1e-11), plus the weight
  bound of tests/rounding.py;
* FP64 gradient vs the oracle's autograd gradient, per event normwise:
  1e-10 plus 64 eps gamma^2 (momentum rounding is of order eps gamma and
  the derivative of the boost adds a factor gamma); d log w / dr (dimensionless) normwise relative to
  max(|d log w / dr|, 1), since the weight is constant for massless and for
  two-body final states and both sides then hold rounding noise only;
* FP64 gradient vs central differences with step h (fourth-order stencil):
  1e-6 normwise (truncation ~h^4 f^(5), rounding ~eps f / h), events with a
  uniform within 10 h of 0 or 1 excluded and counted;
* FP32-amplitude gradient vs the FP64 one: max and median reported; the
  median must stay below 1e-5.
"""
import math
import sys

import pytest
import torch

from oracle import me as orc
from rounding import EPS, boost_gamma, weight_bound

pytestmark = pytest.mark.gpu
SEED = 4


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as m
    m.lib()
    return m


_ENG = {}


def engine(mg, proc, prec='fp64'):
    if (proc, prec) not in _ENG:
        say('create', proc, prec)
        _ENG[(proc, prec)] = mg.MEEngine(proc, prec)
    return _ENG[(proc, prec)]


def normwise(a, b):
    return (a - b).norm(dim=1) / b.norm(dim=1)


def normwise_unit(a, b):
    return (a - b).norm(dim=1) / b.norm(dim=1).clamp_min(1.0)


@pytest.mark.parametrize('proc,n', [('ggttg', 256 + 9), ('ggtt', 512 + 3), ('eemumu', 512 + 3)])
def test_gradient_vs_oracle_autograd(mg, proc, n):
    e = engine(mg, proc)
    r, p_orc, _ = orc.sample(proc, SEED, 0, n)
    f_orc, g_orc, gw_orc = orc.event_weight_and_grad(proc, r)
    say('adjoint fp64', proc, n)
    grad, glogw, f = e.adjoint(e.events_rnd(r), n)
    g = e.rnd_events(grad, n).cpu()
    gw = e.rnd_events(glogw, n).cpu()
    ferr = float(((f.cpu() - f_orc).abs() / f_orc.abs()).max())
    gerr = normwise(g, g_orc)
    werr = normwise_unit(gw, gw_orc)
    say(proc, 'f rel', ferr, 'grad max', float(gerr.max()), 'median', float(gerr.median()),
        'logw max', float(werr.max()))
    gam = boost_gamma(r)
    frel = (f.cpu() - f_orc).abs() / f_orc.abs()
    assert (frel <= 1e-11 + weight_bound(r, p_orc, 1500.0)).all()
    gtol = 1e-10 + 64 * EPS * gam ** 2
    assert (gerr <= gtol).all()
    assert (werr <= gtol).all()
    # gbar scales each event's gradient
    gbar = torch.linspace(0.5, 2.0, n, dtype=torch.float64, device=e.device)
    grad2, _, _ = e.adjoint(e.events_rnd(r), n, gbar=gbar, want_logw=False, want_f=False)
    assert torch.allclose(e.rnd_events(grad2, n).cpu(), g * gbar.cpu()[:, None], rtol=1e-15,
                          atol=0)


def _fd_gradient(e, r, h):
    """Central differences of f = w |M|^2 with the FP64 RAMBO and SIGMAKIN
    kernels, fourth-order stencil on f(r -+ 2h), f(r -+ h).  The two-point
    difference carries a truncation error h^2 f'''/6 that reaches 3e-5
    relative on events with a nearly collinear gluon; this one's is O(h^4)."""
    n, nr = r.shape
    out = torch.zeros(n, nr, dtype=torch.float64)
    for j in range(nr):
        vals = {}
        for s in (-2, -1, 1, 2):
            rr = r.clone()
            rr[:, j] += s * h
            mom, wgt = e.rambo(e.events_rnd(rr), n)
            _, evtw = e.sigmakin(mom, n, wgt=wgt)
            vals[s] = evtw.cpu()
        out[:, j] = (vals[-2] - 8 * vals[-1] + 8 * vals[1] - vals[2]) / (12 * h)
    return out


def test_gradient_vs_finite_differences(mg):
    e = engine(mg, 'ggttg')
    n, h = 1024, 1e-6
    r, _, _ = orc.sample('ggttg', SEED, 0, n)
    say('adjoint vs FD', n)
    grad, _, _ = e.adjoint(e.events_rnd(r), n, want_logw=False, want_f=False)
    g = e.rnd_events(grad, n).cpu()
    fd = _fd_gradient(e, r, h)
    edge = ((r < 10 * h) | (r > 1 - 10 * h)).any(dim=1)
    err = normwise(g, fd)[~edge]
    say('FD check: events', int((~edge).sum()), 'excluded near 0/1', int(edge.sum()),
        'max', float(err.max()), 'median', float(err.median()))
    assert float(err.max()) <= 1e-6


def test_gradient_mixed_vs_fp64(mg):
    e64 = engine(mg, 'ggttg')
    e32 = engine(mg, 'ggttg', 'fp32amp')
    n = 640 + 5
    r, _, _ = orc.sample('ggttg', SEED, 0, n)
    say('adjoint mixed', n)
    g64 = e64.rnd_events(e64.adjoint(e64.events_rnd(r), n)[0], n).cpu()
    g32, _, f32 = e32.adjoint(e32.events_rnd(r), n)
    g32 = e32.rnd_events(g32, n).cpu()
    err = normwise(g32, g64)
    say('mixed gradient vs fp64: max', float(err.max()), 'median', float(err.median()))
    assert e32.count_nonfinite(f32) == 0
    assert float(err.median()) <= 1e-5
    assert float(err.max()) <= 1e-3


def test_autograd_function(mg):
    e = engine(mg, 'ggttg')
    n = 130
    r, _, _ = orc.sample('ggttg', SEED, 0, n)
    rd = r.to(e.device).requires_grad_(True)
    y = e.event_weight(rd)
    c = torch.linspace(-1.0, 1.0, n, dtype=torch.float64, device=e.device)
    (y * c).sum().backward()
    f_orc, g_orc, _ = orc.event_weight_and_grad('ggttg', r)
    assert float(((y.detach().cpu() - f_orc).abs() / f_orc.abs()).max()) <= 1e-12
    want = g_orc * c.cpu()[:, None]
    err = ((rd.grad.cpu() - want).norm(dim=1) / g_orc.norm(dim=1)).max()
    assert float(err) <= 1e-10


def test_gradient_full_size(mg):
    """The gradient workload at full size, sampled events against the oracle."""
    e = engine(mg, 'ggttg')
    n = 1 << 18
    say('adjoint full size', n)
    rnd = e.rng(SEED, n)
    grad, glogw, f = e.adjoint(rnd, n)
    torch.cuda.synchronize()
    assert e.count_nonfinite(grad) == 0 and e.count_nonfinite(f) == 0
    g = torch.Generator().manual_seed(SEED)
    idx = sorted(set([0, n - 1] + torch.randint(0, n, (14,), generator=g).tolist()))
    gg = e.rnd_events(grad, n)[idx].cpu()
    rs = torch.cat([orc.sample('ggttg', SEED, i, 1)[0] for i in idx])
    _, g_orc, _ = orc.event_weight_and_grad('ggttg', rs)
    assert (normwise(gg, g_orc) <= 1e-10 + 64 * EPS * boost_gamma(rs) ** 2).all()


def test_gradient_not_built_for_ggttgg(mg):
    e = engine(mg, 'ggttgg')
    rnd = e.rng(SEED, 64)
    with pytest.raises(RuntimeError, match='not supported'):
        e.adjoint(rnd, 64)
