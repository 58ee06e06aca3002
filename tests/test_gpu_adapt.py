"""Phase-space adaptation with the gradient kernel (GPU).

* Parity: for a trained map g, the adapted weights F(u) = f(g(u)) |g'(u)|
  of the GPU path (f = w |M|^2 from the RAMBO and SIGMAKIN kernels, df/dx
  from the gradient kernel) agree with the same map evaluated on the CPU
  around the FP64 oracle's f and its autograd gradient: the mapped points
  and Jacobians to rounding, f at the same points within the end-to-end
  bound of the parity tests, and the gradient of the training loss with
  respect to every map parameter.
* Reproducibility: the bin lookups of the maps reduce in a fixed order and
  the kernels use no atomics, so two trainings from the same seeds give the
  same parameters bit for bit.
* Adaptation: training must change the sampling and not the integral (the
  adapted and flat estimates of <w |M|^2> agree within their errors).  For
  g g -> t t~ the coupling flow, sampled as a defensive mixture with 10 %
  flat points, cuts the relative variance of the weights several-fold; for
  g g -> t t~ g (gluon pT > 50 GeV, so that the integral is finite) the
  separable warp lowers the training loss and the variance of the bulk of
  the weights (capped at the flat sample's 99.9 % quantile).  Training
  batches and estimates use disjoint Philox streams; the thresholds hold for
  the fixed seeds with the margins stated below.
"""
import copy
import sys

import pytest
import torch

from oracle import me as orc
from rounding import end_to_end_bound, weight_bound

pytestmark = pytest.mark.gpu


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


class OracleWeight(torch.autograd.Function):
    """f(r) = w |M|^2 by the FP64 oracle on the CPU, with its autograd
    gradient as the backward pass."""

    @staticmethod
    def forward(ctx, r, proc):
        with torch.enable_grad():  # the oracle differentiates itself by autograd
            f, g, _ = orc.event_weight_and_grad(proc, r.detach())
        ctx.save_for_backward(g)
        return f

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout[:, None] * g, None


def _train(mg, adapt, proc, flow, iters, seed=4, batch=1 << 12):
    torch.manual_seed(0)
    e = mg.MEEngine(proc)
    nr = e.layout.nrnd

    def uniforms(i, n):
        return e.rnd_events(e.rng(seed, n, offset=i * n), n)

    m, hist = adapt.train(e.event_weight, nr, uniforms, iters=iters, batch=batch, nbins=16,
                          lr=0.01, device=e.device, clip=1.0, flow=flow, mix=0.1)
    return e, m, hist


@pytest.mark.parametrize('proc,flow', [('ggtt', 'coupling'), ('ggttg', 'warp')])
def test_adapted_weights_vs_oracle(mg, proc, flow):
    from paper_2106_12631_amd import adapt
    e, m, _ = _train(mg, adapt, proc, flow, iters=20)
    n = 300
    u = orc.sample(proc, 9, 0, n)[0]
    say('adapted weights vs oracle', proc, flow, n)
    # the map on both devices: points and Jacobians agree to rounding
    with torch.no_grad():
        xg, jg = m(u.to(e.device))
        mc = copy.deepcopy(m).to('cpu')
        xc, jc = mc(u)
    assert float((xg.cpu() - xc).abs().max()) <= 1e-13
    assert float(((jg.cpu() - jc).abs() / jc).max()) <= 1e-12
    # f at the same points: GPU kernels against the oracle, end to end
    x = xg.cpu()
    with torch.no_grad():
        fg = e.event_weight(xg).cpu()
    p, _ = orc.phase_space(proc, x)
    f_orc = OracleWeight.apply(x, proc)
    rel = (fg - f_orc).abs() / f_orc
    bound = end_to_end_bound(x, p) + weight_bound(x, p, 1500.0)
    say(proc, 'f(g(u)) max rel', float(rel.max()), 'max rel / bound', float((rel / bound).max()))
    assert bool((rel <= bound).all())
    # the training loss and its gradient with respect to every map parameter
    ug = u.to(e.device)
    Fg = adapt.sample_weights(m, e.event_weight, ug, mix=0.1)
    Lg = adapt.relative_second_moment(Fg)
    gg = torch.autograd.grad(Lg, list(m.parameters()))
    Fc = adapt.sample_weights(mc, lambda xx: OracleWeight.apply(xx, proc), u, mix=0.1)
    Lc = adapt.relative_second_moment(Fc)
    gc = torch.autograd.grad(Lc, list(mc.parameters()))
    Frel = (Fg.detach().cpu() - Fc.detach()).abs() / Fc.detach()
    num = sum(float(((a.cpu() - b) ** 2).sum()) for a, b in zip(gg, gc)) ** 0.5
    den = sum(float((b ** 2).sum()) for b in gc) ** 0.5
    say(proc, 'F max rel', float(Frel.max()), 'loss rel', abs(float(Lg.detach()) / float(Lc.detach()) - 1),
        'loss gradient normwise', num / den)
    assert float(Frel.max()) <= 1e-10
    assert abs(float(Lg) / float(Lc) - 1) <= 1e-10
    assert num / den <= 1e-8


def test_training_is_reproducible(mg):
    from paper_2106_12631_amd import adapt
    _, m1, h1 = _train(mg, adapt, 'ggtt', 'coupling', iters=15)
    _, m2, h2 = _train(mg, adapt, 'ggtt', 'coupling', iters=15)
    say('reproducibility: losses', h1[-1], h2[-1])
    assert h1 == h2
    for a, b in zip(m1.parameters(), m2.parameters()):
        assert torch.equal(a, b)


def _agree(res):
    f, a = res['flat'], res['adapted']
    say('flat', f, 'adapted', a, 'variance reduction', res['variance_reduction'],
        'capped', res['capped_variance_reduction'])
    assert abs(f['mean'] - a['mean']) <= 4 * (f['error'] ** 2 + a['error'] ** 2) ** 0.5


def test_adaptation_ggtt_coupling_flow(mg):
    from paper_2106_12631_amd import adapt
    torch.manual_seed(0)
    e = mg.MEEngine('ggtt')
    res = adapt.adapt_process(e, seed=4, iters=200, batch=1 << 14, nbins=16, lr=0.003,
                              eval_batch=1 << 18, clip=0.995, flow='coupling', mix=0.1, log=say)
    _agree(res)
    # 10.4x to 10.7x over training seeds 4, 6, 8: the loss on weights capped
    # at the batch's 99.5 % quantile keeps rare large weights from steering
    # the training (uncapped: 1.2x to 9.6x)
    assert res['variance_reduction'] > 4.0


def test_adaptation_ggttg_cut_warp(mg):
    from paper_2106_12631_amd import adapt
    torch.manual_seed(0)
    e = mg.MEEngine('ggttg')
    cut = adapt.pt_cut(e, [4], 50.0)
    res = adapt.adapt_process(e, seed=4, iters=200, batch=1 << 14, nbins=32, lr=0.02,
                              eval_batch=1 << 18, clip=0.999, cut=cut, log=say)
    _agree(res)
    h = res['loss_history']
    assert sum(h[-10:]) < sum(h[:10])
    # capped: 1.53x to 1.58x over training seeds 4, 6, 8
    assert res['capped_variance_reduction'] > 1.2
