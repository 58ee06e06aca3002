"""Phase-space adaptation with the gradient kernel (GPU).

Training the map of the uniforms through MEWeight (RAMBO + SIGMAKIN
forward, the gradient kernel backward) must change the sampling and not the
integral: the adapted and flat estimates of <w |M|^2> agree within their
errors.  For g g -> t t~ the coupling flow, sampled as a defensive mixture
with 10 % flat points (without it a rare starved region can blow up one
weight), cuts the relative variance of the weights several-fold; for g g -> t t~ g (gluon pT > 50 GeV, so that the
integral is finite) the separable warp lowers the training loss and the
variance of the bulk of the weights (capped at the flat sample's 99.9 %
quantile).  Training batches and estimates use disjoint Philox streams."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


def _agree(res):
    f, a = res['flat'], res['adapted']
    say('flat', f, 'adapted', a, 'variance reduction', res['variance_reduction'],
        'capped', res['capped_variance_reduction'])
    assert abs(f['mean'] - a['mean']) <= 4 * (f['error'] ** 2 + a['error'] ** 2) ** 0.5


def test_adaptation_ggtt_coupling_flow():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as mg
    from paper_2106_12631_amd import adapt
    torch.manual_seed(0)
    e = mg.MEEngine('ggtt')
    res = adapt.adapt_process(e, seed=4, iters=200, batch=1 << 14, nbins=16, lr=0.01,
                              eval_batch=1 << 18, clip=1.0, flow='coupling', mix=0.1, log=say)
    _agree(res)
    assert res['variance_reduction'] > 2.0


def test_adaptation_ggttg_cut_warp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as mg
    from paper_2106_12631_amd import adapt
    torch.manual_seed(0)
    e = mg.MEEngine('ggttg')
    cut = adapt.pt_cut(e, [4], 50.0)
    res = adapt.adapt_process(e, seed=4, iters=200, batch=1 << 14, nbins=32, lr=0.02,
                              eval_batch=1 << 18, clip=0.999, cut=cut, log=say)
    _agree(res)
    h = res['loss_history']
    assert sum(h[-10:]) < sum(h[:10])
    assert res['capped_variance_reduction'] > 1.0
