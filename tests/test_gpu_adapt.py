"""Phase-space adaptation with the gradient kernel (GPU): for g g -> t t~ g,
training the uniform warp through MEWeight (RAMBO + SIGMAKIN forward, the
gradient kernel backward) lowers the training loss and the relative
variance of the (capped) event weights, and the adapted and flat estimates
of <w |M|^2> agree within their errors (the map changes the sampling, not
the integral).  The raw variance reduction is reported, not asserted: it is
dominated by a handful of extreme weights at this sample size."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


def test_adaptation_ggttg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as mg
    from paper_2106_12631_amd import adapt
    e = mg.MEEngine('ggttg')
    res = adapt.adapt_process(e, seed=4, iters=60, batch=1 << 13, eval_batch=1 << 16, log=say)
    f, a = res['flat'], res['adapted']
    say('flat', f, 'adapted', a, 'variance reduction', res['variance_reduction'])
    h = res['loss_history']
    assert sum(h[-10:]) < sum(h[:10])
    assert res['capped_variance_reduction'] > 1.0
    assert abs(f['mean'] - a['mean']) <= 4 * (f['error'] ** 2 + a['error'] ** 2) ** 0.5
