"""Precision guard of the reduced-precision forms (GPU).

After an FP32-amplitude or mixed-precision launch, the events whose |M|^2
is ill-conditioned in its invariants (kappa = s / min |2 p_i.p_j| above
1e4, reading R26) are recomputed in FP64.  The events are chosen on the
CPU from the oracle's momenta: the most ill-conditioned ones among the
first 2^17 events of the g g -> t t~ g and g g -> t t~ g g workloads, plus
a seeded sample of ordinary ones.  Checks:
* the guard changes exactly the events with kappa > 1e4 (the others are
  bitwise those of the unguarded launch) and gives them the FP64 path's
  result (1e-13);
* against the oracle: 1e-12 + 8 eps kappa on the recomputed events, 1e-5
  on all events (the unguarded maximum is printed beside it).
"""
import sys

import pytest
import torch

from oracle import me as orc
from rounding import EPS, invariant_condition

pytestmark = pytest.mark.gpu
KMAX = 1.0e4


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


_EVENTS = {}


def events(proc, seed):
    """Oracle momenta and |M|^2 of the 24 most ill-conditioned of the first
    2^17 events and of 40 seeded others."""
    if proc not in _EVENTS:
        _, p, _ = orc.sample(proc, seed, 0, 1 << 17)
        k = invariant_condition(p)
        worst = torch.argsort(k, descending=True)[:24]
        g = torch.Generator().manual_seed(seed)
        others = torch.randint(0, 1 << 17, (40,), generator=g)
        idx = torch.cat([worst, others])
        ps = p[idx].contiguous()
        _EVENTS[proc] = (ps, k[idx], orc.matrix_element(proc, ps))
    return _EVENTS[proc]


@pytest.mark.parametrize('proc,seed,prec', [('ggttg', 2, 'mixed'), ('ggttgg', 3, 'mixed'),
                                            ('ggttgg', 3, 'fp32amp')])
def test_guard_recomputes_ill_conditioned_events(mg, proc, seed, prec):
    p, kappa, want = events(proc, seed)
    n = p.shape[0]
    say('guard', proc, prec, n, 'max kappa', float(kappa.max()))
    guarded = mg.MEEngine(proc, prec)
    plain = mg.MEEngine(proc, prec, params={'flags': mg.FLAG_NO_PRECISION_GUARD})
    e64 = mg.MEEngine(proc, 'fp64')
    mom = guarded.events_mom(p)
    g = guarded.sigmakin(mom, n).cpu()
    u = plain.sigmakin(mom, n).cpu()
    f = e64.sigmakin(mom, n).cpu()
    flagged = kappa > KMAX
    assert int(flagged.sum()) >= 8
    assert torch.equal(g[~flagged], u[~flagged])
    assert float(((g[flagged] - f[flagged]).abs() / f[flagged]).max()) <= 1e-13
    err_g = (g - want).abs() / want
    err_u = (u - want).abs() / want
    say(proc, prec, 'guarded max rel', float(err_g.max()), 'unguarded max rel', float(err_u.max()),
        'flagged', int(flagged.sum()))
    assert bool((err_g[flagged] <= 1e-12 + 8 * EPS * kappa[flagged]).all())
    assert float(err_g.max()) <= 1e-5
    # evtw of the recomputed events follows me
    w = torch.linspace(0.5, 1.5, n, dtype=torch.float64, device=guarded.device)
    me2, evtw = guarded.sigmakin(mom, n, wgt=w)
    assert torch.equal(evtw, me2 * w)
