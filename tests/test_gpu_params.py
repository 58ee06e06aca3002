"""Parity away from the default parameters, through the C ABI (GPU).

Parameters reach the kernels by value (Sec. IV.c keeps them in constant
memory; here a kernel-argument struct per handle), so several handles with
different parameters can be alive and used in one process.  Covered:
* massless quarks (mt = 0) in g g -> q q~ g g: chirality makes half of the
  64 helicities exactly zero, so the helicity filter keeps 32 and the
  event-per-lane kernels run (FP64, FP32 amplitudes, BF16-split matrix-core
  colour sum) instead of the one-helicity-per-lane ones;
* a second parameter point (sqrt(s) = 1000, alpha_s = 0.13, zero top width);
* the flags: zero width in t- and u-channel top propagators (reading R5) and
  weights with (2 pi)^(4 - 3 n) (reading R10);
* two handles with different parameters used alternately.
Tolerances as in test_gpu_parity: 1e-12 relative for FP64 on identical
momenta, 1e-5 for the FP32-amplitude and mixed forms.  With massless quarks
a quark-gluon pair can be nearly collinear: a propagator invariant s_ij
formed from momentum components carries an absolute rounding error of order
eps s on each side, i.e. a relative error eps s / |s_ij| of the propagator,
so the FP64 bound there is 1e-12 + 8 eps s / min |s_ij| over the pairs of
external momenta (reading R26).
"""
import math
import sys

import pytest
import torch

from oracle import me as orc
from oracle.params import DEFAULT, TCHANNEL_ZERO_WIDTH, WEIGHT_2PI
from rounding import EPS, invariant_condition, momentum_bound, weight_bound

pytestmark = pytest.mark.gpu

N = {'eemumu': 1024 + 9, 'ggtt': 1024 + 9, 'ggttg': 256 + 9, 'ggttgg': 128 + 9}
SECOND = dict(sqrts=1000.0, alphas=0.13, wt=0.0)


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


def rel(a, b):
    return (a - b).abs() / b.abs()


_REF = {}


def reference(proc, seed, n, **prm):
    """Oracle uniforms, momenta, weights and |M|^2 at parameters prm."""
    key = (proc, seed, n, tuple(sorted(prm.items())))
    if key not in _REF:
        P = DEFAULT.with_(**prm)
        r, p, w = orc.sample(proc, seed, 0, n, prm=P)
        _REF[key] = (r, p, w, orc.matrix_element(proc, p, P))
    return _REF[key]


@pytest.mark.parametrize('prec,tol', [('fp64', 1e-12), ('fp32amp', 1e-5), ('mixed', 1e-5)])
def test_ggttgg_massless_quarks_event_per_lane(mg, prec, tol):
    n = N['ggttgg']
    say('ggttgg mt=0', prec, n)
    e = mg.MEEngine('ggttgg', prec, params={'mt': 0.0})
    assert e.layout.nhel_good == 32
    r, p, w, want = reference('ggttgg', 3, n, mt=0.0)
    got = e.sigmakin(e.events_mom(p), n).cpu()
    err = rel(got, want)
    kappa = invariant_condition(p)
    say('ggttgg mt=0', prec, 'max rel', float(err.max()), 'median', float(err.median()),
        'max kappa', float(kappa.max()), 'max err / (eps kappa)', float((err / (EPS * kappa)).max()))
    assert e.count_nonfinite(got.to(e.device)) == 0
    assert bool((err <= tol + 8 * EPS * kappa).all())
    # the sampler: massless RAMBO, weight (pi/2)^3 s^2 / 12 for every event
    _, mom, wgt = e.sample(3, n)
    assert torch.equal(wgt.cpu(), w)
    assert bool(((e.mom_events(mom, n).cpu() - p).abs().amax(dim=(1, 2))
                 <= momentum_bound(r, 1500.0)).all())


@pytest.mark.parametrize('proc', list(N))
def test_second_parameter_point_fp64(mg, proc):
    n = N[proc]
    seed = 11
    say('second point', proc, n)
    e = mg.MEEngine(proc, 'fp64', params=SECOND)
    r, p, w, want = reference(proc, seed, n, **SECOND)
    got = e.sigmakin(e.events_mom(p), n).cpu()
    err = rel(got, want)
    say('second point', proc, 'max rel', float(err.max()), 'median', float(err.median()))
    assert float(err.max()) <= 1e-12
    _, mom, wgt = e.sample(seed, n)
    assert bool(((e.mom_events(mom, n).cpu() - p).abs().amax(dim=(1, 2))
                 <= momentum_bound(r, SECOND['sqrts'])).all())
    assert bool(((wgt.cpu() / w - 1).abs() <= weight_bound(r, p, SECOND['sqrts'])).all())


@pytest.mark.parametrize('proc,prec', [('ggttg', 'mixed'), ('ggttgg', 'mixed'),
                                       ('ggttgg', 'fp32amp')])
def test_second_parameter_point_reduced_precision(mg, proc, prec):
    n = N[proc]
    e = mg.MEEngine(proc, prec, params=SECOND)
    r, p, w, want = reference(proc, 11, n, **SECOND)
    say('second point', proc, prec, n)
    got = e.sigmakin(e.events_mom(p), n).cpu()
    err = rel(got, want)
    say('second point', proc, prec, 'max rel', float(err.max()), 'median', float(err.median()))
    assert float(err.max()) <= 1e-5


@pytest.mark.parametrize('proc', ['ggtt', 'ggttg', 'ggttgg'])
def test_tchannel_zero_width_flag(mg, proc):
    n = N[proc]
    say('t-channel zero width', proc, n)
    e = mg.MEEngine(proc, 'fp64', params={'flags': mg.FLAG_TCHANNEL_ZERO_WIDTH})
    r, p, w, want = reference(proc, 12, n, flags=TCHANNEL_ZERO_WIDTH)
    got = e.sigmakin(e.events_mom(p), n).cpu()
    assert float(rel(got, want).max()) <= 1e-12
    # the flag changes the result: the default keeps the width everywhere
    _, _, _, dflt = reference(proc, 12, n)
    assert float(rel(want, dflt).max()) > 1e-9


@pytest.mark.parametrize('proc', ['eemumu', 'ggttg'])
def test_weight_2pi_flag(mg, proc):
    n = N[proc]
    say('weight 2pi', proc, n)
    e = mg.MEEngine(proc, 'fp64', params={'flags': mg.FLAG_WEIGHT_2PI})
    e0 = mg.MEEngine(proc, 'fp64')
    r, p, w, want = reference(proc, 13, n, flags=WEIGHT_2PI)
    _, mom, wgt = e.sample(13, n)
    _, mom0, wgt0 = e0.sample(13, n)
    assert torch.equal(e.mom_events(mom, n), e0.mom_events(mom0, n))
    nf = p.shape[1] - 2
    assert float(rel(wgt.cpu(), w).max()) <= float(weight_bound(r, p, 1500.0).max()) + 1e-15
    assert float(rel(wgt, wgt0 * (2 * math.pi) ** (4 - 3 * nf)).max()) <= 1e-15
    # the cross section does not depend on where the 2 pi factors are applied
    me, evtw = e.sigmakin(mom, n, wgt=wgt)
    me0, evtw0 = e0.sigmakin(mom0, n, wgt=wgt0)
    s, err, _ = e.cross_section(evtw, n)
    s0, err0, _ = e0.cross_section(evtw0, n)
    assert abs(s / s0 - 1) <= 1e-13 and abs(err / err0 - 1) <= 1e-10


def test_two_handles_with_different_parameters(mg):
    """Two handles of one process, default and SECOND, used alternately on
    one stream: each keeps its own parameters."""
    proc, n = 'ggttg', N['ggttg']
    a = mg.MEEngine(proc, 'fp64')
    b = mg.MEEngine(proc, 'fp64', params=SECOND)
    _, pa, _, wa = reference(proc, 2, n)
    _, pb, _, wb = reference(proc, 11, n, **SECOND)
    ma, mb = a.events_mom(pa), b.events_mom(pb)
    say('two handles', proc, n)
    for _ in range(2):
        ga = a.sigmakin(ma, n)
        gb = b.sigmakin(mb, n)
        ga2 = a.sigmakin(ma, n)
        assert float(rel(ga.cpu(), wa).max()) <= 1e-12
        assert float(rel(gb.cpu(), wb).max()) <= 1e-12
        assert torch.equal(ga, ga2)
    # and the handle's sampler uses its own sqrt(s)
    _, mom, _ = b.sample(11, n)
    E = b.mom_events(mom, n)[:, :2, 0].cpu()
    assert bool((E == SECOND['sqrts'] / 2).all())


def test_unknown_flag_bits_are_rejected(mg):
    import ctypes
    L = mg.lib()
    out = ctypes.c_void_p()
    bad = mg.Params(**dict(mg.DEFAULT_PARAMS, flags=8))
    assert L.mg_create(1, 0, ctypes.byref(bad), ctypes.byref(out)) == -1
    neg = mg.Params(**dict(mg.DEFAULT_PARAMS, wt=-1.0))
    assert L.mg_create(1, 0, ctypes.byref(neg), ctypes.byref(out)) == -1
