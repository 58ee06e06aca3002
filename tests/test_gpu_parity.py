"""Parity of the HIP path with the FP64 oracle, through the C ABI (GPU).

Every comparison uses seeded synthetic events.  Tolerances:
* uniforms: bit-exact (integer Philox, exact bits->double map);
* momenta and weights: RAMBO's boost amplifies rounding by ~gamma; the bounds
  of tests/rounding.py (64 eps gamma sqrt(s) for momenta, the same over
  min |k_i| for weights) are the sum of both sides' bounds;
* |M|^2 on identical momenta: 1e-12 relative for FP64 (the benchmark's
  stated FP64 target); FP32 amplitudes are checked against a bound derived
  from single-precision rounding through the diagram sums.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import me as orc
from oracle import philox, rambo
from rounding import end_to_end_bound, momentum_bound, weight_bound

pytestmark = pytest.mark.gpu

CONFIG = {  # process: (seed, events at full size)
    'eemumu': (0, 16384),
    'ggtt': (1, 1 << 20),
    'ggttg': (2, 1 << 20),
    'ggttgg': (3, 1 << 19),
}
# parity sizes the oracle evaluates in seconds: several 64-event pages + a ragged tail
SMALL = {'eemumu': 4096 + 17, 'ggtt': 2048 + 33, 'ggttg': 640 + 5, 'ggttgg': 192 + 7}


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
    key = (proc, prec)
    if key not in _ENG:
        say('create', proc, prec)
        _ENG[key] = mg.MEEngine(proc, prec)
    return _ENG[key]


def rel(a, b):
    return ((a - b).abs() / b.abs())


@pytest.mark.parametrize('proc', list(CONFIG))
def test_rng_bitwise(mg, proc):
    e = engine(mg, proc)
    seed, _ = CONFIG[proc]
    n = SMALL[proc]
    say('rng', proc, n)
    rnd = e.rng(seed, n)
    got = e.rnd_events(rnd, n).cpu().numpy()
    want = philox.uniforms(seed, 0, n, e.layout.nrnd)
    assert np.array_equal(got, want)
    # an event range is reproducible on its own (counter = global index)
    off = 1000
    got2 = e.rnd_events(e.rng(seed, 300, offset=off), 300).cpu().numpy()
    assert np.array_equal(got2, philox.uniforms(seed, off, 300, e.layout.nrnd))


@pytest.mark.parametrize('proc', list(CONFIG))
def test_rambo_parity(mg, proc):
    e = engine(mg, proc)
    seed, _ = CONFIG[proc]
    n = SMALL[proc]
    r, p_orc, w_orc = orc.sample(proc, seed, 0, n)
    say('rambo', proc, n)
    mom, wgt = e.rambo(e.events_rnd(r), n)
    p = e.mom_events(mom, n).cpu()
    w = wgt.cpu()
    dp = (p - p_orc).abs().amax(dim=(1, 2))
    say('rambo', proc, 'max |dp| / bound', float((dp / momentum_bound(r, 1500.0)).max()))
    assert bool((dp <= momentum_bound(r, 1500.0)).all())
    assert bool((rel(w, w_orc) <= weight_bound(r, p_orc, 1500.0)).all())
    # the fused sampler produces the same events as rng + rambo
    rnd2, mom2, wgt2 = e.sample(seed, n, keep_rnd=True)
    assert torch.equal(e.rnd_events(rnd2, n).cpu(), r)
    assert torch.equal(e.mom_events(mom2, n).cpu(), p)
    assert torch.equal(wgt2.cpu(), w)


@pytest.mark.parametrize('proc', list(CONFIG))
def test_sigmakin_fp64_parity(mg, proc):
    e = engine(mg, proc)
    seed, _ = CONFIG[proc]
    n = SMALL[proc]
    r, p_orc, w_orc = orc.sample(proc, seed, 0, n)
    want = orc.matrix_element(proc, p_orc)
    say('sigmakin fp64', proc, n)
    mom = e.events_mom(p_orc)
    wdev = w_orc.to(e.device)
    me, evtw = e.sigmakin(mom, n, wgt=wdev)
    got = me.cpu()
    err = rel(got, want)
    say(proc, 'fp64 max rel', float(err.max()), 'median', float(err.median()))
    assert float(err.max()) <= 1e-12
    assert torch.equal(evtw.cpu(), got * w_orc)


def test_helicity_filtering(mg):
    assert engine(mg, 'eemumu').layout.nhel_good == 4
    for proc in ('ggtt', 'ggttg', 'ggttgg'):
        lay = engine(mg, proc).layout
        assert lay.nhel_good == lay.nhel


@pytest.mark.parametrize('proc', list(CONFIG))
def test_sigmakin_per_helicity(mg, proc):
    """Per-helicity colour-summed |M|^2 sums to IDEN x ME, and the helicities
    dropped by the filter are exactly zero."""
    e = engine(mg, proc)
    n = 130
    r, p_orc, w_orc = orc.sample(proc, CONFIG[proc][0], 0, n)
    mom = e.events_mom(p_orc)
    say('sigmakin_hel', proc, n)
    hel = e.sigmakin_hel(mom, n).cpu()
    me = e.sigmakin(mom, n).cpu()
    assert float(rel(hel.sum(0) / e.layout.iden, me).max()) < 1e-13
    ref = orc.me_per_helicity(proc, p_orc)
    assert int(((ref != 0).any(1)).sum()) == int(((hel != 0).any(1)).sum())


@pytest.mark.parametrize('proc', ['ggtt', 'ggttg', 'ggttgg'])
def test_sigmakin_fp32amp_accuracy(mg, proc):
    e = engine(mg, proc, 'fp32amp')
    n = SMALL[proc]
    r, p_orc, w_orc = orc.sample(proc, CONFIG[proc][0], 0, n)
    want = orc.matrix_element(proc, p_orc)
    say('sigmakin fp32amp', proc, n)
    got = e.sigmakin(e.events_mom(p_orc), n).cpu()
    err = rel(got, want)
    say(proc, 'fp32amp max rel', float(err.max()), 'median', float(err.median()))
    assert e.count_nonfinite(got.to(e.device)) == 0
    assert float(err.median()) < 1e-6
    assert float(err.max()) <= 1e-5


@pytest.mark.parametrize('proc,prec', [('ggttg', 'mixed'), ('ggttgg', 'mixed'),
                                       ('ggttg', 'mixed_f32mfma'), ('ggttgg', 'mixed_f32mfma'),
                                       ('ggtt', 'mixed'), ('eemumu', 'mixed')])
def test_sigmakin_mixed_accuracy(mg, proc, prec):
    """Matrix-core colour sum: within the mixed-precision target of the FP64
    oracle, and close to the FP32-amplitude path (same jamps, VALU colour
    sum); includes a ragged last wave."""
    e = engine(mg, proc, prec)
    n = SMALL[proc]
    r, p_orc, w_orc = orc.sample(proc, CONFIG[proc][0], 0, n)
    want = orc.matrix_element(proc, p_orc)
    say('sigmakin', prec, proc, n)
    mom = e.events_mom(p_orc)
    got = e.sigmakin(mom, n).cpu()
    err = rel(got, want)
    say(proc, prec, 'max rel', float(err.max()), 'median', float(err.median()))
    assert e.count_nonfinite(got.to(e.device)) == 0
    assert float(err.max()) <= 1e-5
    ref32 = engine(mg, proc, 'fp32amp').sigmakin(mom, n).cpu()
    assert float(rel(got, ref32).max()) <= 2e-6


@pytest.mark.parametrize('proc', list(CONFIG))
def test_end_to_end_fp64(mg, proc):
    """Uniforms -> RAMBO -> |M|^2 on both sides (GPU sampler and SIGMAKIN,
    oracle sampler and matrix element): max, median and the number of events
    above 1e-12.  The GPU momenta differ from the oracle's by rounding of
    order eps gamma sqrt(s), which the matrix element carries into the
    result on top of the 1e-12 of identical momenta, amplified by the
    matrix element's sensitivity to its invariants (tests/rounding.py)."""
    e = engine(mg, proc)
    seed, _ = CONFIG[proc]
    n = SMALL[proc]
    r, p_orc, w_orc = orc.sample(proc, seed, 0, n)
    want = orc.matrix_element(proc, p_orc)
    say('end to end', proc, n)
    _, mom, wgt = e.sample(seed, n)
    me, evtw = e.sigmakin(mom, n, wgt=wgt)
    err = rel(me.cpu(), want)
    werr = rel(evtw.cpu(), want * w_orc)
    bound = end_to_end_bound(r, p_orc)
    say(proc, 'end-to-end ME max rel', float(err.max()), 'median', float(err.median()),
        'above 1e-12:', int((err > 1e-12).sum()), 'of', n, '| w ME max rel', float(werr.max()),
        '| max err / bound', float((err / bound).max()))
    assert bool((err <= bound).all())
    assert bool((werr <= bound + weight_bound(r, p_orc, 1500.0)).all())


@pytest.mark.parametrize('proc', list(CONFIG))
def test_full_size_sampled(mg, proc):
    """Full benchmark size, launched as the benchmark launches it; sampled
    events compared with the oracle evaluated event by event."""
    e = engine(mg, proc)
    seed, n = CONFIG[proc]
    say('full size', proc, n)
    _, mom, wgt = e.sample(seed, n)
    me = e.sigmakin(mom, n)
    torch.cuda.synchronize()
    assert e.count_nonfinite(me) == 0
    g = torch.Generator().manual_seed(seed)
    idx = sorted(set([0, n - 1, n // 2] + torch.randint(0, n, (29,), generator=g).tolist()))
    p_gpu = e.mom_events(mom, n)[idx].cpu()
    me_gpu = me[idx].cpu()
    w_gpu = wgt[idx].cpu()
    for k, i in enumerate(idx):
        r, p_orc, w_orc = orc.sample(proc, seed, i, 1)
        assert float((p_gpu[k] - p_orc[0]).abs().max()) <= float(momentum_bound(r, 1500.0)[0])
        assert abs(float(w_gpu[k] / w_orc[0]) - 1) <= float(weight_bound(r, p_orc, 1500.0)[0])
    # the full-size launch's matrix elements on its own momenta
    assert float(rel(me_gpu, orc.matrix_element(proc, p_gpu)).max()) <= 1e-12
    # the matrix elements of the sampled events, on the oracle's momenta
    ps = torch.cat([orc.sample(proc, seed, i, 1)[1] for i in idx])
    want = orc.matrix_element(proc, ps)
    got = e.sigmakin(e.events_mom(ps), len(idx)).cpu()
    assert float(rel(got, want).max()) <= 1e-12
    # end to end (uniforms -> momenta -> |M|^2 on both sides): the
    # momentum rounding of the sampled events adds to the 1e-12
    rs = torch.cat([orc.sample(proc, seed, i, 1)[0] for i in idx])
    say(proc, 'full-size end-to-end max rel', float(rel(me_gpu, want).max()))
    assert bool((rel(me_gpu, want) <= end_to_end_bound(rs, ps)).all())


def test_edge_cases_and_errors(mg):
    e = engine(mg, 'ggtt')
    L = mg.lib()
    import ctypes
    h = e._h
    # nevt = 0 is a no-op success
    assert L.mg_sigmakin(h, None, 0, None, None, None, None) == 0
    assert L.mg_sample(h, 1, 0, 0, None, None, None, None) == 0
    # invalid arguments
    assert L.mg_sigmakin(h, None, 5, None, None, None, None) == -1
    assert L.mg_rng(h, 1, 0, -1, None, None) == -1
    buf = torch.zeros(4096, dtype=torch.float64, device=e.device)
    mis = ctypes.c_void_p(buf.data_ptr() + 4)
    assert L.mg_sigmakin(h, mis, 1, ctypes.c_void_p(buf.data_ptr()), None, None, None) == -5
    out = ctypes.c_void_p()
    assert L.mg_create(7, 0, None, ctypes.byref(out)) == -1
    assert L.mg_create(1, 9, None, ctypes.byref(out)) == -1
    bad = mg.Params(**dict(mg.DEFAULT_PARAMS, sqrts=300.0))
    assert L.mg_create(1, 0, ctypes.byref(bad), ctypes.byref(out)) == -3
    # non-finite counting
    x = torch.tensor([1.0, float('nan'), 2.0, float('inf'), -float('inf')], dtype=torch.float64,
                     device=e.device)
    assert e.count_nonfinite(x) == 3
    # a single event and a single ragged page
    for n in (1, 63, 65):
        r, p_orc, _ = orc.sample('ggtt', 9, 0, n)
        got = e.sigmakin(e.events_mom(p_orc), n).cpu()
        assert float(rel(got, orc.matrix_element('ggtt', p_orc)).max()) <= 1e-12


def test_module_shortcuts(mg):
    """mg.sample / mg.sigmakin (cached default engines) give the engine's results."""
    n = 100
    rnd, mom, wgt = mg.sample(3, n, process='ggttgg')
    me, evtw = mg.sigmakin(mom, n, wgt=wgt, process='ggttgg')
    e = engine(mg, 'ggttgg')
    r = e.rnd_events(rnd, n).cpu()
    _, mom2, wgt2 = e.sample(3, n)
    # AoSoA slots past nevt are not written: compare the events only
    assert torch.equal(e.mom_events(mom, n), e.mom_events(mom2, n)) and torch.equal(wgt, wgt2)
    assert torch.equal(me, e.sigmakin(mom2, n))
    assert torch.equal(evtw, me * wgt)
    p = e.mom_events(mom, 8).cpu()
    ref = orc.matrix_element('ggttgg', p)
    assert float(rel(me[:8].cpu(), ref).max()) <= 1e-12
    assert torch.equal(r, orc.sample('ggttgg', 3, 0, n)[0])


@pytest.mark.parametrize('proc,n', [('ggtt', (1 << 16) + 37), ('ggttg', (1 << 16) + 37),
                                    ('eemumu', (1 << 16) + 37)])
def test_event_per_lane_above_the_group_threshold(mg, proc, n):
    """Launches above a process's group threshold take the event-per-lane
    kernel (below it, several lanes per event): a ragged launch of that size
    against the oracle on the first and last 64 events and 64 seeded others."""
    e = engine(mg, proc)
    seed = CONFIG[proc][0]
    say('event per lane', proc, n)
    _, mom, _ = e.sample(seed, n)
    me = e.sigmakin(mom, n)
    torch.cuda.synchronize()
    assert e.count_nonfinite(me) == 0
    g = torch.Generator().manual_seed(n)
    idx = sorted(set(list(range(64)) + list(range(n - 64, n)) +
                     torch.randint(0, n, (64,), generator=g).tolist()))
    p = e.mom_events(mom, n)[idx].cpu()
    got = me[torch.tensor(idx, device=me.device)].cpu()
    want = orc.matrix_element(proc, p)
    assert float(rel(got, want).max()) <= 1e-12
