"""Cross section and unweighting kernels against the oracle (GPU).

* mg_xsec_stats: sums within 1e-13 relative of the oracle's (a different
  summation order), maximum and finite count exact, the same bits on a
  second call (fixed summation order), up to 2^24 + 3 events;
* mg_unweight: the kept index list is identical to the oracle's (an integer
  result decided by the same FP64 comparison on the same uniforms);
* inputs are seeded synthetic weights (heavy-tailed, with NaN and infinite
  entries) at sizes covering empty, one block, ragged tails and 2^20;
* end to end: the e+e- -> mu+mu- cross section from the GPU path (16384
  events, seed 0) equals the oracle's on the same events within 1e-12 and the
  textbook integral within four standard errors.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import integrate as oi
from oracle import me as orc
from oracle.params import DEFAULT

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


def weights(n, seed, special=True):
    rng = np.random.default_rng(seed)
    f = rng.pareto(1.5, n) * rng.random(n)
    if special and n > 8:
        f[rng.integers(0, n, 3)] = np.nan
        f[rng.integers(0, n, 2)] = np.inf
        f[rng.integers(0, n, 2)] = 0.0
    return f


@pytest.mark.parametrize('n', [0, 1, 255, 256, 257, 4096 + 37, 1 << 20, (1 << 24) + 3])
def test_xsec_stats(mg, n):
    f = weights(n, 100 + n)
    say('xsec_stats', n)
    st = mg.xsec_stats(torch.from_numpy(f).cuda()).cpu().numpy()
    ref = oi.stats(f)
    for k in (0, 1):
        assert st[k] == pytest.approx(ref[k], rel=1e-13, abs=0.0)
    assert st[2] == ref[2] and st[3] == ref[3]
    # fixed summation order: a second call gives the same bits
    st2 = mg.xsec_stats(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.array_equal(st, st2)


@pytest.mark.parametrize('n,fmax,seed,off', [(0, 1.0, 1, 0), (1, 0.5, 2, 0), (255, 2.0, 3, 7),
                                             (256, 1.0, 4, 0), (257, 3.0, 5, 1 << 33),
                                             (4096 + 37, 4.0, 6, 12), (1 << 20, 10.0, 7, 0),
                                             (1000, 0.0, 8, 0)])
def test_unweight_bitexact(mg, n, fmax, seed, off):
    f = weights(n, 200 + n)
    say('unweight', n, fmax, seed, off)
    idx = mg.unweight(torch.from_numpy(f).cuda(), fmax, seed, off).cpu().numpy()
    ref = oi.unweight(f, fmax, seed, off)
    assert idx.dtype == np.int64
    assert np.array_equal(idx, ref)


def test_errors(mg):
    L = mg.lib()
    assert L.mg_xsec_stats(None, 4, None, None, None) == -1
    ws = torch.empty(L.mg_xsec_stats_workspace_bytes(1 << 30) // 8, dtype=torch.float64).cuda()
    out = torch.empty(4, dtype=torch.float64).cuda()
    assert L.mg_xsec_stats(None, 4, out.data_ptr(), ws.data_ptr(), None) == -1
    assert L.mg_xsec_stats(out.data_ptr(), 4, out.data_ptr(), None, None) == -1
    assert L.mg_xsec_stats_workspace_bytes(0) == 32
    assert L.mg_xsec_stats_workspace_bytes(1 << 30) == 2048 * 32
    assert L.mg_unweight(None, 4, 1.0, 0, 0, None, None, None, None) == -1
    f = torch.ones(4, dtype=torch.float64).cuda()
    assert L.mg_unweight(f.data_ptr(), 4, -1.0, 0, 0, f.data_ptr(), f.data_ptr(), f.data_ptr(),
                         None) == -1
    assert L.mg_unweight_workspace_bytes(0) >= 8
    assert L.mg_unweight_workspace_bytes(257) == 16


def test_eemumu_cross_section_end_to_end(mg):
    e = mg.MEEngine('eemumu')
    n = 16384
    say('eemumu cross section', n)
    _, mom, wgt = e.sample(0, n)
    _, evtw = e.sigmakin(mom, n, wgt=wgt)
    sig, err, st = e.cross_section(evtw, n)
    _, p, w = orc.sample('eemumu', 0, 0, n)
    f = (orc.matrix_element('eemumu', p) * w).numpy()
    sig_o, err_o = oi.xsec(oi.stats(f), n, DEFAULT.sqrts, 2)
    assert sig == pytest.approx(sig_o, rel=1e-12)
    assert err == pytest.approx(err_o, rel=1e-6)
    # the textbook integral of |M|^2 over cos(theta)
    import test_oracle_integrate as toi
    exact = toi._sigma_eemumu_exact()
    say('sigma', sig, '+-', err, 'pb; exact', exact)
    assert abs(sig - exact) <= 4 * err
    kept = mg.unweight(evtw, float(st[2]), seed=9)
    assert np.array_equal(kept.cpu().numpy(), oi.unweight(evtw.cpu().numpy(), float(st[2]), 9))
