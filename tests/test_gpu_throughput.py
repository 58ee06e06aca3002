"""The events-per-launch sweep and its plateau workload (GPU).

The sweep gives one JSON record per size, with positive rates, SIGMAKIN
alone at least as fast as sampler + SIGMAKIN; the plateau workload (2^24
e+e- -> mu+mu- events) is checked against the oracle on sampled events."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_throughput_sweep_records():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_12631_amd import throughput
    print('[gpu-test] throughput sweep eemumu', flush=True)
    sys.stdout.flush()
    recs = throughput.sweep('eemumu', 'fp64', [1024, 4096], steps=3, warmup=1)
    assert [r['nevt'] for r in recs] == [1024, 4096]
    for r in recs:
        assert r['sigmakin_MEs_per_s'] > 0 and r['sample_sigmakin_MEs_per_s'] > 0
        assert r['sigmakin_MEs_per_s'] >= r['sample_sigmakin_MEs_per_s']


def test_plateau_workload_parity():
    """The throughput-plateau workload (e+e- -> mu+mu-, 2^24 events, seed 0),
    launched at full size as the benchmark launches it: no non-finite matrix
    element, and sampled events (first, last, middle, 29 seeded others)
    against the oracle event by event: momenta and weights within the RAMBO
    rounding bounds, |M|^2 of the launch's own momenta within 1e-12 and end
    to end within the bound of tests/rounding.py."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as mg
    from oracle import me as orc
    from rounding import end_to_end_bound, momentum_bound, weight_bound
    n, seed = 1 << 24, 0
    e = mg.MEEngine('eemumu', 'fp64')
    print('[gpu-test] plateau workload eemumu', n, flush=True)
    _, mom, wgt = e.sample(seed, n)
    me = e.sigmakin(mom, n)
    torch.cuda.synchronize()
    assert e.count_nonfinite(me) == 0 and e.count_nonfinite(wgt) == 0
    g = torch.Generator().manual_seed(24)
    idx = sorted(set([0, n - 1, n // 2] + torch.randint(0, n, (29,), generator=g).tolist()))
    it = torch.tensor(idx, device=me.device)
    me_gpu, w_gpu = me[it].cpu(), wgt[it].cpu()
    p_gpu = torch.cat([e.mom_events(mom[(i // 64) * 64 * 16:(i // 64 + 1) * 64 * 16], 64)[i % 64:i % 64 + 1]
                       for i in idx]).cpu()
    r = torch.cat([orc.sample('eemumu', seed, i, 1)[0] for i in idx])
    p = torch.cat([orc.sample('eemumu', seed, i, 1)[1] for i in idx])
    w = torch.cat([orc.sample('eemumu', seed, i, 1)[2] for i in idx])
    assert bool(((p_gpu - p).abs().amax(dim=(1, 2)) <= momentum_bound(r, 1500.0)).all())
    assert bool(((w_gpu / w - 1).abs() <= weight_bound(r, p, 1500.0)).all())
    own = orc.matrix_element('eemumu', p_gpu)
    assert float(((me_gpu - own).abs() / own).max()) <= 1e-12
    want = orc.matrix_element('eemumu', p)
    assert bool((((me_gpu - want).abs() / want) <= end_to_end_bound(r, p)).all())


def test_calibration_kernels():
    """The calibration streams run and reach a plausible share of the
    published peaks (between 30 % and 105 %), so the bench's calibrated
    roofline fractions rest on working kernels."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_12631_amd import calibrate
    print('[gpu-test] calibration kernels', flush=True)
    res = calibrate.run(blocks=512)
    assert set(res) == {k[0] for k in calibrate.KINDS.values()}
    for name, r in res.items():
        print('[gpu-test]', name, round(r['achieved_TFLOPs'], 1), 'TFLOP/s', flush=True)
        assert 0.3 <= r['frac'] <= 1.05, name
