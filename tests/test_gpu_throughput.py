"""The events-per-launch sweep (GPU): one JSON record per size, with
positive rates, SIGMAKIN alone at least as fast as sampler + SIGMAKIN."""
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
