"""Host logic of the diagram generator and of bench.py (CPU only).

* The emitted straight-line code and the cost model of the order search
  agree: the flops recomputed by the emitted body under a register budget
  equal the cost model's excess over an unlimited budget; with an unlimited
  budget nothing is recomputed; at a budget above the largest single need
  the live set never exceeds the budget.
* The order search returns a permutation of the diagrams whose cost does
  not exceed the starting order's.
* The recorded schedules of the generated code (written by the build)
  respect the same bounds, and its process constants match the diagram and
  colour counts.
* bench.py refuses more than one GPU with a message and exit status 2.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope='module')
def ggttg():
    from paper_2106_12631_amd.gen import emit
    from paper_2106_12631_amd.gen.diagrams import ProcessDiagrams
    pd = ProcessDiagrams('ggttg')
    order, bils, need = emit.schedule(pd)
    return emit, pd, pd.jamp_coefficients(), order, bils, need


def test_emitted_recomputation_matches_cost_model(ggttg):
    emit, pd, coefs, order, bils, need = ggttg
    unlimited = emit.schedule_cost(order, need, 10 ** 6)
    for budget in (6, 8, 10, 12, 10 ** 6):
        _, algo, execd, peak, rec = emit.emit_body(pd, coefs, order, bils, need, budget)
        assert execd - algo == emit.schedule_cost(order, need, budget) - unlimited
        if budget >= 8:
            assert peak <= budget
    _, algo, execd, peak, rec = emit.emit_body(pd, coefs, order, bils, need, 10 ** 6)
    assert execd == algo and rec == 0


def test_order_search_is_a_permutation_that_does_not_cost_more(ggttg):
    emit, pd, coefs, order, bils, need = ggttg
    best, cost = emit.optimise_order(order, need, 8, iters=300)
    assert sorted(best) == sorted(order)
    assert cost == emit.schedule_cost(best, need, 8) <= emit.schedule_cost(order, need, 8)


def test_generated_code_metadata():
    from paper_2106_12631_amd.gen import emit
    path = os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc', 'generated', 'meta.json')
    if not os.path.exists(path):
        pytest.skip("the generated code is written by the build (paper_2106_12631_amd.build)")
    meta = json.load(open(path))
    want = {'eemumu': (4, 1, 2, 4), 'ggtt': (4, 2, 3, 256), 'ggttg': (5, 6, 16, 256),
            'ggttgg': (6, 24, 123, 512)}
    for proc, (npar, ncol, ndiag, iden) in want.items():
        m = meta[proc]
        assert (m['npar'], m['ncol'], m['ndiag'], m['iden']) == (npar, ncol, ndiag, iden)
        for prec, st in m['schedule'].items():
            if prec.startswith('a'):  # gradient: forward and reverse sweeps
                assert st['flops_reverse_executed_per_hel'] > st['flops_forward_executed_per_hel']
                assert st['flops_forward_executed_per_hel'] >= m['flops_amp_per_hel']
                continue
            assert st['flops_executed_per_hel'] >= st['flops_amp_per_hel'] == m['flops_amp_per_hel']
            assert st['peak_live_wavefunctions'] <= max(emit.BUDGET[prec], 8)
    # gg -> t t~ g g: the FP64 budget trades recomputation for registers
    s = meta['ggttgg']['schedule']
    assert s['f64']['flops_executed_per_hel'] < s['f32']['flops_executed_per_hel']
    assert s['f32m']['recomputed'] == 0


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert 'one GPU only' in r.stderr and r.stdout == ''
