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
* The matrix-core operand tables of the colour matrix decode, in the lane
  layout of the 32x32 MFMA tiles, back to the colour matrix: every row and
  column of C once per split chunk, zeros in the padding.
* The register budget of the measurement build (build.py --no-recompute,
  whose executed flops are taken as the algorithmic flops) leaves nothing
  to recompute in any process's amplitude code.
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


@pytest.mark.parametrize('proc', ['ggtt', 'ggttg', 'ggttgg'])
def test_colour_mfma_tables_decode_to_the_colour_matrix(proc):
    import struct
    from paper_2106_12631_amd.gen import emit
    from paper_2106_12631_amd.gen.diagrams import ProcessDiagrams, colour_matrix
    pd = ProcessDiagrams(proc)
    basis = pd.colour_basis()
    n = len(basis)
    cnum, _ = colour_matrix(basis, len(pd.gluons))
    f32, bf16 = emit.colour_mfma_tables(cnum, n)

    def bf16_value(h):
        return struct.unpack('<f', struct.pack('<I', h << 16))[0]

    # F32: lane l of K block kb holds A[m = l % 32][k = 2 kb + l / 32]
    A = {}
    for kb, row in enumerate(f32):
        for lane, v in enumerate(row):
            A[(lane % 32, 2 * kb + lane // 32)] = v
    for (m, k), v in A.items():
        assert v == (cnum[m][k] if m < n and k < n else 0.0)
    assert all((m, k) in A for m in range(n) for k in range(n))
    # BF16: lane l of K block kb holds the eight K entries of chunk
    # c = 2 kb + l / 32, chunk c = s G + g covering colours 8 g .. 8 g + 7
    G = (n + 7) // 8
    seen = {}
    for kb, row in enumerate(bf16):
        for lane, words in enumerate(row):
            m, c = lane % 32, 2 * kb + lane // 32
            vals = [bf16_value((w >> (16 * t)) & 0xFFFF) for w in words for t in (0, 1)]
            for j, v in enumerate(vals):
                col = 8 * (c % G) + j
                if m < n and c < 3 * G and col < n:
                    assert v == cnum[m][col]
                    seen[(c // G, m, col)] = True
                else:
                    assert v == 0.0
    assert len(seen) == 3 * n * n


@pytest.mark.parametrize('proc', ['eemumu', 'ggtt', 'ggttg', 'ggttgg'])
def test_measurement_build_budget_recomputes_nothing(proc):
    from paper_2106_12631_amd import build
    from paper_2106_12631_amd.gen import emit
    from paper_2106_12631_amd.gen.diagrams import ProcessDiagrams
    pd = ProcessDiagrams(proc)
    order, bils, need = emit.schedule(pd)
    budget = build.NO_RECOMPUTE_BUDGET
    _, algo, execd, peak, rec = emit.emit_body(pd, pd.jamp_coefficients(), order, bils, need,
                                               budget)
    assert rec == 0 and execd == algo and peak < budget


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert 'one GPU only' in r.stderr and r.stdout == ''
