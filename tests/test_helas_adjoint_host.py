"""Dot-product tests of the hand-written reverse-mode HELAS routines (CPU).

tests/host/adj_dot.cpp compiles the device headers helas.h and helas_adj.h
for the host (tests/host/hip/hip_runtime.h stands in for the HIP header) and
checks every adjoint routine against the forward routine it reverses: for
random inputs, output adjoints and tangents, Re<ob, J dx> from forward-mode
dual numbers through the forward routine must equal Re<xb, dx> from the
adjoint routine (the transpose identity of reverse mode).  The external
wavefunction adjoints, themselves built from dual numbers, are checked
against fourth-order central differences of the plain forward routine.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope='module')
def report(tmp_path_factory):
    cxx = shutil.which('g++')
    if cxx is None:
        pytest.skip('no host C++ compiler')
    exe = str(tmp_path_factory.mktemp('adj') / 'adj_dot')
    subprocess.check_call([cxx, '-std=c++17', '-O1', '-I', os.path.join(HERE, 'host'),
                           '-I', os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc'),
                           os.path.join(HERE, 'host', 'adj_dot.cpp'), '-o', exe])
    out = subprocess.check_output([exe], text=True)
    rows = {}
    for line in out.splitlines():
        name, n, worst = line.split()
        rows[name] = (int(n), float(worst))
    return rows


ROUTINES = ['adj_bilinear', 'adj_mdot_i', 'adj_ffv_amp', 'adj_ffv_cur_v0', 'adj_ffv_cur_vm',
            'adj_ffv_cur_fin(massive)', 'adj_ffv_cur_fin(massless)',
            'adj_ffv_cur_fout(massive)', 'adj_ffv_cur_fout(massless)', 'adj_vvv_cur',
            'adj_vvvv_cur<1>', 'adj_vvvv_cur<2>', 'adj_vvvv_cur<3>']
EXTERNALS = ['adj_ext_vector', 'adj_ext_u', 'adj_ext_v', 'adj_ext_u(massless)']


@pytest.mark.parametrize('name', ROUTINES)
def test_adjoint_dot_product(report, name):
    n, worst = report[name]
    assert n == 200
    assert worst <= 1e-11, f'{name}: transpose identity off by {worst:.2e}'


@pytest.mark.parametrize('name', EXTERNALS)
def test_external_adjoint_vs_differences(report, name):
    n, worst = report[name]
    assert n == 200
    assert worst <= 1e-7, f'{name}: adjoint vs central differences off by {worst:.2e}'
