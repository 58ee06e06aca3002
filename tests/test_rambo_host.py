"""The HIP path's RAMBO header compiled for the host, against the oracle (CPU).

tests/host/rambo_host.cpp builds paper_2106_12631_amd/csrc/rambo.h with the
host compiler (tests/host/hip/hip_runtime.h stands in for the HIP header)
and maps the oracle's uniforms of every benchmark workload to momenta and
weights.  The oracle and the header are written independently from the same
method (Kleiss-Stirling-Ellis with the boost from pairwise Minkowski
products), so they must agree to the rounding bounds of tests/rounding.py.
This checks the formulas on the CPU; the GPU parity tests check the device
build of the same header.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from oracle import me as orc
from rounding import EPS, boost_gamma, momentum_bound, weight_bound

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

WORKLOADS = [('eemumu', 0, 0.0), ('ggtt', 1, 173.0), ('ggttg', 2, 173.0), ('ggttgg', 3, 173.0)]


@pytest.fixture(scope='module')
def exe(tmp_path_factory):
    cxx = shutil.which('g++')
    if cxx is None:
        pytest.skip('no host C++ compiler')
    out = str(tmp_path_factory.mktemp('rambo') / 'rambo_host')
    subprocess.check_call([cxx, '-std=c++17', '-O2', '-I', os.path.join(HERE, 'host'),
                           '-I', os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc'),
                           os.path.join(HERE, 'host', 'rambo_host.cpp'), '-o', out])
    return out


@pytest.mark.parametrize('proc,seed,mass', WORKLOADS)
def test_device_rambo_on_host(exe, tmp_path, proc, seed, mass):
    n = 8192
    r, p, w = orc.sample(proc, seed, 0, n)
    nf = p.shape[1] - 2
    fin, fout = str(tmp_path / 'r.bin'), str(tmp_path / 'p.bin')
    r.numpy().tofile(fin)
    subprocess.check_call([exe, str(nf), '1500', repr(mass), fin, fout])
    out = torch.from_numpy(np.fromfile(fout).reshape(n, -1))
    ph, wh = out[:, :-1].reshape(n, nf + 2, 4), out[:, -1]
    dp = (ph - p).abs().amax(dim=(1, 2))
    assert bool((dp <= momentum_bound(r, 1500.0)).all()), float((dp / momentum_bound(r, 1500.0)).max())
    dw = (wh / w - 1).abs()
    assert bool((dw <= weight_bound(r, p, 1500.0)).all())
    # conservation of the host build on its own: within 64 eps gamma sqrt(s)
    tot = ph[:, 2:].sum(1) - ph[:, :2].sum(1)
    assert bool((tot.abs().amax(1) <= momentum_bound(r, 1500.0)).all())
    # masses on shell: |p^2 - m^2| <= 64 eps gamma s
    m2 = ph[:, 2:, 0] ** 2 - (ph[:, 2:, 1:] ** 2).sum(-1)
    want = torch.tensor(orc.PROCESSES[proc].final_masses(orc.DEFAULT)) ** 2
    assert bool(((m2 - want).abs().amax(1) <= 64 * EPS * boost_gamma(r) * 1500.0 ** 2).all())
