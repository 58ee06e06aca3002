"""Why the gradient's finite-difference check uses a fourth-order stencil (CPU).

The benchmark's gradient check names central differences with h = 1e-6.
On a few events of the g g -> t t~ g workload (seed 4; listed with their
miss in tests/golden/fd_truncation_ggttg_seed4.txt, found by scanning the
first 1024 events with the oracle) the two-point stencil misses the
oracle's reverse-mode gradient by up to 3e-5.  That miss is the stencil's
truncation error h^2 f'''/6, not an error of either gradient: it scales as
h^2 (halving h divides it by 4), and the fourth-order stencil on the same
events and the same h agrees with the reverse-mode gradient to rounding
(eps |f| / h).  So the GPU check compares against the fourth-order stencil
at h = 1e-6.
"""
import os

import torch

from oracle import me as orc
from oracle import rambo
from oracle.params import DEFAULT

HERE = os.path.dirname(os.path.abspath(__file__))


def _events():
    rows = []
    for line in open(os.path.join(HERE, 'golden', 'fd_truncation_ggttg_seed4.txt')):
        if line.strip() and not line.startswith('#'):
            i, miss = line.split()
            rows.append((int(i), float(miss)))
    return rows


def _f(r):
    masses = orc.PROCESSES['ggttg'].final_masses(DEFAULT)
    p, w = rambo.event_momenta(r, DEFAULT.sqrts, masses)
    return orc.matrix_element('ggttg', p) * w


def _stencil(r, h, taps):
    out = torch.zeros_like(r)
    for k in range(r.shape[1]):
        for s, c in taps:
            rr = r.clone()
            rr[:, k] += s * h
            out[:, k] += c * _f(rr)
        out[:, k] /= h
    return out


TWO = ((1, 0.5), (-1, -0.5))
FOUR = ((-2, 1 / 12), (-1, -8 / 12), (1, 8 / 12), (2, -1 / 12))


def test_two_point_miss_is_truncation():
    rows = _events()
    assert rows, 'no listed events'
    idx = [i for i, _ in rows]
    r = torch.cat([orc.sample('ggttg', 4, i, 1)[0] for i in idx])
    _, g, _ = orc.event_weight_and_grad('ggttg', r)

    def miss(d):
        return (d - g).norm(dim=1) / g.norm(dim=1)

    e2 = miss(_stencil(r, 2e-6, TWO))
    e1 = miss(_stencil(r, 1e-6, TWO))
    e05 = miss(_stencil(r, 5e-7, TWO))
    # the listed misses are reproduced, and they scale as h^2
    want = torch.tensor([m for _, m in rows], dtype=torch.float64)
    assert torch.allclose(e1, want, rtol=1e-3)
    assert (e1 > 1e-6).all()
    assert ((e2 / e1 - 4).abs() < 0.05).all()
    assert ((e1 / e05 - 4).abs() < 0.05).all()
    # the fourth-order stencil at the same step meets the 1e-6 bound with room
    e4 = miss(_stencil(r, 1e-6, FOUR))
    assert float(e4.max()) < 1e-8
