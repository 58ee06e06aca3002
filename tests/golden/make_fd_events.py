"""Write fd_truncation_ggttg_seed4.txt: the events of the g g -> t t~ g
gradient workload (seed 4, first 1024 events) on which the two-point
central difference of f = w |M|^2 with h = 1e-6 misses the oracle's
reverse-mode gradient by more than 1e-6 (normwise), with that miss.

Calls only the oracle.  Usage: python tests/golden/make_fd_events.py
"""
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import me as orc  # noqa: E402
from oracle import rambo  # noqa: E402
from oracle.params import DEFAULT  # noqa: E402


def f_of_r(r):
    masses = orc.PROCESSES['ggttg'].final_masses(DEFAULT)
    p, w = rambo.event_momenta(r, DEFAULT.sqrts, masses)
    return orc.matrix_element('ggttg', p) * w


def main():
    n, h = 1024, 1e-6
    r, _, _ = orc.sample('ggttg', 4, 0, n)
    _, g, _ = orc.event_weight_and_grad('ggttg', r)
    fd = torch.zeros_like(r)
    for k in range(r.shape[1]):
        a, b = r.clone(), r.clone()
        a[:, k] += h
        b[:, k] -= h
        fd[:, k] = (f_of_r(a) - f_of_r(b)) / (2 * h)
    err = (fd - g).norm(dim=1) / g.norm(dim=1)
    bad = torch.nonzero(err > 1e-6).flatten().tolist()
    with open(os.path.join(HERE, 'fd_truncation_ggttg_seed4.txt'), 'w') as fh:
        fh.write("# g g -> t t~ g, seed 4, events 0..1023: two-point central differences\n"
                 "# (h = 1e-6) of f = w |M|^2 against the oracle's reverse-mode gradient,\n"
                 "# events missing by more than 1e-6 normwise.  Written by make_fd_events.py\n"
                 "# from the oracle only.\n# columns: event index, normwise miss\n")
        for i in bad:
            fh.write(f"{i} {float(err[i]):.6e}\n")


if __name__ == '__main__':
    torch.set_num_threads(4)
    main()
