"""Squared matrix elements, the sampling chain and its gradient (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Plain definition (Sec. II; readings R1, R13):
    ME(p) = (1/IDEN) sum_helicities sum_colours |M(p, hel, colours)|^2
with IDEN = (initial spin states) x (initial colour states) x (identical
final-particle factor) = 4 (e+e- -> mu+mu-), 4*64 = 256 (gg -> tt~,
gg -> tt~g), 4*64*2 = 512 (gg -> tt~gg), and the event weight
evtw = w_RAMBO * ME.  Every helicity is summed (no filtering).

Two colour treatments are offered for g g -> t t~ + n g:
* ``colour='dual'`` (default): dual amplitudes A_w from
  ``amplitudes.dual_amplitudes`` and the brute-force colour matrix C,
  sum_colours |M|^2 = sum_{w,w'} A_w C_{w w'} conj(A_w') -- the colour-flow
  quadratic form of Sec. II;
* ``colour='explicit'``: the amplitude for every one of the 8^n 3 3 colour
  basis assignments squared and summed (plain definition; small samples).
"""
import itertools
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import amplitudes as amp
from . import colour, philox, rambo
from .params import DEFAULT, WEIGHT_2PI, Params

F64 = torch.float64
C128 = torch.complex128


@dataclass(frozen=True)
class Process:
    name: str
    npar: int
    ngluon: int          # 0 for e+e- -> mu+mu-
    iden: int

    @property
    def nfinal(self):
        return self.npar - 2

    @property
    def nrnd(self):
        return 4 * self.nfinal

    def final_masses(self, prm):
        if self.name == 'eemumu':
            return [0.0, 0.0]
        return [prm.mt, prm.mt] + [0.0] * (self.npar - 4)


PROCESSES = {
    'eemumu': Process('eemumu', 4, 0, 4),
    'ggtt': Process('ggtt', 4, 2, 256),
    'ggttg': Process('ggttg', 5, 3, 256),
    'ggttgg': Process('ggttgg', 6, 4, 512),
}

_CMAT = {}


def colour_basis(ngluon, gluon_legs):
    """Orderings (as tuples of gluon legs) and the colour matrix over them."""
    if ngluon not in _CMAT:
        perms, C = colour.colour_matrix(ngluon)
        _CMAT[ngluon] = (perms, torch.tensor(C, dtype=F64))
    perms, C = _CMAT[ngluon]
    words = [tuple(gluon_legs[i] for i in perm) for perm in perms]
    return words, C


def _hel_tensors(npar):
    tab = np.array(amp.helicity_table(npar), dtype=np.float64)     # (H, npar)
    return [torch.tensor(tab[:, k], dtype=F64)[:, None] for k in range(npar)]


def me_per_helicity(proc, p, prm=DEFAULT, colour_mode='dual'):
    """sum_colours |M|^2 for every helicity: (2^npar, N) float64 (not /IDEN)."""
    proc = PROCESSES[proc] if isinstance(proc, str) else proc
    p = p.to(F64)
    hel = _hel_tensors(proc.npar)
    pb = p[None]                                                     # (1, N, npar, 4)
    if proc.name == 'eemumu':
        rows = []
        for h in amp.helicity_table(4):
            a = amp.amp_eemumu(p, h, prm)
            rows.append(a.real ** 2 + a.imag ** 2)
        return torch.stack(rows)
    legs = [0, 1] + list(range(4, proc.npar))
    if colour_mode == 'dual':
        A = amp.dual_amplitudes(pb, hel, prm)
        words, C = colour_basis(proc.ngluon, legs)
        Av = torch.stack([A[w] for w in words], dim=-1)              # (H, N, ncol)
        Cc = C.to(C128)
        quad = torch.einsum('hns,st,hnt->hn', Av, Cc, torch.conj(Av))
        return quad.real
    if colour_mode == 'explicit':
        if proc.ngluon == 2:
            cols = list(itertools.product(range(8), range(8), range(3), range(3)))
            rows = []
            for h in amp.helicity_table(proc.npar):
                a = amp.amp_ggtt_explicit(p, h, prm, cols)
                rows.append((a.real ** 2 + a.imag ** 2).sum(-1))
            return torch.stack(rows)
        # general n: batch over the colour basis states of every particle
        eye8 = torch.eye(8, dtype=C128)
        eye3 = torch.eye(3, dtype=C128)
        combos = list(itertools.product(*([range(8)] * proc.ngluon), range(3), range(3)))
        hel_b = [h[None] for h in hel]                               # (1, H, 1)
        total = 0
        for c0 in range(0, len(combos), 256):
            idx = torch.tensor(combos[c0:c0 + 256])
            gcol = {leg: eye8[idx[:, k]][:, None, None, :] for k, leg in enumerate(legs)}
            tcol = eye3[idx[:, -2]][:, None, None, :]
            tbcol = eye3[idx[:, -1]][:, None, None, :]
            a = amp.amp_full_colour(p[None, None], hel_b, prm, gcol, tcol, tbcol)
            total = total + (a.real ** 2 + a.imag ** 2).sum(0)
        return total
    raise ValueError(colour_mode)


def matrix_element(proc, p, prm=DEFAULT, colour_mode='dual', chunk=256):
    """ME per event, (N,) float64: helicity- and colour-summed |M|^2 / IDEN."""
    proc = PROCESSES[proc] if isinstance(proc, str) else proc
    outs = []
    for s in range(0, p.shape[0], chunk):
        ph = me_per_helicity(proc, p[s:s + chunk], prm, colour_mode)
        outs.append(ph.sum(0) / proc.iden)
    return torch.cat(outs) if outs else torch.zeros(0, dtype=F64)


def phase_space(proc, r, prm=DEFAULT):
    """RAMBO momenta (nevt, npar, 4) and weights (nevt,) for uniforms r;
    with the WEIGHT_2PI flag the weights carry (2 pi)^(4 - 3 nfinal)."""
    proc = PROCESSES[proc] if isinstance(proc, str) else proc
    p, w = rambo.event_momenta(r, prm.sqrts, proc.final_masses(prm))
    if prm.flags & WEIGHT_2PI:
        w = w * (2.0 * math.pi) ** (4 - 3 * proc.nfinal)
    return p, w


def sample(proc, seed, evt_offset, nevt, prm=DEFAULT):
    """Randoms (nevt, nrnd), momenta (nevt, npar, 4), weights (nevt,)."""
    proc = PROCESSES[proc] if isinstance(proc, str) else proc
    r = torch.from_numpy(philox.uniforms(seed, evt_offset, nevt, proc.nrnd))
    p, w = phase_space(proc, r, prm)
    return r, p, w


def event_weight_and_grad(proc, r, prm=DEFAULT):
    """f = ME(p(r)) w(r) per event and its reverse-mode derivatives.

    Returns (f, df/dr, dlogw/dr) with shapes (N,), (N, nrnd), (N, nrnd).
    Events are independent, so the gradient of the sum is the per-event
    gradient.  The Newton rescaling is differentiated through its converged
    iterations, which reproduces the implicit-function derivative up to the
    stopping tolerance.
    """
    proc = PROCESSES[proc] if isinstance(proc, str) else proc
    r = r.detach().to(F64).clone().requires_grad_(True)
    p, w = phase_space(proc, r, prm)
    me = matrix_element(proc, p, prm, chunk=max(1, r.shape[0]))
    f = me * w
    (gf,) = torch.autograd.grad(f.sum(), r, retain_graph=True)
    if w.requires_grad:
        (gw,) = torch.autograd.grad(torch.log(w).sum(), r)
    else:  # massless RAMBO: the weight depends on n and sqrt(s) only
        gw = torch.zeros_like(r)
    return f.detach(), gf, gw
