"""Pins for the oracle's matrix elements and gradient (CPU only).

What fixes each part:
* e+e- -> mu+mu-: the photon + Z closed form; exactly 4 of 16 helicities
  nonzero for massless leptons (Sec. II, Fig. 1).
* g g -> t t~: the textbook LO closed form (zero top width), and the three
  written-out diagrams with an explicit colour sum.
* g g -> t t~ g (g): the dual-amplitude form against the plain colour-dressed
  recursion (explicit colour sum; random colour states), the gluon Ward
  identity per dual amplitude, Lorentz invariance, Bose and charge-conjugation
  symmetry, the number of diagrams.
* the gradient: central finite differences.
"""
import math

import numpy as np
import pytest
import torch

import closed_forms as cf
from oracle import amplitudes as A
from oracle import colour, me, rambo
from oracle.params import DEFAULT

F64 = torch.float64
C128 = torch.complex128
NOWIDTH = DEFAULT.with_(wt=0.0)


def _rel(a, b):
    return float(((a - b).abs() / b.abs()).max())


def test_diagram_counts():
    assert [A.count_diagrams(n) for n in (2, 3, 4)] == [3, 16, 123]


def test_eemumu_closed_form_and_helicities():
    p = _two_to_two(512, 0.0, 4)
    got = me.matrix_element('eemumu', p)
    want = torch.from_numpy(cf.eemumu(p.numpy(), DEFAULT.alpha_inv, DEFAULT.mZ, DEFAULT.wZ,
                                      DEFAULT.sw2))
    assert _rel(got, want) < 1e-13
    ph = me.me_per_helicity('eemumu', p)
    nonzero = (ph != 0).any(dim=1)
    assert int(nonzero.sum()) == 4
    # QED value at 90 degrees in the e-/mu- plane: e^4 (1 + cos^2) with cos = 0
    e4 = (4 * math.pi / DEFAULT.alpha_inv) ** 2
    assert e4 == pytest.approx(0.0089947, abs=5e-8)


def _two_to_two(n, m, seed):
    """On-shell 2 -> 2 events at sqrt(s) = 1500 from seeded angles (exact
    kinematics, no sampler rounding)."""
    g = torch.Generator().manual_seed(seed)
    E = 750.0
    P = math.sqrt(E * E - m * m)
    c = 2 * torch.rand(n, generator=g, dtype=F64) - 1
    ph = 2 * math.pi * torch.rand(n, generator=g, dtype=F64)
    st = torch.sqrt(1 - c * c)
    d = torch.stack([st * torch.cos(ph), st * torch.sin(ph), c], dim=-1)
    p = torch.zeros(n, 4, 4, dtype=F64)
    p[:, 0] = torch.tensor([E, 0.0, 0.0, E], dtype=F64)
    p[:, 1] = torch.tensor([E, 0.0, 0.0, -E], dtype=F64)
    p[:, 2, 0] = E
    p[:, 2, 1:] = P * d
    p[:, 3, 0] = E
    p[:, 3, 1:] = -P * d
    return p


def test_ggtt_closed_form():
    p = _two_to_two(512, NOWIDTH.mt, 3)
    got = me.matrix_element('ggtt', p, NOWIDTH)
    want = torch.from_numpy(cf.ggQQ(p.numpy(), NOWIDTH.gs, NOWIDTH.mt))
    assert _rel(got, want) < 1e-13
    # on sampled events the tops are off shell by the sampler's rounding,
    # which the t-channel propagators see at the 1e-12 level
    r, p, w = me.sample('ggtt', 1, 0, 512, NOWIDTH)
    got = me.matrix_element('ggtt', p, NOWIDTH)
    want = torch.from_numpy(cf.ggQQ(p.numpy(), NOWIDTH.gs, NOWIDTH.mt))
    assert _rel(got, want) < 1e-11


def test_ggtt_closed_form_at_90_degrees():
    # theta = 90 degrees: tau1 = tau2 = 1/2
    p = _two_to_two(1, NOWIDTH.mt, 0)
    P = p[0, 2, 1:].norm()
    p[0, 2, 1:] = torch.tensor([P, 0, 0], dtype=F64)
    p[0, 3, 1:] = torch.tensor([-P, 0, 0], dtype=F64)
    got = float(me.matrix_element('ggtt', p, NOWIDTH)[0])
    rho = 4 * 173.0 ** 2 / 1500.0 ** 2
    want = NOWIDTH.gs ** 4 * (1 / 1.5 - 3 / 8) * (0.5 + rho - rho * rho)
    assert got == pytest.approx(want, rel=1e-14)


def test_ggtt_explicit_diagrams_vs_dual():
    r, p, w = me.sample('ggtt', 1, 0, 16)
    a = me.matrix_element('ggtt', p, colour_mode='dual')
    b = me.matrix_element('ggtt', p, colour_mode='explicit')
    assert _rel(a, b) < 1e-13


def test_colour_matrices():
    for n, den, diag in ((2, 3, 16), (3, 9, 64), (4, 54, 512)):
        perms, Cm = colour.colour_matrix(n)
        R = colour.rationalise(Cm)
        assert np.allclose(Cm, Cm.T, atol=0, rtol=0)
        assert np.linalg.eigvalsh(Cm).min() > 0
        # diagonal: sum_a Tr(T^a1..T^an T^an..T^a1) = N C_F^n
        assert all(R[i][i] * den == diag for i in range(len(R)))
        assert all((R[i][j] * den).denominator == 1 for i in range(len(R)) for j in range(len(R)))
    # textbook 2-gluon matrix (1/3) [[16, -2], [-2, 16]]
    _, C2 = colour.colour_matrix(2)
    assert np.allclose(C2 * 3, [[16, -2], [-2, 16]], atol=1e-12)


@pytest.mark.slow
def test_ggttg_dual_vs_explicit_colour_sum():
    r, p, w = me.sample('ggttg', 2, 0, 1)
    a = me.matrix_element('ggttg', p, colour_mode='dual')
    b = me.matrix_element('ggttg', p, colour_mode='explicit')
    assert _rel(a, b) < 1e-13


@pytest.mark.parametrize("proc,ng", [('ggttg', 3), ('ggttgg', 4)])
def test_dual_decomposition_random_colour_states(proc, ng):
    """Full colour-dressed amplitude = sum_w (c_t T^w c_tb) A_w for random
    complex colour wavefunctions, helicity by helicity."""
    g = torch.Generator().manual_seed(17)

    def rc(n):
        return torch.complex(torch.randn(n, generator=g, dtype=F64),
                             torch.randn(n, generator=g, dtype=F64))

    r, p, w = me.sample(proc, 5, 0, 2)
    npar = p.shape[1]
    legs = [0, 1] + list(range(4, npar))
    gcol = {l: rc(8) for l in legs}
    tcol, tbcol = rc(3), rc(3)
    T = torch.tensor(colour.T, dtype=C128)
    for hel in A.helicity_table(npar)[::7]:
        full = A.amp_full_colour(p, hel, DEFAULT, gcol, tcol, tbcol)
        dual = A.dual_amplitudes(p, hel, DEFAULT)
        rec = 0
        for word, aw in dual.items():
            m = torch.eye(3, dtype=C128)
            for l in word:
                m = m @ torch.einsum('a,aij->ij', gcol[l], T)
            rec = rec + aw * (tcol @ m @ tbcol)
        assert _rel(rec, full) < 1e-12


@pytest.mark.parametrize("proc", ['ggttg', 'ggttgg'])
def test_ward_identity_per_dual_amplitude(proc):
    """eps_j -> k_j for one gluon makes every dual amplitude vanish."""
    r, p, w = me.sample(proc, 6, 0, 3, NOWIDTH)
    npar = p.shape[1]
    for leg in (0, 4):
        for hel in A.helicity_table(npar)[::11]:
            phys = A.dual_amplitudes(p, hel, NOWIDTH)
            ward = A.dual_amplitudes(p, hel, NOWIDTH, override={leg: p[:, leg]})
            scale = max(float(v.abs().max()) for v in phys.values())
            worst = max(float(v.abs().max()) for v in ward.values())
            # normalised by the physical amplitudes times the gluon energy
            assert worst < 1e-12 * scale * float(p[:, leg, 0].max())


def _boost(p, beta):
    b = torch.as_tensor(beta, dtype=F64)
    b2 = float(b @ b)
    gam = 1 / math.sqrt(1 - b2)
    bp = p[..., 1:] @ b
    E = gam * (p[..., 0] + bp)
    v = p[..., 1:] + ((gam - 1) * bp / b2 + gam * p[..., 0])[..., None] * b
    return torch.cat([E[..., None], v], dim=-1)


def _rotate(p, axis, ang):
    k = torch.as_tensor(axis, dtype=F64)
    k = k / k.norm()
    v = p[..., 1:]
    c, s = math.cos(ang), math.sin(ang)
    vr = v * c + torch.linalg.cross(k.expand_as(v), v) * s + k * (v @ k)[..., None] * (1 - c)
    return torch.cat([p[..., :1], vr], dim=-1)


@pytest.mark.parametrize("proc", ['ggtt', 'ggttg', 'ggttgg'])
def test_lorentz_invariance(proc):
    # zero top width: a width in t-channel propagators breaks the Ward
    # identity, and with it the frame independence of the helicity sum
    r, p, w = me.sample(proc, 7, 0, 8, NOWIDTH)
    a = me.matrix_element(proc, p, NOWIDTH)
    pb = _rotate(_boost(p, [0.3, -0.5, 0.6]), [1.0, 2.0, 0.5], 0.7)
    b = me.matrix_element(proc, pb, NOWIDTH)
    assert _rel(b, a) < 1e-11


@pytest.mark.parametrize("proc", ['ggttg', 'ggttgg'])
def test_bose_and_charge_conjugation(proc):
    r, p, w = me.sample(proc, 8, 0, 8)
    a = me.matrix_element(proc, p)
    swap_in = p[:, [1, 0] + list(range(2, p.shape[1]))]
    swap_q = p[:, [0, 1, 3, 2] + list(range(4, p.shape[1]))]
    assert _rel(me.matrix_element(proc, swap_in), a) < 1e-12
    assert _rel(me.matrix_element(proc, swap_q), a) < 1e-12
    if proc == 'ggttgg':
        swap_out = p[:, [0, 1, 2, 3, 5, 4]]
        assert _rel(me.matrix_element(proc, swap_out), a) < 1e-12


def test_width_only_shifts_slightly():
    r, p, w = me.sample('ggttg', 2, 0, 16)
    a = me.matrix_element('ggttg', p, DEFAULT)
    b = me.matrix_element('ggttg', p, NOWIDTH)
    assert 0 < _rel(a, b) < 1e-2


def test_gradient_vs_finite_differences():
    r, p, w = me.sample('ggttg', 4, 0, 6)
    f, gf, gw = me.event_weight_and_grad('ggttg', r)
    masses = me.PROCESSES['ggttg'].final_masses(DEFAULT)
    h = 1e-6
    fd = torch.zeros_like(gf)
    fdw = torch.zeros_like(gw)
    for k in range(r.shape[1]):
        rp, rm = r.clone(), r.clone()
        rp[:, k] += h
        rm[:, k] -= h
        pp, wp = rambo.event_momenta(rp, DEFAULT.sqrts, masses)
        pm, wm = rambo.event_momenta(rm, DEFAULT.sqrts, masses)
        fd[:, k] = (me.matrix_element('ggttg', pp) * wp - me.matrix_element('ggttg', pm) * wm) / (2 * h)
        fdw[:, k] = (torch.log(wp) - torch.log(wm)) / (2 * h)
    assert float(((gf - fd).norm(dim=1) / fd.norm(dim=1)).max()) < 1e-6
    assert float(((gw - fdw).norm(dim=1) / fdw.norm(dim=1)).max()) < 1e-6


def test_full_colour_recursion_reduces_to_written_out_ggtt():
    """The colour-dressed recursion at n = 2 equals the three written-out
    g g -> t t~ diagrams for every explicit colour state, helicity by
    helicity, and its explicit colour sum equals the textbook closed form
    (zero top width, exactly on-shell kinematics)."""
    p = _two_to_two(6, NOWIDTH.mt, 11)
    cols = list(__import__('itertools').product(range(8), range(8), range(3), range(3)))
    eye8 = torch.eye(8, dtype=C128)
    eye3 = torch.eye(3, dtype=C128)
    idx = torch.tensor(cols)
    gcol = {0: eye8[idx[:, 0]][:, None, :], 1: eye8[idx[:, 1]][:, None, :]}
    tcol = eye3[idx[:, 2]][:, None, :]
    tbcol = eye3[idx[:, 3]][:, None, :]
    recs, wos = [], []
    for hel in A.helicity_table(4):
        recs.append(A.amp_full_colour(p[None], hel, NOWIDTH, gcol, tcol, tbcol))  # (576, N)
        wos.append(A.amp_ggtt_explicit(p, hel, NOWIDTH, cols).T)                  # (576, N)
    rec, wo = torch.stack(recs), torch.stack(wos)
    # relative to the largest amplitude of the event (some helicities vanish)
    scale = wo.abs().amax(dim=(0, 1))
    assert float(((rec - wo).abs().amax(dim=(0, 1)) / scale).max()) <= 1e-13
    total = (rec.real ** 2 + rec.imag ** 2).sum(dim=(0, 1))
    want = torch.from_numpy(cf.ggQQ(p.numpy(), NOWIDTH.gs, NOWIDTH.mt))
    assert _rel(total / 256.0, want) < 1e-13
