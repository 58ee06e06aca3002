"""The general amplitude bodies of the SIGMAKIN kernels (GPU).

Every SIGMAKIN kernel holds the amplitude body twice: for events whose
incoming momenta are (E,0,0,E) and (E,0,0,-E), as RAMBO writes them, with
those zero components as compile-time constants, and for any other momenta.
The RAMBO-based parity tests run the first; these run the second, on the
oracle's events rotated in space or boosted along z, with whole waves of
events in RAMBO's frame and waves that mix the two, against the oracle on the
same momenta.  With a top width in the t-channel propagators |M|^2 depends on
the frame (the Ward identity is broken), so each side is evaluated on the
identical transformed momenta rather than compared with the untransformed
result.
"""
import math
import sys

import pytest
import torch

from oracle import me as orc

pytestmark = pytest.mark.gpu

F64 = torch.float64
SEED = {'eemumu': 0, 'ggtt': 1, 'ggttg': 2, 'ggttgg': 3}
SMALL = {'eemumu': 4096 + 17, 'ggtt': 2048 + 33, 'ggttg': 640 + 5, 'ggttgg': 192 + 7}
# events [0, KEEP) stay in RAMBO's frame: two whole waves on the beam body
KEEP = 128


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as m
    m.lib()
    return m


def transformed(p, seed):
    """Events [0, KEEP) unchanged, then in turn unchanged, rotated about a
    random axis by a random angle, boosted along z with rapidity in (-1, 1)
    (the beams stay on the axis but with unequal energies).  Returns the
    momenta and the kind of each event (0 unchanged, 1 rotated, 2 boosted)."""
    n = p.shape[0]
    g = torch.Generator().manual_seed(seed)
    kind = torch.zeros(n, dtype=torch.long)
    kind[KEEP:] = torch.arange(n - KEEP) % 3
    q = p.clone()
    axis = torch.randn(n, 3, generator=g, dtype=F64)
    axis = axis / axis.norm(dim=1, keepdim=True)
    ang = 2 * math.pi * torch.rand(n, generator=g, dtype=F64)
    y = 2 * torch.rand(n, generator=g, dtype=F64) - 1
    r = kind == 1
    if r.any():
        k = axis[r][:, None, :].expand(-1, p.shape[1], -1)
        v = p[r][..., 1:]
        c = torch.cos(ang[r])[:, None, None]
        s = torch.sin(ang[r])[:, None, None]
        vr = v * c + torch.linalg.cross(k, v, dim=-1) * s + k * (v * k).sum(-1, keepdim=True) * (1 - c)
        q[r, :, 1:] = vr
    b = kind == 2
    if b.any():
        ch = torch.cosh(y[b])[:, None]
        sh = torch.sinh(y[b])[:, None]
        E, pz = p[b][..., 0], p[b][..., 3]
        q[b, :, 0] = E * ch + pz * sh
        q[b, :, 3] = pz * ch + E * sh
    return q, kind


def rel(a, b):
    return (a - b).abs() / b.abs()


CASES = [(proc, 'fp64') for proc in SEED] + \
        [(proc, 'fp32amp') for proc in ('ggtt', 'ggttg', 'ggttgg')] + \
        [(proc, 'mixed') for proc in SEED]


@pytest.mark.parametrize('proc,prec', CASES)
def test_general_body_against_the_oracle(mg, proc, prec):
    n = SMALL[proc]
    _, p, _ = orc.sample(proc, SEED[proc], 0, n)
    q, kind = transformed(p, 100 + SEED[proc])
    want = orc.matrix_element(proc, q)
    say('frames', proc, prec, n)
    e = mg.MEEngine(proc, prec)
    got = e.sigmakin(e.events_mom(q), n).cpu()
    err = rel(got, want)
    tol = 1e-12 if prec == 'fp64' else 1e-5
    for k, name in enumerate(('beam frame', 'rotated', 'boosted along z')):
        ek = err[kind == k]
        say(proc, prec, name, int(ek.numel()), 'max rel', float(ek.max()))
        assert float(ek.max()) <= tol
    # the beam-frame events agree with the untransformed launch, whose waves
    # all take the beam body
    base = e.sigmakin(e.events_mom(p), n).cpu()
    same = kind == 0
    assert float(rel(got[same], base[same]).max()) <= (1e-13 if prec == 'fp64' else 1e-6)


def test_general_body_event_per_lane_full_waves(mg):
    """A launch above the group threshold of g g -> t t~ g (event per lane)
    with transformed events: the oracle on the first and last 64 events and
    64 seeded others."""
    n = (1 << 16) + 37
    e = mg.MEEngine('ggttg', 'fp64')
    say('frames event per lane', n)
    _, mom, _ = e.sample(SEED['ggttg'], n)
    p = e.mom_events(mom, n).cpu()
    q, kind = transformed(p, 7)
    me = e.sigmakin(e.events_mom(q), n)
    torch.cuda.synchronize()
    assert e.count_nonfinite(me) == 0
    g = torch.Generator().manual_seed(n)
    idx = sorted(set(list(range(64)) + list(range(n - 64, n)) +
                     torch.randint(0, n, (64,), generator=g).tolist()))
    got = me[torch.tensor(idx, device=me.device)].cpu()
    want = orc.matrix_element('ggttg', q[idx])
    assert float(rel(got, want).max()) <= 1e-12
