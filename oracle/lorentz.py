"""Explicit Dirac algebra, helicity spinors and polarisation vectors (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Implements the "external particle" objects of the helicity-amplitude method
(Sec. II, Fig. 1: IXXXXX/OXXXXX and their vector analogue) from the
textbook definitions (Peskin & Schroeder ch. 3; HELAS manual KEK-91-11), as
explicit 4-component objects:

* metric diag(+,-,-,-); momenta (E, px, py, pz);
* chiral (Weyl) representation: gamma^0 = [[0,1],[1,0]],
  gamma^k = [[0,sigma^k],[-sigma^k,0]], gamma^5 = diag(-1,-1,1,1), so the
  upper two components are left-handed;
* two-component helicity states chi_lambda(p^) with (sigma.p^) chi = lambda chi;
* u(p,l) = (sqrt(E - l|p|) chi_l, sqrt(E + l|p|) chi_l),
  v(p,l) = (sqrt(E + l|p|) chi_-l, -sqrt(E - l|p|) chi_-l),
  with E - l|p| taken as exactly 0 for a massless fermion of helicity +1
  (reading R15: massless spinors have exact zeros in the other chirality);
* eps(k, l) = (-l e1 - i e2)/sqrt(2) with e1 = (0, cos th cos ph,
  cos th sin ph, -sin th), e2 = (0, -sin ph, cos ph, 0); eps* for outgoing.
Directions along -z (p + pz = 0) use the limit th = pi, ph = 0.
All functions act on batched float64/complex128 torch tensors (..., 4).
"""
import math
import torch

C128 = torch.complex128
F64 = torch.float64

METRIC = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)

_I2 = torch.eye(2, dtype=C128)
_Z2 = torch.zeros(2, 2, dtype=C128)
SIGMA = [
    torch.tensor([[0, 1], [1, 0]], dtype=C128),
    torch.tensor([[0, -1j], [1j, 0]], dtype=C128),
    torch.tensor([[1, 0], [0, -1]], dtype=C128),
]


def _block(a, b, c, d):
    return torch.cat([torch.cat([a, b], 1), torch.cat([c, d], 1)], 0)


GAMMA = torch.stack([_block(_Z2, _I2, _I2, _Z2)]
                    + [_block(_Z2, s, -s, _Z2) for s in SIGMA])      # gamma^mu
GAMMA5 = torch.diag(torch.tensor([-1, -1, 1, 1], dtype=C128))
PL = (torch.eye(4, dtype=C128) - GAMMA5) / 2
PR = (torch.eye(4, dtype=C128) + GAMMA5) / 2


def mdot(a, b):
    """Minkowski product a.b = a^0 b^0 - a.b (bilinear, no conjugation)."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] \
        - a[..., 3] * b[..., 3]


def slash(v):
    """v-slash = gamma^mu v_mu = gamma^mu g_{mu nu} v^nu, shape (..., 4, 4)."""
    vl = v.to(C128) * METRIC.to(C128)
    return torch.einsum('...m,mab->...ab', vl, GAMMA)


def _lam(lam, like):
    """Helicity as a float64 tensor broadcastable against like[..., 0]."""
    return torch.as_tensor(lam, dtype=F64)


def _chi(p, lam):
    """Two-component helicity eigenstate chi_lam for the direction of p.

    p: real (..., 4); lam: +-1 (int or tensor broadcastable to p[..., 0]).
    Uses P + pz = pT^2/(P - pz) for pz < 0 (no cancellation) and the
    th = pi, ph = 0 limit where P + pz = 0.
    """
    px, py, pz = p[..., 1], p[..., 2], p[..., 3]
    P = torch.sqrt(px * px + py * py + pz * pz)
    pt2 = px * px + py * py
    ppz = torch.where(pz >= 0, P + pz, pt2 / torch.where(P - pz > 0, P - pz, 1.0))
    along_mz = ppz <= 0
    safe = torch.where(along_mz, 1.0, ppz)
    nrm = torch.where(along_mz, 1.0, torch.sqrt(2.0 * P * safe))
    pxy = torch.complex(px, py)
    one = torch.ones_like(P).to(C128)
    zero = torch.zeros_like(P).to(C128)
    # lam = +1: (cos th/2, e^{i ph} sin th/2); lam = -1: (-e^{-i ph} sin th/2, cos th/2)
    ap = torch.where(along_mz, zero, safe.to(C128) / nrm)
    bp = torch.where(along_mz, one, pxy / nrm)
    am = torch.where(along_mz, -one, -torch.conj(pxy) / nrm)
    bm = torch.where(along_mz, zero, safe.to(C128) / nrm)
    pos = _lam(lam, P) > 0
    return torch.stack([torch.where(pos, ap, am), torch.where(pos, bp, bm)], dim=-1)


def _omegas(p, m, lam):
    """(sqrt(E - lam P), sqrt(E + lam P)); E - P = m^2/(E + P) for stability."""
    E = p[..., 0]
    P = torch.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2 + p[..., 3] ** 2)
    epp = E + P
    emp = (m * m) / epp if m != 0.0 else torch.zeros_like(E)
    s_emp, s_epp = torch.sqrt(emp), torch.sqrt(epp)
    pos = _lam(lam, E) > 0
    return torch.where(pos, s_emp, s_epp), torch.where(pos, s_epp, s_emp)


def u_spinor(p, m, lam):
    wm, wp = _omegas(p, m, lam)
    chi = _chi(p, lam)
    return torch.cat([wm[..., None] * chi, wp[..., None] * chi], dim=-1)


def v_spinor(p, m, lam):
    # sqrt(E + lam P) multiplies the upper (left) part, -sqrt(E - lam P) the lower.
    wm, wp = _omegas(p, m, lam)
    chi = _chi(p, -_lam(lam, p[..., 0]))
    return torch.cat([wp[..., None] * chi, -wm[..., None] * chi], dim=-1)


def bar(psi):
    """Dirac adjoint psi^dagger gamma^0 as a row spinor (..., 4)."""
    return torch.einsum('...a,ab->...b', torch.conj(psi), GAMMA[0])


def polarisation(k, lam):
    """eps^mu(k, lam) for a massless vector of momentum k (contravariant)."""
    kx, ky, kz = k[..., 1], k[..., 2], k[..., 3]
    K = torch.sqrt(kx * kx + ky * ky + kz * kz)
    kt = torch.sqrt(kx * kx + ky * ky)
    cth = kz / K
    sth = kt / K
    has_t = kt > 0
    cph = torch.where(has_t, kx / torch.where(has_t, kt, 1.0), 1.0)
    sph = torch.where(has_t, ky / torch.where(has_t, kt, 1.0), 0.0)
    zero = torch.zeros_like(K)
    e1 = torch.stack([zero, cth * cph, cth * sph, -sth], dim=-1).to(C128)
    e2 = torch.stack([zero, -sph, cph, zero], dim=-1).to(C128)
    lam = _lam(lam, K)[..., None]
    return (-lam * e1 - 1j * e2) / math.sqrt(2.0)


def fermion_propagator(q, m, w):
    """i (q-slash + m) / (q^2 - m^2 + i m w), shape (..., 4, 4)."""
    den = mdot(q, q).to(C128) - m * m + 1j * m * w
    num = slash(q) + m * torch.eye(4, dtype=C128)
    return 1j * num / den[..., None, None]
