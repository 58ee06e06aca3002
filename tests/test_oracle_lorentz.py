"""Pins for the oracle's spinors and polarisation vectors (CPU only).

Textbook identities: Dirac equation, normalisation, completeness, helicity
eigenvalues, transversality of polarisation vectors.
"""
import math

import pytest
import torch

from oracle import lorentz as L

C = torch.complex128


def _momenta(m, n=64, seed=0):
    g = torch.Generator().manual_seed(seed)
    pv = (torch.rand(n, 3, generator=g, dtype=torch.float64) - 0.5) * 800.0
    # include the special directions: along -z, along +z and transverse
    pv[0] = torch.tensor([0.0, 0.0, -300.0], dtype=torch.float64)
    pv[1] = torch.tensor([0.0, 0.0, 300.0], dtype=torch.float64)
    pv[2] = torch.tensor([200.0, 0.0, 0.0], dtype=torch.float64)
    pv[3] = torch.tensor([1e-7, -2e-7, -300.0], dtype=torch.float64)
    E = torch.sqrt(m * m + (pv ** 2).sum(-1))
    return torch.cat([E[:, None], pv], dim=1)


@pytest.mark.parametrize("m", [0.0, 173.0])
@pytest.mark.parametrize("lam", [-1, 1])
def test_dirac_equation_and_norm(m, lam):
    p = _momenta(m)
    u = L.u_spinor(p, m, lam)
    v = L.v_spinor(p, m, lam)
    ps = L.slash(p)
    eye = torch.eye(4, dtype=C)
    scale = p[:, 0].max()
    assert torch.einsum('nab,nb->na', ps - m * eye, u).abs().max() < 1e-12 * scale ** 1.5
    assert torch.einsum('nab,nb->na', ps + m * eye, v).abs().max() < 1e-12 * scale ** 1.5
    ubu = torch.einsum('na,na->n', L.bar(u), u)
    vbv = torch.einsum('na,na->n', L.bar(v), v)
    assert torch.allclose(ubu, torch.full_like(ubu, 2 * m), atol=1e-10)
    assert torch.allclose(vbv, torch.full_like(vbv, -2 * m), atol=1e-10)
    # u^dagger u = 2E
    assert torch.allclose((u.conj() * u).sum(-1).real, 2 * p[:, 0], rtol=1e-13)


@pytest.mark.parametrize("m", [0.0, 173.0])
def test_completeness(m):
    p = _momenta(m)
    eye = torch.eye(4, dtype=C)
    su = sum(torch.einsum('na,nb->nab', L.u_spinor(p, m, l), L.bar(L.u_spinor(p, m, l)))
             for l in (-1, 1))
    sv = sum(torch.einsum('na,nb->nab', L.v_spinor(p, m, l), L.bar(L.v_spinor(p, m, l)))
             for l in (-1, 1))
    scale = p[:, 0].max()
    assert (su - (L.slash(p) + m * eye)).abs().max() < 1e-12 * scale
    assert (sv - (L.slash(p) - m * eye)).abs().max() < 1e-12 * scale


@pytest.mark.parametrize("lam", [-1, 1])
def test_helicity_eigenstates(lam):
    m = 173.0
    p = _momenta(m)
    phat = p[:, 1:] / p[:, 1:].norm(dim=-1, keepdim=True)
    # spin operator Sigma.p^ = diag(sigma.p^, sigma.p^)
    sp = sum(phat[:, k, None, None].to(C) * L.SIGMA[k] for k in range(3))
    z = torch.zeros_like(sp)
    Sig = torch.cat([torch.cat([sp, z], -1), torch.cat([z, sp], -1)], -2)
    u = L.u_spinor(p, m, lam)
    assert (torch.einsum('nab,nb->na', Sig, u) - lam * u).abs().max() < 1e-10
    # antiparticle of helicity lam: v carries spin projection -lam
    v = L.v_spinor(p, m, lam)
    assert (torch.einsum('nab,nb->na', Sig, v) + lam * v).abs().max() < 1e-10


def test_massless_chirality_exact_zeros():
    p = _momenta(0.0)
    up = L.u_spinor(p, 0.0, 1)
    um = L.u_spinor(p, 0.0, -1)
    assert (up[:, :2] == 0).all() and (um[:, 2:] == 0).all()
    vp = L.v_spinor(p, 0.0, 1)
    vm = L.v_spinor(p, 0.0, -1)
    assert (vp[:, 2:] == 0).all() and (vm[:, :2] == 0).all()


@pytest.mark.parametrize("lam", [-1, 1])
def test_polarisation_vectors(lam):
    k = _momenta(0.0)
    e = L.polarisation(k, lam)
    assert (L.mdot(k.to(C), e)).abs().max() < 1e-11
    assert torch.allclose(L.mdot(e, e.conj()).real, torch.full((k.shape[0],), -1.0,
                                                               dtype=torch.float64), atol=1e-14)
    # helicity: i k^ x eps = lam eps (spatial parts), and eps^0 = 0
    kh = (k[:, 1:] / k[:, 1:].norm(dim=-1, keepdim=True)).to(C)
    cross = torch.linalg.cross(kh, e[:, 1:])
    assert (1j * cross - lam * e[:, 1:]).abs().max() < 1e-13
    assert (e[:, 0] == 0).all()
    other = L.polarisation(k, -lam)
    assert L.mdot(e, other.conj()).abs().max() < 1e-14


def test_polarisation_along_z_textbook():
    k = torch.tensor([[10.0, 0, 0, 10.0]], dtype=torch.float64)
    s2 = 1 / math.sqrt(2)
    assert torch.allclose(L.polarisation(k, 1)[0],
                          torch.tensor([0, -s2, -1j * s2, 0], dtype=C))
    assert torch.allclose(L.polarisation(k, -1)[0],
                          torch.tensor([0, s2, -1j * s2, 0], dtype=C))
