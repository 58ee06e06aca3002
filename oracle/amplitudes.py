"""Tree-level helicity amplitudes from Feynman rules (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Feynman rules (Peskin & Schroeder conventions, metric (+,-,-,-)), all
momenta entering a vertex counted as incoming:
  f f V vertex          i gamma^mu (cL P_L + cR P_R)
      photon             cL = cR = -e Q_f
      Z                  cL = -(e/(sW cW)) gL, cR = -(e/(sW cW)) gR,
                         gL = T3 - Q sW^2, gR = -Q sW^2
      gluon              i g_s gamma^mu T^a
  g g g   (a,mu,k1)(b,nu,k2)(c,rho,k3)
                         g_s f^{abc} [g^{mu nu}(k1-k2)^rho + g^{nu rho}(k2-k3)^mu
                                      + g^{rho mu}(k3-k1)^nu]
  g g g g (a,mu)(b,nu)(c,rho)(d,sig)
                         -i g_s^2 [f^{abe}f^{cde}(g^{mu rho}g^{nu sig} - g^{mu sig}g^{nu rho})
                                 + f^{ace}f^{bde}(g^{mu nu}g^{rho sig} - g^{mu sig}g^{nu rho})
                                 + f^{ade}f^{bce}(g^{mu nu}g^{rho sig} - g^{mu rho}g^{nu sig})]
  propagators            photon -i g/q^2, gluon -i g delta/q^2 (Feynman gauge),
                         Z -i (g - q q/mZ^2)/(q^2 - mZ^2 + i mZ GZ) (unitary gauge),
                         top i (q-slash + m)/(q^2 - m^2 + i m Gt) (reading R5).
Each function returns i M (an overall phase does not affect |M|^2).

Processes and particle order (reading R7): e+ e- -> mu+ mu- (the two
s-channel diagrams of Fig. 1); g g -> t t~ (g)(g) with legs
0, 1 = incoming gluons along +z / -z, 2 = t, 3 = t~, 4, 5 = outgoing gluons.
"""
import itertools

import numpy as np
import torch

from . import colour
from .lorentz import (C128, F64, PL, PR, GAMMA, bar, fermion_propagator, mdot,
                      polarisation, slash, u_spinor, v_spinor)

_F = torch.tensor(colour.F, dtype=C128)
_T = torch.tensor(colour.T, dtype=C128)
_FF1 = torch.einsum('abe,cde->abcd', _F, _F)
_FF2 = torch.einsum('ace,bde->abcd', _F, _F)
_FF3 = torch.einsum('ade,bce->abcd', _F, _F)


def helicity_table(npar):
    """All 2^npar helicity combinations; particle 0 is the slowest index and
    helicity -1 precedes +1."""
    return [tuple(-1 if ((h >> (npar - 1 - k)) & 1) == 0 else 1 for k in range(npar))
            for h in range(2 ** npar)]


# --------------------------------------------------------------------------
# e+ e- -> mu+ mu-
# --------------------------------------------------------------------------

def amp_eemumu(p, hel, prm):
    """i M for e+(p0) e-(p1) -> mu+(p2) mu-(p3), massless leptons.

    p: (N, 4, 4) float64; hel: 4 helicities.  Sums the photon and Z
    s-channel diagrams of Fig. 1 with explicit Dirac matrices.
    """
    e = prm.e
    sw2 = prm.sw2
    sw, cw = np.sqrt(sw2), np.sqrt(1.0 - sw2)
    Q, T3 = -1.0, -0.5
    vb1 = bar(v_spinor(p[:, 0], 0.0, hel[0]))      # incoming e+
    u2 = u_spinor(p[:, 1], 0.0, hel[1])            # incoming e-
    v3 = v_spinor(p[:, 2], 0.0, hel[2])            # outgoing mu+
    ub4 = bar(u_spinor(p[:, 3], 0.0, hel[3]))      # outgoing mu-
    q = p[:, 0] + p[:, 1]
    q2 = mdot(q, q).to(C128)
    couplings = {
        'photon': (-e * Q, -e * Q),
        'Z': (-(e / (sw * cw)) * (T3 - Q * sw2), -(e / (sw * cw)) * (-Q * sw2)),
    }

    def current(rowsp, colsp, cL, cR):
        # J^mu = rowsp gamma^mu (cL PL + cR PR) colsp, contravariant mu
        chir = cL * PL + cR * PR
        mats = torch.einsum('mab,bc->mac', GAMMA, chir)
        return torch.einsum('na,mab,nb->nm', rowsp, mats, colsp)

    metric = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)
    total = torch.zeros(p.shape[0], dtype=C128)
    for name, (cL, cR) in couplings.items():
        je = 1j * current(vb1, u2, cL, cR)
        jm = 1j * current(ub4, v3, cL, cR)
        jdot = (je * jm * metric).sum(-1)
        if name == 'photon':
            total = total + (-1j / q2) * jdot
        else:
            qc = q.to(C128) * metric                     # q_mu
            qje = (qc * je).sum(-1)
            qjm = (qc * jm).sum(-1)
            den = q2 - prm.mZ ** 2 + 1j * prm.mZ * prm.wZ
            total = total + (-1j / den) * (jdot - qje * qjm / prm.mZ ** 2)
    return total


# --------------------------------------------------------------------------
# external states for g g -> t t~ + n g
# --------------------------------------------------------------------------

def qcd_externals(p, hel, mt, override=None):
    """Wavefunctions and incoming momenta for g g -> t t~ + n g.

    Returns (gluons, ubar_t, v_tb, p_t) where gluons is a list of
    (label, eps, k) with k the momentum flowing into the diagram.
    p: (..., npar, 4); hel: helicity per particle (ints or tensors broadcast).
    override: optional dict leg -> 4-vector replacing that gluon's
    polarisation (used for the Ward identity, eps -> k).
    """
    npar = p.shape[-2]
    gl = []
    for leg in [0, 1] + list(range(4, npar)):
        pk = p[..., leg, :]
        if override is not None and leg in override:
            eps = override[leg].to(C128)
        elif leg < 2:
            eps = polarisation(pk, hel[leg])
        else:
            eps = torch.conj(polarisation(pk, hel[leg]))
        gl.append((leg, eps, pk if leg < 2 else -pk))
    ubt = bar(u_spinor(p[..., 2, :], mt, hel[2]))
    vtb = v_spinor(p[..., 3, :], mt, hel[3])
    return gl, ubt, vtb, p[..., 2, :]


def _v3(j1, k1, j2, k2):
    """Lorentz part of the 3-gluon vertex contracted with two currents,
    legs (out, j1, j2); the out leg has incoming momentum -(k1+k2)."""
    return (j1 * mdot(-(2 * k1 + k2), j2)[..., None]
            + mdot(j1, j2)[..., None] * (k1 - k2)
            + j2 * mdot(k1 + 2 * k2, j1)[..., None])


def amp_ggtt_explicit(p, hel, prm, colours):
    """i M for g g -> t t~ written out as its three Feynman diagrams.

    colours: iterable of (a1, a2, i, j).  Returns (N, ncolours) complex.
    """
    g = prm.gs
    gl, ubt, vtb, p3 = qcd_externals(p, hel, prm.mt)
    (_, e1, k1), (_, e2, k2) = gl
    # both top propagators separate the two incoming gluons: t-channel
    S13 = fermion_propagator(p3 - k1, prm.mt, prm.top_width(True))
    S23 = fermion_propagator(p3 - k2, prm.mt, prm.top_width(True))
    # t-channel: gluon 0 next to the top
    L1 = torch.einsum('na,nab,nbc,ncd,nd->n', ubt, 1j * g * slash(e1), S13,
                      1j * g * slash(e2), vtb)
    L2 = torch.einsum('na,nab,nbc,ncd,nd->n', ubt, 1j * g * slash(e2), S23,
                      1j * g * slash(e1), vtb)
    # s-channel: three-gluon vertex, gluon propagator, quark vertex
    V = g * _v3(e1, k1, e2, k2)
    s = mdot(k1 + k2, k1 + k2).to(C128)
    L3 = (-1j / s) * torch.einsum('na,nab,nb->n', ubt, 1j * g * slash(V), vtb)
    out = []
    T = _T
    for (a1, a2, i, j) in colours:
        c1 = (T[a1] @ T[a2])[i, j]
        c2 = (T[a2] @ T[a1])[i, j]
        c3 = sum(_F[a1, a2, c] * T[c][i, j] for c in range(8))
        out.append(L1 * c1 + L2 * c2 + L3 * c3)
    return torch.stack(out, dim=-1)


# --------------------------------------------------------------------------
# recursion over gluon subsets, explicit adjoint colour indices
# --------------------------------------------------------------------------

def _n_in(S):
    """Incoming gluons (legs 0 and 1) among the gluon legs S."""
    return sum(1 for l in S if l < 2)


def _subsets(items):
    items = tuple(items)
    for r in range(1, len(items) + 1):
        yield from itertools.combinations(items, r)


def _set_partitions(s, nblocks):
    """Unordered partitions of the tuple s into nblocks nonempty blocks."""
    s = tuple(s)
    if nblocks == 1:
        yield (s,)
        return
    first, rest = s[0], s[1:]
    # the block holding `first`, then partition the remainder
    for r in range(0, len(rest) + 1):
        for extra in itertools.combinations(rest, r):
            blk = (first,) + extra
            remain = tuple(x for x in rest if x not in extra)
            if len(remain) < nblocks - 1:
                continue
            for tail in _set_partitions(remain, nblocks - 1):
                yield (blk,) + tail


def amp_full_colour(p, hel, prm, gcol, tcol, tbcol, override=None):
    """i M for g g -> t t~ + n g with explicit colour wavefunctions.

    gcol: dict leg -> complex adjoint vector (..., 8) for each gluon;
    tcol: (..., 3) colour row vector of the t; tbcol: (..., 3) column vector
    of the t~.  The recursion sums every tree diagram exactly once: gluon
    currents over unordered 2- and 3-partitions (3- and 4-gluon vertices),
    the quark line over the gluon subset attached last.
    """
    g = prm.gs
    gl, ubt, vtb, p3 = qcd_externals(p, hel, prm.mt, override)
    labels = [l for (l, _, _) in gl]
    J, K = {}, {}
    for (l, eps, k) in gl:
        J[(l,)] = gcol[l][..., :, None] * eps[..., None, :]          # (..., 8, 4)
        K[(l,)] = k
    for S in _subsets(labels):
        if len(S) < 2:
            continue
        KS = sum(K[(l,)] for l in S)
        K[S] = KS
        acc = 0
        for (S1, S2) in _set_partitions(S, 2):
            J1, J2 = J[S1], J[S2]
            K1, K2 = K[S1][..., None, None, :], K[S2][..., None, None, :]
            j1 = J1[..., :, None, :]
            j2 = J2[..., None, :, :]
            lor = _v3(j1, K1, j2, K2)                                 # (..., 8b, 8c, 4)
            acc = acc + g * torch.einsum('abc,...bcm->...am', _F, lor)
        for (S1, S2, S3) in _set_partitions(S, 3):
            J1, J2, J3 = J[S1], J[S2], J[S3]
            d12 = mdot(J1[..., :, None, :], J2[..., None, :, :])      # (..., b, c)
            d13 = mdot(J1[..., :, None, :], J3[..., None, :, :])      # (..., b, d)
            d23 = mdot(J2[..., :, None, :], J3[..., None, :, :])      # (..., c, d)
            t1 = (torch.einsum('abcd,...cm,...bd->...am', _FF1, J2, d13)
                  - torch.einsum('abcd,...dm,...bc->...am', _FF1, J3, d12))
            t2 = (torch.einsum('abcd,...bm,...cd->...am', _FF2, J1, d23)
                  - torch.einsum('abcd,...dm,...bc->...am', _FF2, J3, d12))
            t3 = (torch.einsum('abcd,...bm,...cd->...am', _FF3, J1, d23)
                  - torch.einsum('abcd,...cm,...bd->...am', _FF3, J2, d13))
            acc = acc + (-1j * g * g) * (t1 + t2 + t3)
        J[S] = (-1j / mdot(KS, KS).to(C128))[..., None, None] * acc
    # quark line: U[S] is the t row spinor with the gluons of S attached
    metric = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)

    def attach(Urow, Jc):
        # Urow (..., 3i, 4x) times i g gamma^mu J^a_mu T^a_{ij} -> (..., 3j, 4y)
        w = torch.einsum('...ix,aij->...ajx', Urow, _T)
        sl = torch.einsum('...am,mxy->...axy', Jc * metric, GAMMA)
        return 1j * g * torch.einsum('...ajx,...axy->...jy', w, sl)

    U = {(): tcol[..., :, None] * ubt[..., None, :]}                  # (..., 3, 4)
    allS = tuple(labels)
    for S in _subsets(labels):
        if S == allS:
            continue
        KS = K[S]
        acc = 0
        for S2 in _subsets(S):
            S1 = tuple(x for x in S if x not in S2)
            acc = acc + attach(U[S1], J[S2])
        # t-channel: exactly one incoming gluon (legs 0, 1) on the t side
        prop = fermion_propagator(p3 - KS, prm.mt, prm.top_width(_n_in(S) == 1))
        U[S] = torch.einsum('...jy,...yz->...jz', acc, prop)
    amp = 0
    for S2 in _subsets(allS):
        S1 = tuple(x for x in allS if x not in S2)
        row = attach(U[S1], J[S2])
        amp = amp + torch.einsum('...jy,...y,...j->...', row, vtb, tbcol)
    return amp


# --------------------------------------------------------------------------
# recursion over gluon subsets, colour decomposed onto T-strings
# --------------------------------------------------------------------------

def _add(d, key, val):
    d[key] = d[key] + val if key in d else val


def dual_amplitudes(p, hel, prm, override=None):
    """Dual (colour-ordered) amplitudes A_w for g g -> t t~ + n g.

    The full amplitude is  i M = sum_w (T^{w_1} ... T^{w_n})_{i j} A_w  over
    the orderings w of the gluon legs.  Obtained from the same Feynman rules
    as ``amp_full_colour`` by writing each gluon current as a matrix
    sum_a J^a T^a, so that f^{abc} T^a -> -i [T^b, T^c] and the two f's of
    the 4-gluon vertex become nested commutators.  Returns a dict
    word (tuple of gluon legs) -> (...,) complex.
    """
    g = prm.gs
    gl, ubt, vtb, p3 = qcd_externals(p, hel, prm.mt, override)
    labels = [l for (l, _, _) in gl]
    J, K = {}, {}
    for (l, eps, k) in gl:
        J[(l,)] = {(l,): eps}
        K[(l,)] = k
    for S in _subsets(labels):
        if len(S) < 2:
            continue
        KS = sum(K[(l,)] for l in S)
        K[S] = KS
        acc = {}
        for (S1, S2) in _set_partitions(S, 2):
            for u, ju in J[S1].items():
                for v, jv in J[S2].items():
                    lor = g * _v3(ju, K[S1], jv, K[S2])
                    # f^{abc} T^a M1^b M2^c = -i [M1, M2]
                    _add(acc, u + v, -1j * lor)
                    _add(acc, v + u, 1j * lor)
        for (S1, S2, S3) in _set_partitions(S, 3):
            for x, jx in J[S1].items():
                for y, jy in J[S2].items():
                    for z, jz in J[S3].items():
                        dxy, dxz, dyz = mdot(jx, jy), mdot(jx, jz), mdot(jy, jz)
                        c = -1j * g * g
                        # f^{abe}f^{cde}: Y(X.Z) - Z(X.Y), colour -[X,[Y,Z]]
                        l1 = c * (jy * dxz[..., None] - jz * dxy[..., None])
                        # f^{ace}f^{bde}: X(Y.Z) - Z(X.Y), colour -[Y,[X,Z]]
                        l2 = c * (jx * dyz[..., None] - jz * dxy[..., None])
                        # f^{ade}f^{bce}: X(Y.Z) - Y(X.Z), colour -[Z,[X,Y]]
                        l3 = c * (jx * dyz[..., None] - jy * dxz[..., None])
                        for word, coef, lor in (
                                (x + y + z, -1, l1), (x + z + y, 1, l1),
                                (y + z + x, 1, l1), (z + y + x, -1, l1),
                                (y + x + z, -1, l2), (y + z + x, 1, l2),
                                (x + z + y, 1, l2), (z + x + y, -1, l2),
                                (z + x + y, -1, l3), (z + y + x, 1, l3),
                                (x + y + z, 1, l3), (y + x + z, -1, l3)):
                            _add(acc, word, coef * lor)
        prop = (-1j / mdot(KS, KS).to(C128))[..., None]
        J[S] = {w: prop * v for w, v in acc.items()}
    U = {(): {(): ubt}}
    allS = tuple(labels)
    for S in _subsets(labels):
        if S == allS:
            continue
        acc = {}
        for S2 in _subsets(S):
            S1 = tuple(x for x in S if x not in S2)
            for u, Uu in U[S1].items():
                for v, jv in J[S2].items():
                    _add(acc, u + v, torch.einsum('...a,...ab->...b', Uu,
                                                  1j * g * slash(jv)))
        prop = fermion_propagator(p3 - K[S], prm.mt, prm.top_width(_n_in(S) == 1))
        U[S] = {w: torch.einsum('...a,...ab->...b', r, prop) for w, r in acc.items()}
    A = {}
    for S2 in _subsets(allS):
        S1 = tuple(x for x in allS if x not in S2)
        for u, Uu in U[S1].items():
            for v, jv in J[S2].items():
                val = torch.einsum('...a,...ab,...b->...', Uu, 1j * g * slash(jv), vtb)
                _add(A, u + v, val)
    return A


def count_diagrams(ngluon):
    """Number of tree diagrams generated by the recursion (4-gluon vertex
    counted once): the same subset structure with every current replaced by
    its diagram count."""
    labels = tuple(range(ngluon))
    c = {}
    for S in _subsets(labels):
        if len(S) == 1:
            c[S] = 1
            continue
        c[S] = (sum(c[a] * c[b] for a, b in _set_partitions(S, 2))
                + sum(c[a] * c[b] * c[d] for a, b, d in _set_partitions(S, 3)))
    U = {(): 1}
    for S in _subsets(labels):
        U[S] = sum(U[tuple(x for x in S if x not in S2)] * c[S2] for S2 in _subsets(S))
    return U[labels]
