"""RAMBO phase-space sampling, massless and massive (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's phase-space sampler (Sec. IV.a, IV.b) is RAMBO; the method is
R. Kleiss, W.J. Stirling, S.D. Ellis, Comput. Phys. Commun. 40 (1986) 359.
Written here from that method, in float64 torch ops so that the gradient
oracle can differentiate through it.

Per final-state particle i, with its four uniforms (r0, r1, r2, r3) in slots
4i .. 4i+3 (reading R8):
  c = 2 r0 - 1, phi = 2 pi r1, q0 = -ln(r2 r3),
  q = q0 (sqrt(1-c^2) cos phi, sqrt(1-c^2) sin phi, c).
The q_i are boosted to the rest frame of Q = sum q_i and scaled to sqrt(s).
The boost is evaluated in a form that is identical in exact arithmetic but
keeps its accuracy when the q_i are nearly collinear (reading: the published
M = sqrt(Q^2) and boost formulas lose about gamma^2 = (Q^0/M)^2 of their
digits, up to 1e5 for two-body final states).  With n_i the unit vectors of
the q_i, the Minkowski products of the massless q_i are
  q_i.q_j = q_i^0 q_j^0 |n_i - n_j|^2 / 2,
so that M^2 = sum_{i != j} q_i.q_j; the rest-frame energies are
E_i = (q_i.Q)/M = sum_{j != i} q_i.q_j / M and the rest-frame three-momenta
q_i - Q (q_i^0 + E_i) / (Q^0 + M), the boost of the method written with the
rest-frame energy instead of b = -Q/M and a = 1/(1 + gamma).
The massless weight is the phase-space volume (measure prod d^3p/(2E)
delta^4, no 2pi factors, no flux; reading R10)
  w0 = (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!).
Masses are introduced by solving sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s) for
xi with Newton's method (start xi0 = sqrt(1 - (sum m / sqrt s)^2), stop at
|f| <= 1e-14 sqrt(s), at most 50 steps; reading R11), then
  k_i = (sqrt(m_i^2 + xi^2 E_i^2), xi p_i),
  w = w0 xi^(2n-3) prod(|k_i|/k_i^0) sqrt(s) / sum(|k_i|^2 / k_i^0).
Initial momenta: p1 = sqrt(s)/2 (1,0,0,1), p2 = sqrt(s)/2 (1,0,0,-1).
"""
import math
import torch

F64 = torch.float64


def massless_weight(n, s):
    """w0 = (pi/2)^(n-1) s^(n-2) / ((n-1)!(n-2)!)."""
    return (math.pi / 2.0) ** (n - 1) * s ** (n - 2) / (
        math.factorial(n - 1) * math.factorial(n - 2))


def rambo_massless(r, sqrts, n):
    """r: (nevt, 4n) float64 tensor.  Returns p (nevt, n, 4) and w0 (scalar)."""
    r = r.to(F64)
    nevt = r.shape[0]
    q0, nhat = [], []
    for i in range(n):
        r0, r1, r2, r3 = (r[:, 4 * i + k] for k in range(4))
        c = 2.0 * r0 - 1.0
        sth = torch.sqrt(1.0 - c * c)
        phi = 2.0 * math.pi * r1
        q0.append(-torch.log(r2 * r3))
        nhat.append(torch.stack([sth * torch.cos(phi), sth * torch.sin(phi), c], dim=-1))
    q0 = torch.stack(q0, dim=1)                    # (nevt, n)
    nhat = torch.stack(nhat, dim=1)                # (nevt, n, 3)
    qv = q0[:, :, None] * nhat                     # (nevt, n, 3)
    Q0 = q0.sum(dim=1)                             # (nevt,)
    Qv = qv.sum(dim=1)                             # (nevt, 3)
    # Minkowski products q_i.q_j of the massless q_i, i != j
    dots = torch.zeros(nevt, n, n, dtype=F64)
    for i in range(n):
        for j in range(n):
            if i != j:
                dn = nhat[:, i] - nhat[:, j]
                dots[:, i, j] = 0.5 * q0[:, i] * q0[:, j] * (dn * dn).sum(-1)
    M = torch.sqrt(dots.sum(dim=(1, 2)))           # sqrt(Q.Q)
    E = dots.sum(dim=2) / M[:, None]               # q_i.Q / M: rest-frame energies
    pv = qv - Qv[:, None, :] * ((q0 + E) / (Q0 + M)[:, None])[:, :, None]
    x = sqrts / M
    p = x[:, None, None] * torch.cat([E[:, :, None], pv], dim=-1)
    assert p.shape == (nevt, n, 4)
    return p, massless_weight(n, sqrts * sqrts)


class NoPhaseSpace(ValueError):
    pass


def rambo_massive(r, sqrts, masses):
    """Final-state momenta (nevt, n, 4) and weights (nevt,) for given masses."""
    n = len(masses)
    p, w0 = rambo_massless(r, sqrts, n)
    nevt = p.shape[0]
    if all(m == 0.0 for m in masses):
        return p, torch.full((nevt,), w0, dtype=F64)
    msum = sum(masses)
    if msum >= sqrts:
        raise NoPhaseSpace("sum of masses >= sqrt(s)")
    m2 = torch.tensor([m * m for m in masses], dtype=F64)
    E = p[:, :, 0]
    xi = torch.full((nevt,), math.sqrt(1.0 - (msum / sqrts) ** 2), dtype=F64)
    for it in range(51):
        root = torch.sqrt(m2[None, :] + (xi[:, None] * E) ** 2)
        f = root.sum(1) - sqrts
        if bool((f.abs() <= 1e-14 * sqrts).all()):
            break
        if it == 50:
            raise NoPhaseSpace("Newton solve for the RAMBO scale did not converge")
        fp = (xi[:, None] * E * E / root).sum(1)
        xi = xi - f / fp
    k0 = torch.sqrt(m2[None, :] + (xi[:, None] * E) ** 2)
    kv = xi[:, None, None] * p[:, :, 1:]
    k = torch.cat([k0[:, :, None], kv], dim=-1)
    kabs = torch.sqrt((kv ** 2).sum(-1))
    w = (w0 * xi ** (2 * n - 3) * torch.prod(kabs / k0, dim=1)
         * sqrts / (kabs ** 2 / k0).sum(1))
    return k, w


def initial_momenta(nevt, sqrts):
    """p1 along +z, p2 along -z, each with energy sqrt(s)/2: (nevt, 2, 4)."""
    h = sqrts / 2.0
    p = torch.zeros(nevt, 2, 4, dtype=F64)
    p[:, 0, 0] = h
    p[:, 0, 3] = h
    p[:, 1, 0] = h
    p[:, 1, 3] = -h
    return p


def event_momenta(r, sqrts, masses):
    """All momenta (nevt, 2 + n, 4) = initial + RAMBO final, and weights."""
    k, w = rambo_massive(r, sqrts, masses)
    return torch.cat([initial_momenta(k.shape[0], sqrts).to(k.dtype), k], dim=1), w
