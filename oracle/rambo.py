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
    q = []
    for i in range(n):
        r0, r1, r2, r3 = (r[:, 4 * i + k] for k in range(4))
        c = 2.0 * r0 - 1.0
        sth = torch.sqrt(1.0 - c * c)
        phi = 2.0 * math.pi * r1
        q0 = -torch.log(r2 * r3)
        q.append(torch.stack([q0, q0 * sth * torch.cos(phi),
                              q0 * sth * torch.sin(phi), q0 * c], dim=-1))
    q = torch.stack(q, dim=1)                      # (nevt, n, 4)
    Q = q.sum(dim=1)                               # (nevt, 4)
    M = torch.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(-1))
    b = -Q[:, 1:] / M[:, None]
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    x = sqrts / M
    bq = (b[:, None, :] * q[:, :, 1:]).sum(-1)     # (nevt, n)
    p0 = x[:, None] * (gam[:, None] * q[:, :, 0] + bq)
    pv = x[:, None, None] * (q[:, :, 1:] + b[:, None, :] * q[:, :, :1]
                             + a[:, None, None] * bq[:, :, None] * b[:, None, :])
    p = torch.cat([p0[:, :, None], pv], dim=-1)
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
