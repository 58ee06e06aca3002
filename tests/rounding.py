"""Rounding bounds for comparisons of two FP64 RAMBO implementations.

RAMBO boosts the massless momenta q_i from the frame of their sum Q to its
rest frame, gamma = Q^0 / sqrt(Q^2).  Both the oracle and the HIP path form
the boost from the pairwise Minkowski products of the q_i (exact for nearly
collinear q_i), so rounding in the momenta grows only like gamma: one ulp
of a q_i component is gamma ulps of the rest-frame momenta.  Each side is
within 32 eps gamma sqrt(s) of the exact momenta (the oracle's pin against
the published boost in extended precision), so two sides differ by at most
64 eps gamma sqrt(s).  The massive weight contains |k_i| / k_i^0 and
|k_i|^2 / k_i^0: an absolute momentum error dk is a relative error
dk / |k_i| of those factors, so the weights agree within
64 eps gamma sqrt(s) / min_i |k_i|.  Derivatives with respect to the
uniforms pick up one more factor gamma (the derivative of the boost with
respect to Q).  Two-body final states reach gamma ~ 370 when the two q_i
are nearly collinear.
"""
import math

import torch

EPS = 2.0 ** -52


def boost_gamma(r):
    """gamma of the RAMBO boost for event-major uniforms r (nevt, 4 nparf)."""
    q0 = -torch.log(r[:, 2::4] * r[:, 3::4])
    c = 2 * r[:, 0::4] - 1
    ph = 2 * math.pi * r[:, 1::4]
    st = torch.sqrt(1 - c * c)
    q = torch.stack([q0, q0 * st * torch.cos(ph), q0 * st * torch.sin(ph), q0 * c], -1)
    Q = q.sum(1)
    return Q[:, 0] / torch.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(-1))


def momentum_bound(r, sqrts):
    """Per-event bound on max |p_a - p_b| over all components (GeV)."""
    return 64 * EPS * boost_gamma(r) * sqrts


def weight_bound(r, p, sqrts):
    """Per-event bound on |w_a / w_b - 1| for momenta p (nevt, npar, 4)."""
    kmin = torch.sqrt((p[:, 2:, 1:] ** 2).sum(-1)).amin(1)
    return 64 * EPS * boost_gamma(r) * sqrts / kmin


def invariant_condition(p):
    """kappa = s / min_{i<j} |2 p_i.p_j| per event, momenta p (nevt, npar, 4).

    A propagator invariant formed from momentum components carries an
    absolute rounding error of order eps s, i.e. a relative error
    eps s / |s_ij| of the propagator: kappa measures how much a matrix
    element amplifies relative rounding of its momenta."""
    npar = p.shape[1]
    s = (p[:, 0, 0] + p[:, 1, 0]) ** 2 - ((p[:, 0, 1:] + p[:, 1, 1:]) ** 2).sum(-1)
    m = None
    for i in range(npar):
        for j in range(i + 1, npar):
            d = (2 * (p[:, i, 0] * p[:, j, 0] - (p[:, i, 1:] * p[:, j, 1:]).sum(-1))).abs()
            m = d if m is None else torch.minimum(m, d)
    return s / m


def end_to_end_bound(r, p):
    """Per-event bound on the relative difference of |M|^2 computed end to
    end (uniforms -> momenta -> |M|^2) by two FP64 implementations: 1e-12 on
    identical momenta, plus the momentum rounding of both sides (order
    eps gamma relative to sqrt(s)) amplified by kappa."""
    return 1e-12 + 8 * EPS * boost_gamma(r) * invariant_condition(p)
