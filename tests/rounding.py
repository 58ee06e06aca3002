"""Rounding bounds for comparisons of two FP64 RAMBO implementations.

RAMBO boosts the massless momenta q_i from the frame of their sum Q to its
rest frame.  With gamma = Q^0 / sqrt(Q^2), rounding in Q and the boost is
amplified by ~gamma^2 in the momenta and the weight, and derivatives with
respect to the uniforms pick up one more factor gamma (the derivative of
the boost with respect to Q).  Two-body final states reach gamma^2 ~ 1e5
when the two q_i are nearly collinear.
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
