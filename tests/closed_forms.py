"""Closed forms and textbook results used to pin the oracle.

Each function is an independent statement of a known result, not a retyping
of oracle code:
* e+e- -> mu+mu- through photon and Z, massless fermions: helicity
  amplitudes (1 +- cos th)^2 |A_ij|^2 (e.g. Peskin & Schroeder ch. 5 with the
  Z added through its chiral couplings).
* g g -> Q Qbar at LO: the spin- and colour-averaged |M|^2 of
  Ellis, Stirling & Webber, "QCD and collider physics", heavy-quark
  production chapter, in terms of tau1,2 = 2 p1,2.p3 / s and rho = 4 m^2/s.
* RAMBO: phase-space volumes R_n with the measure prod d^3p/(2E) delta^4,
  massless closed form and the two-body recursion for massive states.
"""
import math

import numpy as np
from scipy import integrate


def mdot(a, b):
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def eemumu(p, alpha_inv, mZ, wZ, sw2):
    """Spin-averaged |M|^2 for e+(p0) e-(p1) -> mu+(p2) mu-(p3), massless."""
    p = np.asarray(p)
    e2 = 4 * math.pi / alpha_inv
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    # angle between e- (p1) and mu- (p3)
    c = (p[:, 1, 1:] * p[:, 3, 1:]).sum(-1) / (
        np.linalg.norm(p[:, 1, 1:], axis=-1) * np.linalg.norm(p[:, 3, 1:], axis=-1))
    Q = -1.0
    gL, gR = -0.5 + sw2, sw2
    cw2 = 1 - sw2
    chi = s / (s - mZ ** 2 + 1j * mZ * wZ)

    def A(gi, gj):
        return Q * Q + gi * gj / (sw2 * cw2) * chi

    tot = e2 * e2 * ((1 + c) ** 2 * (abs(A(gL, gL)) ** 2 + abs(A(gR, gR)) ** 2)
                     + (1 - c) ** 2 * (abs(A(gL, gR)) ** 2 + abs(A(gR, gL)) ** 2))
    return tot / 4.0


def ggQQ(p, gs, m):
    """Spin- and colour-averaged |M|^2 for g(p0) g(p1) -> Q(p2) Qbar(p3)."""
    p = np.asarray(p)
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    t1 = 2 * mdot(p[:, 0], p[:, 2]) / s
    t2 = 2 * mdot(p[:, 1], p[:, 2]) / s
    rho = 4 * m * m / s
    return gs ** 4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2))


def kallen(a, b, c):
    return a * a + b * b + c * c - 2 * a * b - 2 * a * c - 2 * b * c


def R2(s, ma, mb):
    lam = kallen(s, ma * ma, mb * mb)
    return 0.0 if lam <= 0 else (math.pi / 2) * math.sqrt(lam) / s


def Rn_massless(n, s):
    return (math.pi / 2) ** (n - 1) * s ** (n - 2) / (math.factorial(n - 1) * math.factorial(n - 2))


def Rn(s, masses):
    """Phase-space volume by the recursion R_n(s) = int ds' R_2(s; m1, sqrt s') R_{n-1}(s')."""
    masses = list(masses)
    if len(masses) == 2:
        return R2(s, *masses)
    m1, rest = masses[0], masses[1:]
    lo = sum(rest) ** 2
    hi = (math.sqrt(s) - m1) ** 2
    val, _ = integrate.quad(lambda sp: R2(s, m1, math.sqrt(sp)) * Rn(sp, rest), lo, hi,
                            epsabs=0, epsrel=1e-11, limit=200)
    return val
