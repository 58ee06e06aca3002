"""Physics inputs and derived couplings (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper keeps physics parameters (masses, couplings) in constant memory
(Sec. IV.c) but prints no values.  The inputs here are the benchmark
workloads' (sqrt(s) = 1500 GeV, alpha = 1/132.5, mZ = 91.188, GammaZ = 2.441,
mt = 173, Gammat = 1.49, alpha_s = 0.118).  sin^2(theta_W) is not given and is
derived in the G_F scheme (reading R3):
    mW^2 = mZ^2/2 + sqrt(mZ^4/4 - pi alpha mZ^2 / (sqrt(2) G_F)),
    sW^2 = 1 - mW^2/mZ^2.

Two switches (bits of ``flags``):
* TCHANNEL_ZERO_WIDTH (reading R5): the top width enters every top
  propagator, except, with this bit, the t-channel ones (those with exactly
  one incoming particle on each side), where a width breaks gauge
  invariance;
* WEIGHT_2PI (reading R10): the RAMBO weight is the phase-space volume of
  the measure prod d^3p/(2E) delta^4 without 2 pi factors; with this bit it
  carries (2 pi)^(4 - 3n).
"""
import math
from dataclasses import dataclass, replace


TCHANNEL_ZERO_WIDTH = 1
WEIGHT_2PI = 2


@dataclass(frozen=True)
class Params:
    sqrts: float = 1500.0
    alpha_inv: float = 132.5
    gfermi: float = 1.16639e-5
    mZ: float = 91.188
    wZ: float = 2.441
    mt: float = 173.0
    wt: float = 1.49
    alphas: float = 0.118
    flags: int = 0

    @property
    def e(self):
        return math.sqrt(4.0 * math.pi / self.alpha_inv)

    @property
    def gs(self):
        return math.sqrt(4.0 * math.pi * self.alphas)

    @property
    def mW2(self):
        a = 1.0 / self.alpha_inv
        mz2 = self.mZ ** 2
        return mz2 / 2.0 + math.sqrt(mz2 * mz2 / 4.0
                                     - math.pi * a * mz2 / (math.sqrt(2.0) * self.gfermi))

    @property
    def sw2(self):
        return 1.0 - self.mW2 / self.mZ ** 2

    def top_width(self, t_channel):
        """Width of a top propagator: t_channel = exactly one incoming
        particle on each side of it."""
        return 0.0 if (t_channel and self.flags & TCHANNEL_ZERO_WIDTH) else self.wt

    def with_(self, **kw):
        return replace(self, **kw)


DEFAULT = Params()
