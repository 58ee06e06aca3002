"""Cross section and hit-or-miss unweighting from weighted events (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A matrix-element generator produces a fiducial cross section and a sample
of unweighted events from a larger set of weighted events (Sec. II).  With
RAMBO weights w_i (no (2 pi) factors, no flux; reading R10) and matrix
elements ME_i averaged over initial helicities and colours, each event's
weight is f_i = w_i ME_i and, for massless partons at fixed sqrt(s),

    sigma = (hbar c)^2 (2 pi)^(4 - 3 n) / (2 s) * <f>,
    error = (hbar c)^2 (2 pi)^(4 - 3 n) / (2 s) * sqrt((<f^2> - <f>^2) / (N - 1)),

with n final-state particles and the averages over all N events (non-finite
f count as zero).  Hit-or-miss keeps event i iff u_i fmax < f_i, with u_i
the Philox uniform of (seed, event) at counter block 2^31 (a block no
sampler uses).  Plain numpy; the result is the set of kept indices.
"""
import math

import numpy as np

from . import philox

HBARC2_PB = 0.3893793721e9  # (hbar c)^2 in pb GeV^2
UNWEIGHT_BLOCK = 0x80000000


def stats(f):
    """(sum, sum of squares, max, count) over the finite entries of f."""
    f = np.asarray(f, dtype=np.float64)
    fin = f[np.isfinite(f)]
    return (float(fin.sum()), float((fin * fin).sum()), float(fin.max()) if fin.size else 0.0,
            float(fin.size))


def xsec(st, n, sqrts, nfinal, weights_with_2pi=False):
    """sigma and its Monte Carlo error [pb] from stats() of n events;
    weights_with_2pi: the weights already carry (2 pi)^(4 - 3 nfinal)."""
    s = sqrts * sqrts
    twopi = 1.0 if weights_with_2pi else (2.0 * math.pi) ** (4 - 3 * nfinal)
    scale = HBARC2_PB * twopi / (2.0 * s)
    mean = st[0] / n
    var = max(st[1] / n - mean * mean, 0.0)
    err = math.sqrt(var / (n - 1)) if n > 1 else float('inf')
    return scale * mean, scale * err


def unweight_uniforms(seed, evt_offset, n):
    """u_i for events evt_offset .. evt_offset + n - 1."""
    seed = int(seed)
    ev = np.arange(evt_offset, evt_offset + n, dtype=np.uint64)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    ctr = np.stack([ev & np.uint64(0xFFFFFFFF), ev >> np.uint64(32),
                    np.full_like(ev, UNWEIGHT_BLOCK), np.zeros_like(ev)], axis=-1)
    x = philox.philox4x32_10(ctr, np.broadcast_to(key, (n, 2)))
    return philox.bits_to_uniform(x[:, 0] | (x[:, 1] << np.uint64(32)))


def unweight(f, fmax, seed, evt_offset=0):
    """Indices (increasing) of the events kept by hit-or-miss."""
    f = np.asarray(f, dtype=np.float64)
    u = unweight_uniforms(seed, evt_offset, f.size)
    with np.errstate(invalid='ignore'):
        keep = u * fmax < f
    return np.nonzero(keep)[0].astype(np.int64)
