"""Philox4x32-10 counter-based generator and the uniform-double map (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's random-number component (Sec. IV.b) draws four uniforms per
particle from cuRAND and relies on host and device producing identical
sequences for event-by-event reproducibility (Sec. III).  Here the generator
is Philox4x32 with 10 rounds from Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a bijection of a 128-bit counter
under a 64-bit key, so any event's numbers depend only on (seed, event index).

Conventions (documented readings, not from the paper):
* key     = (seed mod 2^32, seed >> 32)
* counter = (event mod 2^32, event >> 32, block j, 0)
* block j yields words x0..x3; slot s of an event uses block s // 2 and the
  64-bit word  w = x[2 (s mod 2)] + 2^32 x[2 (s mod 2) + 1]
* u = ((w >> 11) + 1/2) * 2^-53, strictly inside (0, 1).
"""
import numpy as np

# Round multipliers and Weyl key increments as published for Philox4x32.
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Apply 10 Philox rounds.

    ctr: uint array (..., 4) of 32-bit words; key: uint array (..., 2).
    Returns uint64 array (..., 4) holding the four 32-bit output words.
    Each round: the products M0*c0 and M1*c2 are split into high and low
    halves; the new counter is (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key is
    advanced by the Weyl constants between rounds.
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i] & _MASK for i in range(4))
    k0, k1 = key[..., 0] & _MASK, key[..., 1] & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0           # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _SH32, p0 & _MASK
        hi1, lo1 = p1 >> _SH32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def bits_to_uniform(w64):
    """Map a 64-bit word to ((w >> 11) + 1/2) 2^-53, an FP64 in (0, 1)."""
    w64 = np.asarray(w64, dtype=np.uint64)
    return ((w64 >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def uniforms(seed, evt_offset, nevt, nrnd):
    """Uniforms for events evt_offset .. evt_offset+nevt-1, shape (nevt, nrnd).

    Row e, column s is slot s of global event evt_offset + e (see module doc).
    """
    seed = int(seed)
    ev = np.arange(evt_offset, evt_offset + nevt, dtype=np.uint64)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    out = np.empty((nevt, nrnd), dtype=np.float64)
    nblk = (nrnd + 1) // 2
    for j in range(nblk):
        ctr = np.stack([ev & _MASK, ev >> _SH32,
                        np.full_like(ev, j), np.zeros_like(ev)], axis=-1)
        x = philox4x32_10(ctr, np.broadcast_to(key, (nevt, 2)))
        for half in range(2):
            s = 2 * j + half
            if s >= nrnd:
                break
            w = x[:, 2 * half] | (x[:, 2 * half + 1] << _SH32)
            out[:, s] = bits_to_uniform(w)
    return out
