"""SU(3) colour algebra by brute force (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The colour-flow decomposition of Sec. II writes each amplitude as a sum of
dual amplitudes times colour structures; the squared amplitude is a
quadratic form with a colour matrix that is the same for every event.  For
one quark line and n gluons the structures are the T-strings
(T^{a_s1} ... T^{a_sn})_{ij}, one per ordering s of the gluons, and the
colour matrix is their overlap summed over all external colours:
    C[s, s'] = sum_{a, i, j} (T^s)_{ij} conj((T^s')_{ij})      (reading R2)
computed here by summing over every assignment of adjoint indices with the
explicit Gell-Mann matrices, T^a = lambda^a / 2.
"""
import itertools
import math
from fractions import Fraction

import numpy as np

_S3 = 1.0 / math.sqrt(3.0)


def gell_mann():
    """The eight Gell-Mann matrices lambda^1..lambda^8, shape (8, 3, 3)."""
    L = np.zeros((8, 3, 3), dtype=np.complex128)
    L[0][0, 1] = L[0][1, 0] = 1
    L[1][0, 1] = -1j
    L[1][1, 0] = 1j
    L[2][0, 0] = 1
    L[2][1, 1] = -1
    L[3][0, 2] = L[3][2, 0] = 1
    L[4][0, 2] = -1j
    L[4][2, 0] = 1j
    L[5][1, 2] = L[5][2, 1] = 1
    L[6][1, 2] = -1j
    L[6][2, 1] = 1j
    L[7][0, 0] = L[7][1, 1] = _S3
    L[7][2, 2] = -2 * _S3
    return L


T = gell_mann() / 2.0


def structure_constants():
    """f^{abc} = -2i Tr([T^a, T^b] T^c), real and totally antisymmetric."""
    f = np.zeros((8, 8, 8))
    for a, b, c in itertools.product(range(8), repeat=3):
        comm = T[a] @ T[b] - T[b] @ T[a]
        v = -2j * np.trace(comm @ T[c])
        f[a, b, c] = v.real
    return f


F = structure_constants()


def tstring(adj):
    """T^{a1} T^{a2} ... for a sequence of adjoint indices (3x3)."""
    m = np.eye(3, dtype=np.complex128)
    for a in adj:
        m = m @ T[a]
    return m


def colour_matrix(ngluon):
    """C[s, s'] over the orderings s of ngluon gluons (itertools order).

    Returns (orderings, C) with C a float64 array.  The sum over the 8^n
    adjoint assignments is done explicitly.
    """
    perms = list(itertools.permutations(range(ngluon)))
    npm = len(perms)
    C = np.zeros((npm, npm), dtype=np.complex128)
    for adj in itertools.product(range(8), repeat=ngluon):
        mats = np.array([tstring([adj[g] for g in s]) for s in perms])  # (npm,3,3)
        flat = mats.reshape(npm, 9)
        C += flat @ flat.conj().T
    assert np.abs(C.imag).max() < 1e-12
    return perms, C.real


def rationalise(C, max_den=1000):
    """Exact rationals for C (entries are rational with small denominators)."""
    R = [[Fraction(x).limit_denominator(max_den) for x in row] for row in C]
    err = max(abs(float(R[i][j]) - C[i][j]) for i in range(len(R)) for j in range(len(R)))
    assert err < 1e-10, err
    return R
