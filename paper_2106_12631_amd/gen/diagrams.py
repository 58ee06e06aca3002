"""Tree-diagram enumeration and colour-flow projection for the generated kernels.

The paper's matrix-element code is generated per process from its Feynman
diagrams (Sec. II: the meta-code determines the diagrams and emits the
routine calls; Table "tab-compl" counts the generated calls).  This module
is the build-time equivalent for the four processes of the benchmark:

* wavefunctions ("nodes") are built bottom-up over subsets of external legs,
  one node per distinct sub-diagram, so a sub-diagram shared by several
  diagrams is computed once (the reuse shown in Fig. 1);
* every diagram is closed at a vertex containing a fixed root leg (the
  flow-in fermion), which makes each tree appear exactly once;
* the colour factor of every node is kept as a polynomial in the generators
  T^a of the external gluons (a "Lie polynomial": word -> coefficient), using
  f^{abc} T^a -> -i [T^b, T^c] for the 3-gluon vertex and nested commutators
  for the three f f terms of the 4-gluon vertex, and products of T's along
  the quark line.  A diagram's colour factor is then a combination of
  T-strings, which gives its coefficient in each colour-flow (dual)
  amplitude -- the colour-flow decomposition of Sec. II.
"""
import itertools
from dataclasses import dataclass, field
from fractions import Fraction

IN, OUT = 'in', 'out'

# external particle -> (wavefunction kind, flavour, routine)
EXTERNAL = {
    ('g', IN): ('V', 'g', 'vec_in'),
    ('g', OUT): ('V', 'g', 'vec_out'),
    ('t', OUT): ('Fout', 't', 'ubar'),
    ('t~', OUT): ('Fin', 't', 'v'),
    ('e+', IN): ('Fout', 'e', 'vbar'),
    ('e-', IN): ('Fin', 'e', 'u'),
    ('mu+', OUT): ('Fin', 'mu', 'v'),
    ('mu-', OUT): ('Fout', 'mu', 'ubar'),
}

# f f V couplings: (fermion flavour, boson) -> (cL, cR) coupling names
FFV = {
    ('t', 'g'): ('gs', 'gs'),
    ('e', 'a'): ('cqed', 'cqed'),
    ('mu', 'a'): ('cqed', 'cqed'),
    ('e', 'z'): ('czl', 'czr'),
    ('mu', 'z'): ('czl', 'czr'),
}
COLOURED_FERMIONS = {'t'}
FERMION_MASS = {'t': ('mt', 'wt'), 'e': (None, None), 'mu': (None, None)}
BOSON_MASS = {'g': None, 'a': None, 'z': ('mz', 'wz')}

PROCESSES = {
    'eemumu': [('e+', IN), ('e-', IN), ('mu+', OUT), ('mu-', OUT)],
    'ggtt': [('g', IN), ('g', IN), ('t', OUT), ('t~', OUT)],
    'ggttg': [('g', IN), ('g', IN), ('t', OUT), ('t~', OUT), ('g', OUT)],
    'ggttgg': [('g', IN), ('g', IN), ('t', OUT), ('t~', OUT), ('g', OUT), ('g', OUT)],
}


# --------------------------------------------------------------------------
# Lie polynomials: dict word(tuple of gluon legs) -> complex coefficient
# --------------------------------------------------------------------------

def pmul(a, b):
    out = {}
    for wa, ca in a.items():
        for wb, cb in b.items():
            w = wa + wb
            out[w] = out.get(w, 0) + ca * cb
    return {w: c for w, c in out.items() if c != 0}


def padd(*terms):
    out = {}
    for coef, poly in terms:
        for w, c in poly.items():
            out[w] = out.get(w, 0) + coef * c
    return {w: c for w, c in out.items() if c != 0}


def comm(a, b):
    return padd((1, pmul(a, b)), (-1, pmul(b, a)))


ONE = {(): 1}


@dataclass
class Node:
    idx: int
    kind: str            # 'V', 'Fout', 'Fin'
    flav: str            # boson ('g', 'a', 'z') or fermion flavour
    legs: frozenset
    colour: dict
    op: tuple            # construction
    uses: int = 0


@dataclass
class Diagram:
    fout: Node
    vec: Node
    fin: Node
    colour: dict
    rep: bool            # counts as a distinct Feynman diagram (4-gluon structures grouped)


def _partitions2(s):
    s = sorted(s)
    first, rest = s[0], s[1:]
    for r in range(0, len(rest)):
        for extra in itertools.combinations(rest, r):
            a = frozenset((first,) + extra)
            b = frozenset(s) - a
            if b:
                yield a, b


def _partitions3(s):
    s = sorted(s)
    first, rest = s[0], s[1:]
    for r in range(0, len(rest) - 1):
        for extra in itertools.combinations(rest, r):
            a = frozenset((first,) + extra)
            for b, c in _partitions2(frozenset(s) - a):
                yield a, b, c


def _subsets(legs):
    legs = sorted(legs)
    for r in range(1, len(legs) + 1):
        for c in itertools.combinations(legs, r):
            yield frozenset(c)


class ProcessDiagrams:
    """Nodes and diagrams of one process."""

    def __init__(self, name):
        self.name = name
        self.particles = PROCESSES[name]
        self.npar = len(self.particles)
        self.gluons = [i for i, (p, _) in enumerate(self.particles) if p == 'g']
        self.nodes = []
        kinds = [EXTERNAL[pd] for pd in self.particles]
        roots = [i for i, k in enumerate(kinds) if k[0] == 'Fin']
        self.root = roots[-1]
        self.ext = {}
        for i, (kind, flav, routine) in enumerate(kinds):
            col = {(i,): 1} if self.particles[i][0] == 'g' else dict(ONE)
            n = self._new(kind, flav, frozenset([i]), col, ('ext', i, routine))
            self.ext[i] = n
        self.by_subset = {frozenset([i]): [self.ext[i]] for i in range(self.npar) if i != self.root}
        others = [i for i in range(self.npar) if i != self.root]
        for S in _subsets(others):
            if len(S) < 2:
                continue
            lst = []
            for A, B in _partitions2(S):
                for a in self.by_subset.get(A, []):
                    for b in self.by_subset.get(B, []):
                        lst += self._combine(a, b, S)
            for A, B, C in _partitions3(S):
                for a in self.by_subset.get(A, []):
                    for b in self.by_subset.get(B, []):
                        for c in self.by_subset.get(C, []):
                            if a.flav == b.flav == c.flav == 'g' and a.kind == b.kind == c.kind == 'V':
                                for s in (1, 2, 3):
                                    lst.append(self._vvvv(s, a, b, c, S))
            self.by_subset[S] = lst
        self.diagrams = self._close(frozenset(others))
        self._close_early()
        self._prune()

    def _new(self, kind, flav, legs, colour, op):
        n = Node(len(self.nodes), kind, flav, legs, colour, op)
        self.nodes.append(n)
        return n

    def _combine(self, a, b, S):
        out = []
        for x, y in ((a, b), (b, a)):
            if x.kind == 'V' and y.kind == 'V' and x.flav == y.flav == 'g' and x.idx < y.idx:
                # f^{out x y}: colour -i [X, Y]
                col = padd((-1j, pmul(x.colour, y.colour)), (1j, pmul(y.colour, x.colour)))
                out.append(self._new('V', 'g', S, col, ('vvv', x, y)))
            if x.kind == 'Fout' and y.kind == 'V' and (x.flav, y.flav) in FFV:
                col = pmul(x.colour, y.colour) if y.flav == 'g' else dict(x.colour)
                out.append(self._new('Fout', x.flav, S, col, ('ffv_fout', x, y)))
            if x.kind == 'V' and y.kind == 'Fin' and (y.flav, x.flav) in FFV:
                col = pmul(x.colour, y.colour) if x.flav == 'g' else dict(y.colour)
                out.append(self._new('Fin', y.flav, S, col, ('ffv_fin', x, y)))
            if x.kind == 'Fout' and y.kind == 'Fin' and x.flav == y.flav:
                if x.flav in COLOURED_FERMIONS:
                    continue  # not needed with the root at the flow-in quark
                for (f, boson) in FFV:
                    if f == x.flav:
                        out.append(self._new('V', boson, S, dict(ONE), ('ffv_v', x, y, boson)))
        return out

    def _vvvv(self, s, x, y, z, S):
        X, Y, Z = x.colour, y.colour, z.colour
        if s == 1:
            col = padd((-1, comm(X, comm(Y, Z))))
        elif s == 2:
            col = padd((-1, comm(Y, comm(X, Z))))
        else:
            col = padd((-1, comm(Z, comm(X, Y))))
        return self._new('V', 'g', S, col, ('vvvv', s, x, y, z))

    def _close(self, allS):
        root = self.ext[self.root]
        diags = []
        for A, B in _partitions2(allS):
            for X, Y in ((A, B), (B, A)):
                for f in self.by_subset.get(X, []):
                    for v in self.by_subset.get(Y, []):
                        if f.kind == 'Fout' and f.flav == root.flav and v.kind == 'V' \
                                and (root.flav, v.flav) in FFV:
                            col = pmul(f.colour, v.colour) if v.flav == 'g' else dict(f.colour)
                            diags.append(Diagram(f, v, root, col, self._is_rep(f) and self._is_rep(v)))
        return diags

    def _close_early(self):
        """Close a diagram whose last attachment before the root is a single
        external gluon w one vertex earlier: F' X [prop] w root becomes
        F' X Fin(w) with Fin(w) = the root spinor after absorbing w.  The
        same Feynman diagram (same propagators, vertices and colour factor),
        but the four Fin(w) currents replace every fermion current that
        carried all but one gluon."""
        root = self.ext[self.root]
        fins = {}
        out = []
        for d in self.diagrams:
            if d.fin is root and d.vec.op[0] == 'ext' and d.fout.op[0] == 'ffv_fout':
                fprev, x = d.fout.op[1], d.fout.op[2]
                w = d.vec
                if w.idx not in fins:
                    col = pmul(w.colour, root.colour) if w.flav == 'g' else dict(root.colour)
                    fins[w.idx] = self._new('Fin', root.flav, w.legs | root.legs, col,
                                            ('ffv_fin', w, root))
                out.append(Diagram(fprev, x, fins[w.idx], d.colour, d.rep))
            else:
                out.append(d)
        self.diagrams = out

    def _is_rep(self, n):
        if n.op[0] == 'ext':
            return True
        if n.op[0] == 'vvvv' and n.op[1] != 1:
            return False
        return all(self._is_rep(c) for c in n.op[1:] if isinstance(c, Node))

    def _prune(self):
        used = set()

        def mark(n):
            if n.idx in used:
                return
            used.add(n.idx)
            for c in n.op[1:]:
                if isinstance(c, Node):
                    mark(c)
        for d in self.diagrams:
            for n in (d.fout, d.vec, d.fin):
                mark(n)
        self.used = [n for n in self.nodes if n.idx in used]

    # ---------------------------------------------------------------- colour
    def colour_basis(self):
        """Orderings of the gluon legs: the colour-flow basis."""
        return [tuple(p) for p in itertools.permutations(self.gluons)]

    def jamp_coefficients(self):
        """For every diagram, {flow index: complex coefficient}."""
        basis = self.colour_basis() if self.gluons else [()]
        index = {w: k for k, w in enumerate(basis)}
        out = []
        for d in self.diagrams:
            coefs = {}
            for w, c in d.colour.items():
                if w not in index:
                    raise ValueError(f"colour word {w} outside the T-string basis")
                coefs[index[w]] = coefs.get(index[w], 0) + c
            out.append({k: v for k, v in coefs.items() if v != 0})
        return out

    @property
    def ndiagrams(self):
        return sum(1 for d in self.diagrams if d.rep)


# --------------------------------------------------------------------------
# colour matrix by brute force over the adjoint indices (own SU(3) tables)
# --------------------------------------------------------------------------

def _su3_generators():
    import numpy as np
    r3 = 3 ** -0.5
    lam = np.zeros((8, 3, 3), dtype=complex)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([r3, r3, -2 * r3])
    return lam / 2


def colour_matrix(basis, ngluon):
    """Integer numerators and common denominator of
    C[s, t] = sum_{a, i, j} (T^s)_{ij} conj((T^t)_{ij})."""
    import numpy as np
    T = _su3_generators()
    nb = len(basis)
    legs = sorted(basis[0])
    pos = {leg: k for k, leg in enumerate(legs)}
    C = np.zeros((nb, nb), dtype=complex)
    for adj in itertools.product(range(8), repeat=ngluon):
        mats = []
        for w in basis:
            m = np.eye(3, dtype=complex)
            for leg in w:
                m = m @ T[adj[pos[leg]]]
            mats.append(m.ravel())
        M = np.array(mats)
        C += M @ M.conj().T
    if abs(C.imag).max() > 1e-12:
        raise ValueError("colour matrix is not real")
    F = [[Fraction(x).limit_denominator(10000) for x in row] for row in C.real]
    den = 1
    for row in F:
        for x in row:
            den = den * x.denominator // __import__('math').gcd(den, x.denominator)
    num = [[int(x * den) for x in row] for row in F]
    if max(abs(num[i][j] / den - C.real[i, j]) for i in range(nb) for j in range(nb)) > 1e-9:
        raise ValueError("colour matrix is not rational with a small denominator")
    return num, den
