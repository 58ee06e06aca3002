"""Emit straight-line HIP code for the generated matrix-element kernels.

For each process this writes ``csrc/generated/<proc>.inc`` with, inside
``namespace mg::gen_<proc>``:
  * constants NPAR, NCOL, NDIAG, NAMP, IDEN, CDEN and the colour-matrix
    numerators CNUM (integers over the common denominator CDEN);
  * ``jamps<T>(p, hcode, c, J)``: external wavefunctions for helicity code
    ``hcode``, every node (off-shell current) once, every diagram's
    amplitude accumulated into the colour-flow amplitudes J with the
    coefficients of the colour projection (Sec. II);
  * ``colour_sum<T>(J)``: sum_ij CNUM_ij Re(conj(J_i) J_j) / CDEN;
and ``generated/meta.json`` with diagram/call counts and the algorithmic
flop count per helicity (per-routine counts below: add, mul = 1 flop,
fused multiply-add = 2, divide, square root = 1).
"""
import json
import os

from .diagrams import (BOSON_MASS, FERMION_MASS, FFV, IN, OUT, PROCESSES, ProcessDiagrams,
                       colour_matrix)

IDEN = {'eemumu': 4, 'ggtt': 256, 'ggttg': 256, 'ggttgg': 512}

# algorithmic flops of each device routine (counted from helas.h)
FLOPS = {
    'vec_in': 22, 'vec_out': 22, 'ubar': 30, 'u': 30, 'v': 30, 'vbar': 30,
    'ffv_amp': 118, 'ffv_cur_v0': 104, 'ffv_cur_vm': 140,
    'ffv_cur_fin': 171, 'ffv_cur_fout': 171,
    # vector-like vertices (cL = cR): the coupling applied once
    'ffv_amp_v': 104, 'ffv_cur_fin_v': 165, 'ffv_cur_fout_v': 165,
    'vvv_cur': 187, 'vvvv_cur': 128,
    'ffv_bil': 88, 'amp_dot': 30,
    'jamp_acc': 2,
}


class Bil:
    """Shared bilinear F gamma^mu (cL P_L + cR P_R) Fin of an (F, Fin) pair
    closing several diagrams with the same couplings: each diagram is then
    i (bil . V)."""

    def __init__(self, idx, fout, fin, couplings):
        self.idx = idx
        self.fout = fout
        self.fin = fin
        self.couplings = couplings
        self.op = ('bil', fout, fin)


def _f32_bits(v):
    import struct
    return struct.unpack('<I', struct.pack('<f', float(v)))[0]


def colour_mfma_tables(cnum, ncol):
    """The A operands of the matrix-core colour sum (csrc/colour_mfma.h) for
    the numerators cnum, per K block kb and lane l (m = l % 32 the row of C,
    kh = l / 32 the half of the K block):
      F32:  one float, C[m][2 kb + kh];
      BF16: eight BF16 values packed two per 32-bit word, low half first:
            C[m][8 g + j], j = 0..7, g = (2 kb + kh) % G for the chunk
            c = 2 kb + kh of the three-way split (the split index does not
            change C), zero past the matrix and the last chunk.
    Every numerator has at most 8 significant bits, so its BF16 bits are the
    upper half of its FP32 bits."""
    kbf = (ncol + 1) // 2
    f32 = [[float(cnum[l & 31][2 * kb + (l >> 5)])
            if (l & 31) < ncol and 2 * kb + (l >> 5) < ncol else 0.0
            for l in range(64)] for kb in range(kbf)]
    g_ = (ncol + 7) // 8
    nch = 3 * g_
    kbb = (nch + 1) // 2
    bf16 = []
    for kb in range(kbb):
        row = []
        for l in range(64):
            m, c = l & 31, 2 * kb + (l >> 5)
            g = c % g_
            words = []
            for q in range(4):
                half = []
                for t in range(2):
                    col = 8 * g + 2 * q + t
                    v = cnum[m][col] if (m < ncol and c < nch and col < ncol) else 0
                    bits = _f32_bits(v)
                    assert bits & 0xFFFF == 0, "numerator not exact in BF16"
                    half.append(bits >> 16)
                words.append(half[0] | (half[1] << 16))
            row.append(words)
        bf16.append(row)
    return f32, bf16


def _deps(n):
    return [c for c in n.op[1:] if hasattr(c, 'idx')]


def schedule(pd):
    """Order the amplitude terms greedily so that each step needs as few new
    wavefunctions as possible (keeps live ranges short).  Returns the list
    of (diagram index, closing form) and the bilinear nodes."""
    def gkey(d):
        return (d.fout.idx, d.fin.idx, FFV[(d.fin.flav, d.vec.flav)])
    groups = {}
    for k, d in enumerate(pd.diagrams):
        groups.setdefault(gkey(d), []).append(k)
    bils = {}
    nxt = 10 ** 6
    for key, ks in groups.items():
        if len(ks) > 1:
            d = pd.diagrams[ks[0]]
            bils[key] = Bil(nxt, d.fout, d.fin, key[2])
            nxt += 1

    def need(k):
        d = pd.diagrams[k]
        b = bils.get(gkey(d))
        return [d.vec, b] if b is not None else [d.fout, d.vec, d.fin]

    def closure(nodes, done):
        out, stack = set(), list(nodes)
        while stack:
            n = stack.pop()
            if n.idx in done or n.idx in out:
                continue
            out.add(n.idx)
            stack.extend(_deps(n))
        return out

    # pending[x] = consumers of x (wavefunctions or amplitude terms) not yet emitted
    pending = {}
    seen = set()

    def count(n):
        if n.idx in seen:
            return
        seen.add(n.idx)
        for c in _deps(n):
            pending[c.idx] = pending.get(c.idx, 0) + 1
            count(c)
    for k in range(len(pd.diagrams)):
        for n in need(k):
            pending[n.idx] = pending.get(n.idx, 0) + 1
            count(n)
    nodes = {}

    def reg(n):
        nodes[n.idx] = n
        for c in _deps(n):
            reg(c)
    for k in range(len(pd.diagrams)):
        for n in need(k):
            reg(n)

    def effect(k, done):
        new = closure(need(k), done)
        dec = {}
        for m in new:
            for c in _deps(nodes[m]):
                dec[c.idx] = dec.get(c.idx, 0) + 1
        for n in need(k):
            dec[n.idx] = dec.get(n.idx, 0) + 1
        freed = sum(1 for x, d in dec.items() if pending[x] - d == 0)
        return new, dec, freed

    done = set()
    remaining = list(range(len(pd.diagrams)))
    order = []
    while remaining:
        best, best_key = None, None
        for k in remaining:
            new, dec, freed = effect(k, done)
            key = (len(new) - freed, len(new), k)
            if best_key is None or key < best_key:
                best, best_key = k, key
        new, dec, freed = effect(best, done)
        for x, d in dec.items():
            pending[x] -= d
        remaining.remove(best)
        order.append(best)
        done |= new
    return order, bils, need


def _node_flops(n):
    if isinstance(n, Bil):
        return FLOPS['ffv_bil']
    op = n.op[0]
    if op == 'ext':
        return FLOPS[n.op[2]]
    if op == 'ffv_v':
        return FLOPS['ffv_cur_v0'] if BOSON_MASS[n.op[3]] is None else FLOPS['ffv_cur_vm']
    if op in ('ffv_fout', 'ffv_fin'):
        f, vec = (n.op[1], n.op[2]) if op == 'ffv_fout' else (n.op[2], n.op[1])
        cl, cr = FFV[(f.flav, vec.flav)]
        return FLOPS[f'ffv_cur_{op[4:]}' + ('_v' if cl == cr else '')]
    return FLOPS[{'vvv': 'vvv_cur', 'vvvv': 'vvvv_cur'}[op]]


def schedule_cost(order, need, budget):
    """Executed flops of the wavefunctions (with recomputation) for a
    diagram order under a live-wavefunction budget: the same policy as
    emit_body (compute on first use, evict the farthest next use)."""
    import bisect
    uses_at = {}
    clos = []
    for pos, k in enumerate(order):
        out, stack = {}, list(need(k))
        while stack:
            n = stack.pop()
            if n.idx in out:
                continue
            out[n.idx] = n
            stack.extend(_deps(n))
        clos.append(out)
        for x in out:
            uses_at.setdefault(x, []).append(pos)
    INF = 10 ** 9

    def next_use(x, pos):
        lst = uses_at[x]
        i = bisect.bisect_left(lst, pos)
        return lst[i] if i < len(lst) else INF

    live = {}
    cost = 0

    def ensure(n, pos, pinned):
        nonlocal cost
        if n.idx in live:
            return
        deps = _deps(n)
        pin = pinned | {n.idx} | {d.idx for d in deps}
        for d in deps:
            ensure(d, pos, pin)
        while len(live) >= budget:
            cand = [x for x in live if x not in pin and live[x].op[0] != 'ext']
            if not cand:
                break
            del live[max(cand, key=lambda x: next_use(x, pos))]
        cost += _node_flops(n)
        live[n.idx] = n

    for pos, k in enumerate(order):
        nd = need(k)
        pin = {n.idx for n in nd}
        for n in nd:
            ensure(n, pos, pin)
        for x in list(live):
            if next_use(x, pos + 1) == INF and live[x].op[0] != 'ext':
                del live[x]
    return cost


def optimise_order(order, need, budget, iters=4000, seed=12345):
    """Local search (random moves of one diagram or of a block, accepted
    when the recomputation cost does not grow) over the diagram order."""
    import random
    rng = random.Random(seed)
    best = list(order)
    best_cost = schedule_cost(best, need, budget)
    n = len(best)
    if n < 3:
        return best, best_cost
    for _ in range(iters):
        cand = list(best)
        i, j = sorted(rng.sample(range(n), 2))
        r = rng.random()
        if r < 0.4:
            x = cand.pop(i)
            cand.insert(j, x)
        elif r < 0.7:
            x = cand.pop(j)
            cand.insert(i, x)
        else:
            L = rng.randint(2, min(12, n - i))
            blk = cand[i:i + L]
            del cand[i:i + L]
            k = rng.randint(0, len(cand))
            cand[k:k] = blk
        c = schedule_cost(cand, need, budget)
        if c <= best_cost:
            best, best_cost = cand, c
    return best, best_cost


def _ksum(legs, particles):
    """C++ initialiser of the incoming momentum sum of the given legs."""
    comps = []
    for mu in range(4):
        terms = []
        for l in sorted(legs):
            sign = '+' if particles[l][1] == IN else '-'
            terms.append(f"{sign}p[{l}][{mu}]")
        s = ''.join(terms)
        comps.append(s[1:] if s.startswith('+') else s)
    return '{' + ', '.join(comps) + '}'


def _coef_value(coef, amp):
    c = complex(coef)
    if c == 1:
        return amp
    if c == -1:
        return f"-{amp}"
    if c == 1j:
        return f"times_i({amp})"
    if c == -1j:
        return f"-times_i({amp})"
    return f"cx<T>{{(T){c.real!r}, (T){c.imag!r}}} * {amp}"


def _coef_expr(coef, amp):
    c = complex(coef)
    if c == 1:
        return f"+ {amp}"
    if c == -1:
        return f"- {amp}"
    if c == 1j:
        return f"+ times_i({amp})"
    if c == -1j:
        return f"- times_i({amp})"
    return f"+ cx<T>{{(T){c.real!r}, (T){c.imag!r}}} * {amp}"


def _fermion_width(f, n, parts):
    """(mass, width) coupling names of the propagator of fermion current n:
    a top propagator with exactly one incoming particle on each side (t- or
    u-channel) takes the width 'wtt', which the zero-width flag sets to 0."""
    m, wd = FERMION_MASS[f.flav]
    if wd == 'wt' and sum(1 for l in n.legs if parts[l][1] == IN) == 1:
        wd = 'wtt'
    return m, wd


def _node_code(n, name, dn, parts):
    """C++ statement computing wavefunction n into `name`; dn = names of its
    inputs in op order.  Returns (code, flops)."""
    op = n.op
    if isinstance(n, Bil):
        cl, cr = n.couplings
        return (f"cx<T> {name}[4]; ffv_bilinear<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, {name});",
                FLOPS['ffv_bil'])
    K = _ksum(n.legs, parts)
    if op[0] == 'vvv':
        a, b = op[1], op[2]
        return (f"cx<T> {name}[4]; {{ const R KA[4] = {_ksum(a.legs, parts)}; "
                f"const R KB[4] = {_ksum(b.legs, parts)}; "
                f"vvv_cur<T>({dn[0]}, KA, {dn[1]}, KB, c.gs, {name}); }}", FLOPS['vvv_cur'])
    if op[0] == 'vvvv':
        s = op[1]
        return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                f"vvvv_cur<{s}, T>({dn[0]}, {dn[1]}, {dn[2]}, K, c.gs2, {name}); }}",
                FLOPS['vvvv_cur'])
    if op[0] == 'ffv_fout':
        f, vec = op[1], op[2]
        cl, cr = FFV[(f.flav, vec.flav)]
        m, wd = _fermion_width(f, n, parts)
        if cl == cr:
            return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                    f"ffv_cur_fout_v<T>({dn[0]}, {dn[1]}, c.{cl}, K, c.{m}, c.{wd}, {name}); }}",
                    FLOPS['ffv_cur_fout_v'])
        return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                f"ffv_cur_fout<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, c.{m}, c.{wd}, {name}); }}",
                FLOPS['ffv_cur_fout'])
    if op[0] == 'ffv_fin':
        vec, f = op[1], op[2]
        cl, cr = FFV[(f.flav, vec.flav)]
        m, wd = _fermion_width(f, n, parts)
        if cl == cr:
            return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                    f"ffv_cur_fin_v<T>({dn[0]}, {dn[1]}, c.{cl}, K, c.{m}, c.{wd}, {name}); }}",
                    FLOPS['ffv_cur_fin_v'])
        return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                f"ffv_cur_fin<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, c.{m}, c.{wd}, {name}); }}",
                FLOPS['ffv_cur_fin'])
    if op[0] == 'ffv_v':
        fo, fi, boson = op[1], op[2], op[3]
        cl, cr = FFV[(fo.flav, boson)]
        bm = BOSON_MASS[boson]
        if bm is None:
            return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                    f"ffv_cur_v0<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, {name}); }}",
                    FLOPS['ffv_cur_v0'])
        return (f"cx<T> {name}[4]; {{ const R K[4] = {K}; "
                f"ffv_cur_vm<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, c.{bm[0]}, c.{bm[1]}, {name}); }}",
                FLOPS['ffv_cur_vm'])
    raise ValueError(op)


def _ext_code(n, name, npar):
    l, routine = n.op[1], n.op[2]
    hel = f"((hcode >> {npar - 1 - l}) & 1u) ? 1 : -1"
    p = f"p[{l}]"
    if routine in ('vec_in', 'vec_out'):
        return (f"cx<T> {name}[4]; ext_vector<T>({p}, {hel}, "
                f"{'false' if routine == 'vec_in' else 'true'}, {name});", FLOPS[routine])
    mass = {'t': 'c.mt'}.get(n.flav, '0.0')
    fn = {'ubar': ('ext_u', 'true'), 'u': ('ext_u', 'false'),
          'v': ('ext_v', 'false'), 'vbar': ('ext_v', 'true')}[routine]
    return f"cx<T> {name}[4]; {fn[0]}<T>({p}, {mass}, {hel}, {fn[1]}, {name});", FLOPS[routine]


def emit_body(pd, coefs, order, bils, need, budget, fence_every=4):
    """Straight-line body of jamps() for one register budget (in live
    wavefunctions).  Wavefunctions are computed on first use; when the
    budget is full the live one whose next use is farthest is dropped
    (Belady) and recomputed when needed again, its input passed through an
    opaque copy so the compiler cannot merge the two computations back into
    one long-lived value.  Returns (lines, algorithmic flops, executed
    flops, peak live, recomputations)."""
    import bisect
    parts = pd.particles
    npar = pd.npar

    def full_closure(nodes):
        out, stack = {}, list(nodes)
        while stack:
            n = stack.pop()
            if n.idx in out:
                continue
            out[n.idx] = n
            stack.extend(_deps(n))
        return out

    uses_at = {}
    for pos, k in enumerate(order):
        for x in full_closure(need(k)):
            uses_at.setdefault(x, []).append(pos)
    INF = 10 ** 9

    def next_use(x, pos):
        lst = uses_at.get(x, [])
        i = bisect.bisect_left(lst, pos)
        return lst[i] if i < len(lst) else INF

    live = {}
    version = {}
    L = []
    algo, execd = 0, 0
    peak, recomputes = 0, 0
    computed_once = set()

    def evict(pos, pinned):
        while len(live) >= budget:
            cand = [x for x in live if x not in pinned and live[x][1].op[0] != 'ext']
            if not cand:
                return
            victim = max(cand, key=lambda x: next_use(x, pos))
            del live[victim]

    def ensure(n, pos, pinned):
        nonlocal algo, execd, peak, recomputes
        if n.idx in live:
            return live[n.idx][0]
        deps = _deps(n)
        pin = set(pinned) | {n.idx} | {d.idx for d in deps}
        dn = [ensure(d, pos, pin) for d in deps]
        evict(pos, pin)
        v = version.get(n.idx, 0)
        version[n.idx] = v + 1
        base = f"b{n.idx - 10 ** 6}" if isinstance(n, Bil) else f"w{n.idx}"
        name = base if v == 0 else f"{base}_{v}"
        if n.op[0] == 'ext':
            code, fl = _ext_code(n, name, npar)
            if v > 0:
                recomputes += 1
        else:
            if v > 0:  # opaque copy of one input defeats common-subexpression merging
                L.append(f"  cx<T> o{n.idx}_{v}[4] = {{{dn[0]}[0], {dn[0]}[1], {dn[0]}[2], {dn[0]}[3]}}; "
                         f"opaque4(o{n.idx}_{v});")
                dn = [f"o{n.idx}_{v}"] + dn[1:]
                recomputes += 1
            code, fl = _node_code(n, name, dn, parts)
        L.append("  " + code)
        execd += fl
        if n.idx not in computed_once:
            computed_once.add(n.idx)
            algo += fl
        live[n.idx] = (name, n)
        peak = max(peak, len(live))
        return name

    for pos, k in enumerate(order):
        d, cf = pd.diagrams[k], coefs[k]
        nd = need(k)
        pin = {n.idx for n in nd}
        if pos % fence_every == 0:
            L.append("  fence<UNI, BEAM>(p);")
        names = [ensure(n, pos, pin) for n in nd]
        cl, cr = FFV[(d.fin.flav, d.vec.flav)]
        if len(nd) == 2:   # shared bilinear . vector
            L.append(f"  {{ const cx<T> a = times_i(mdot({names[0]}, {names[1]}));")
            fl = FLOPS['amp_dot']
        elif cl == cr:
            L.append(f"  {{ const cx<T> a = ffv_amp_v<T>({names[0]}, {names[1]}, {names[2]}, "
                     f"c.{cl});")
            fl = FLOPS['ffv_amp_v']
        else:
            L.append(f"  {{ const cx<T> a = ffv_amp<T>({names[0]}, {names[1]}, {names[2]}, "
                     f"c.{cl}, c.{cr});")
            fl = FLOPS['ffv_amp']
        algo += fl
        execd += fl
        for kk, coef in sorted(cf.items()):
            L.append(f"    jacc(J[{kk}], {_coef_value(coef, 'a')});")
            algo += FLOPS['jamp_acc']
            execd += FLOPS['jamp_acc']
        L.append("  }")
        for x in list(live):
            if next_use(x, pos + 1) == INF and live[x][1].op[0] != 'ext':
                del live[x]
    return L, algo, execd, peak, recomputes



# ----------------------------------------------------------------------------
# reverse mode
# ----------------------------------------------------------------------------
ADJ_FLOPS = {  # algorithmic flops of the adjoint routines of helas_adj.h
    'ffv_amp': 118 + 64 + 160, 'mdot_i': 64, 'bilinear': 160,
    'ffv_cur_v0': 16 + 160 + 16 + 12, 'ffv_cur_vm': 88 + 200 + 16 + 60,
    'ffv_cur_fin': 200 + 60 + 120, 'ffv_cur_fout': 200 + 60 + 120,
    'vvv_cur': 260, 'vvvv_cur': 230, 'ext': 4 * 110, 'jbar': 0,
}


def _legs_of(n):
    if isinstance(n, Bil):
        return n.fout.legs | n.fin.legs
    return n.legs


def emit_adjoint_body(pd, coefs, order, bils, need, budget, lds=False, lds_span=0, spans=None):
    """Reverse sweep of jamps() for one helicity: the colour-flow adjoints
    Jb (already formed) are propagated back through the amplitude terms (in
    reverse order) and the wavefunctions (each once all its consumers are
    done) to the external momenta, accumulated into pb[leg][mu] for the
    final-state legs.  Forward values are recomputed from the externals
    under the same live-wavefunction budget as the forward code (Belady
    eviction).  Wavefunctions whose legs are all initial-state carry no
    momentum dependence and are not differentiated.  With lds the adjoint
    accumulators live in slots of the workgroup's LDS (ws.slot(s), reused
    once a wavefunction has been back-propagated) instead of registers,
    except those open for at most lds_span steps (spans: {node: steps} of a
    previous pass; short-lived ones stay in registers).  Returns (lines,
    executed flops, number of slots, {node: steps open})."""
    import bisect
    parts = pd.particles
    npar = pd.npar

    def final(n):
        return any(parts[l][1] == OUT for l in _legs_of(n))

    def closure(nodes):
        out, stack = {}, list(nodes)
        while stack:
            n = stack.pop()
            if n.idx in out:
                continue
            out[n.idx] = n
            stack.extend(_deps(n))
        return out

    first_use = {}
    nodes = {}
    for pos, k in enumerate(order):
        for x, n in closure(need(k)).items():
            first_use.setdefault(x, pos)
            nodes[x] = n
    # reverse step list: ('amp', pos) then ('node', n) for the nodes first
    # used at pos, larger leg sets (consumers) first
    steps = []
    for pos in reversed(range(len(order))):
        steps.append(('amp', pos, list(need(order[pos]))))
        born = [nodes[x] for x, f in first_use.items() if f == pos]
        born.sort(key=lambda n: (-len(_legs_of(n)), -n.idx))
        for n in born:
            if final(n):
                steps.append(('node', n, _deps(n)))
    uses_at = {}
    for si, st in enumerate(steps):
        for x in closure(st[2]):
            uses_at.setdefault(x, []).append(si)
    INF = 10 ** 9

    def next_use(x, si):
        lst = uses_at.get(x, [])
        i = bisect.bisect_left(lst, si)
        return lst[i] if i < len(lst) else INF

    live = {}
    version = {}
    L = []
    execd = 0

    def evict(si, pinned):
        while len(live) >= budget:
            cand = [x for x in live if x not in pinned and live[x][1].op[0] != 'ext']
            if not cand:
                return
            del live[max(cand, key=lambda x: next_use(x, si))]

    def ensure(n, si, pinned):
        nonlocal execd
        if n.idx in live:
            return live[n.idx][0]
        deps = _deps(n)
        pin = set(pinned) | {n.idx} | {d.idx for d in deps}
        dn = [ensure(d, si, pin) for d in deps]
        evict(si, pin)
        v = version.get(n.idx, 0)
        version[n.idx] = v + 1
        base = f"rb{n.idx - 10 ** 6}" if isinstance(n, Bil) else f"rw{n.idx}"
        name = f"{base}_{v}"
        if n.op[0] == 'ext':
            code, fl = _ext_code(n, name, npar)
        else:
            if v > 0:
                L.append(f"  cx<T> o{name}[4] = {{{dn[0]}[0], {dn[0]}[1], {dn[0]}[2], {dn[0]}[3]}}; "
                         f"opaque4(o{name});")
                dn = [f"o{name}"] + dn[1:]
            code, fl = _node_code(n, name, dn, parts)
        L.append("  " + code)
        execd += fl
        live[n.idx] = (name, n)
        return name

    declared = set()
    slot_of, free_slots, nslots = {}, [], [0]
    opened, span_of = {}, {}
    cur_step = [0]

    def in_lds(n):
        return lds and (spans is None or spans.get(n.idx, 10 ** 9) > lds_span)

    def bar(n):
        """Name of n's adjoint accumulator (declared on first use), or a sink."""
        if not final(n):
            return None
        opened.setdefault(n.idx, cur_step[0])
        if in_lds(n):
            if n.idx not in slot_of:
                if free_slots:
                    slot_of[n.idx] = free_slots.pop()
                else:
                    slot_of[n.idx] = nslots[0]
                    nslots[0] += 1
                L.append(f"  ws.clear({slot_of[n.idx]});")
            return f"ws.slot({slot_of[n.idx]})"
        nm = f"wb{n.idx - 10 ** 6}b" if isinstance(n, Bil) else f"wb{n.idx}"
        if n.idx not in declared:
            declared.add(n.idx)
            L.append(f"  cx<T> {nm}[4] = {{{{(T)0, (T)0}}, {{(T)0, (T)0}}, {{(T)0, (T)0}}, {{(T)0, (T)0}}}};")
        return nm

    def release(n):
        """n has been back-propagated: its slot takes the next accumulator."""
        if n.idx in opened:
            span_of[n.idx] = cur_step[0] - opened[n.idx]
        if n.idx in slot_of:
            free_slots.append(slot_of.pop(n.idx))

    sink_count = [0]

    def acc(n):
        nm = bar(n)
        if nm is None:
            sink_count[0] += 1
            nm = f"sink{sink_count[0]}"
            L.append(f"  cx<T> {nm}[4] = {{}};")
        return nm

    def kback(legs, kname):
        for l in sorted(legs):
            if parts[l][1] == OUT:
                L.append(f"  for (int m = 0; m < 4; ++m) pb[{l}][m] -= (double){kname}[m];")

    for si, st in enumerate(steps):
        cur_step[0] = si
        if si % ADJ_FENCE_EVERY == 0:
            L.append("  fence<UNI, BEAM>(p);")
        if st[0] == 'amp':
            pos, nd = st[1], st[2]
            k = order[pos]
            d = pd.diagrams[k]
            pin = {n.idx for n in nd}
            names = [ensure(n, si, pin) for n in nd]
            terms = []
            for kk, coef in sorted(coefs[k].items()):
                terms.append(_coef_expr(complex(coef).conjugate(), f"Jb[{kk}]"))
            expr = " ".join(terms)
            expr = expr[2:] if expr.startswith('+ ') else expr
            an = [acc(x) for x in nd]
            L.append(f"  {{ const cx<T> ab = {expr};")
            if len(nd) == 2:
                L.append(f"    adj_mdot_i({names[0]}, {names[1]}, ab, {an[0]}, {an[1]}); }}")
                execd += ADJ_FLOPS['mdot_i']
            else:
                cl, cr = FFV[(d.fin.flav, d.vec.flav)]
                L.append(f"    adj_ffv_amp<T>({names[0]}, {names[1]}, {names[2]}, c.{cl}, c.{cr}, ab, "
                         f"{an[0]}, {an[1]}, {an[2]}); }}")
                execd += ADJ_FLOPS['ffv_amp']
        else:
            n, deps = st[1], st[2]
            pin = {n.idx} | {x.idx for x in deps}
            dn = [ensure(x, si, pin) for x in deps]
            wb = bar(n)
            op = n.op
            if isinstance(n, Bil):
                cl, cr = n.couplings
                L.append(f"  adj_bilinear<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, {wb}, "
                         f"{acc(deps[0])}, {acc(deps[1])});")
                execd += ADJ_FLOPS['bilinear']
                release(n)
                continue
            if op[0] == 'ext':
                l, routine = op[1], op[2]
                if parts[l][1] != OUT:
                    continue
                hel = f"((hcode >> {npar - 1 - l}) & 1u) ? 1 : -1"
                if routine in ('vec_in', 'vec_out'):
                    L.append(f"  adj_ext_vector<T>(p[{l}], {hel}, "
                             f"{'false' if routine == 'vec_in' else 'true'}, {wb}, pb[{l}]);")
                else:
                    mass = {'t': 'c.mt'}.get(n.flav, '0.0')
                    fn = {'ubar': ('adj_ext_u', 'true'), 'u': ('adj_ext_u', 'false'),
                          'v': ('adj_ext_v', 'false'), 'vbar': ('adj_ext_v', 'true')}[routine]
                    L.append(f"  {fn[0]}<T>(p[{l}], {mass}, {hel}, {fn[1]}, {wb}, pb[{l}]);")
                execd += ADJ_FLOPS['ext']
                release(n)
                continue
            K = _ksum(n.legs, parts)
            accs = {x.idx: acc(x) for x in deps}
            L.append("  {")
            if op[0] == 'vvv':
                a, b = op[1], op[2]
                L.append(f"    const R KA[4] = {_ksum(a.legs, parts)}; const R KB[4] = {_ksum(b.legs, parts)};")
                L.append("    T KAb[4] = {(T)0, (T)0, (T)0, (T)0}, KBb[4] = {(T)0, (T)0, (T)0, (T)0};")
                L.append(f"    adj_vvv_cur<T>({dn[0]}, KA, {dn[1]}, KB, c.gs, {wb}, {accs[a.idx]}, KAb, "
                         f"{accs[b.idx]}, KBb);")
                for legs, kn in ((a.legs, 'KAb'), (b.legs, 'KBb')):
                    for l in sorted(legs):
                        if parts[l][1] == OUT:
                            L.append(f"    for (int m = 0; m < 4; ++m) pb[{l}][m] -= (double){kn}[m];")
                execd += ADJ_FLOPS['vvv_cur']
            else:
                L.append(f"    const R K[4] = {K}; T Kb[4] = {{(T)0, (T)0, (T)0, (T)0}};")
                if op[0] == 'vvvv':
                    sgn, x, y, z = op[1], op[2], op[3], op[4]
                    L.append(f"    adj_vvvv_cur<{sgn}, T>({dn[0]}, {dn[1]}, {dn[2]}, K, c.gs2, {wb}, "
                             f"{accs[x.idx]}, {accs[y.idx]}, {accs[z.idx]}, Kb);")
                    execd += ADJ_FLOPS['vvvv_cur']
                elif op[0] == 'ffv_fout':
                    f, vec = op[1], op[2]
                    cl, cr = FFV[(f.flav, vec.flav)]
                    m, wd = _fermion_width(f, n, parts)
                    L.append(f"    adj_ffv_cur_fout<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, c.{m}, c.{wd}, "
                             f"{wb}, {accs[f.idx]}, {accs[vec.idx]}, Kb);")
                    execd += ADJ_FLOPS['ffv_cur_fout']
                elif op[0] == 'ffv_fin':
                    vec, f = op[1], op[2]
                    cl, cr = FFV[(f.flav, vec.flav)]
                    m, wd = _fermion_width(f, n, parts)
                    L.append(f"    adj_ffv_cur_fin<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, c.{m}, c.{wd}, "
                             f"{wb}, {accs[vec.idx]}, {accs[f.idx]}, Kb);")
                    execd += ADJ_FLOPS['ffv_cur_fin']
                elif op[0] == 'ffv_v':
                    fo, fi, boson = op[1], op[2], op[3]
                    cl, cr = FFV[(fo.flav, boson)]
                    bm = BOSON_MASS[boson]
                    if bm is None:
                        L.append(f"    adj_ffv_cur_v0<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, {wb}, "
                                 f"{accs[fo.idx]}, {accs[fi.idx]}, Kb);")
                        execd += ADJ_FLOPS['ffv_cur_v0']
                    else:
                        L.append(f"    adj_ffv_cur_vm<T>({dn[0]}, {dn[1]}, c.{cl}, c.{cr}, K, c.{bm[0]}, "
                                 f"c.{bm[1]}, {wb}, {accs[fo.idx]}, {accs[fi.idx]}, Kb);")
                        execd += ADJ_FLOPS['ffv_cur_vm']
                else:
                    raise ValueError(op)
                for l in sorted(n.legs):
                    if parts[l][1] == OUT:
                        L.append(f"    for (int m = 0; m < 4; ++m) pb[{l}][m] -= (double)Kb[m];")
            L.append("  }")
            release(n)
    return L, execd, nslots[0], span_of


# register budget in live wavefunctions (4 complex each) per precision, the
# measured best for gg -> t t~ g g on gfx950 (FP64 wavefunctions take 16
# VGPRs, FP32 ones 8, fewer where components are zero at compile time; the
# colour-flow amplitudes stay live besides them).  With the beam bodies
# (2^19 events, ms): FP64 one helicity per lane 14: 19.5, 16: 19.4, 18:
# 19.1-19.2, 20: 19.6 (404 B of spills per lane); FP32 one helicity per lane
# 13: 13.4, 15: 13.2-13.3, the largest budget that fits 256 registers (two
# waves per SIMD; 17 needs AGPRs, one wave per SIMD: 16.4).  'f32m' is the
# FP32 body of the event-per-lane kernel whose colour sum runs on the matrix
# cores (28: 23.8, 36: 26.1 M MEs/s before the beam bodies).  The gradient
# kernel (gg -> t t~ g, 2^18 events): FP64 budget 8: 4.19 ms, 12 or 14:
# 4.0-4.1 ms.
BUDGET = {'f64': 18, 'f32': 15, 'f32m': 36, 'a64': 12, 'a32': 12}
# processes with a generated reverse-mode (adjoint) body for the gradient kernel
GRAD_PROCESSES = ('eemumu', 'ggtt', 'ggttg')
# local-search moves over the diagram order (gg -> t t~ g g at FP64 budget 16:
# 2500 moves leave 4.5k recomputed flops per helicity, 20000 leave 3.5k)
OPT_ITERS = 20000
# amplitude terms between two scheduling fences per precision (gg -> t t~ g g:
# without fences FP64 halves its throughput; between 2 and 8 it moves by
# under 1 %; FP32 one helicity per lane gains 4 % from 4 to 8 and loses 30 %
# at 16; the mixed kernel gains 1 % from 4 to 12)
FENCE = {'f64': 4, 'f32': 8, 'f32m': 12, 'a64': 4, 'a32': 4}


# reverse-sweep steps between two fences in the adjoint code
ADJ_FENCE_EVERY = int(os.environ.get('MG_ADJ_FENCE_EVERY', 4))


# (process, precision) pairs whose adjoint accumulators live in LDS slots
# (MG_ADJ_LDS=ggttg:a64,...; 'none' for none).  FP64 g g -> t t~ g: in
# registers its reverse sweep needs 512 registers and 1.8 KB of scratch per
# lane (10.1 ms for 2^18 events); with the accumulators open for more than 6
# reverse steps in 8 LDS slots (36.9 KB per wave, four waves per CU) 6.1 ms.
# Its FP32 sweep fits registers better and runs slower from LDS (5.3 against
# 4.3 ms), as do the smaller processes, which do not spill.
ADJ_LDS = tuple(tuple(x.split(':')) for x in
                os.environ.get('MG_ADJ_LDS', 'ggttg:a64').split(',') if ':' in x)
# accumulators open for at most this many reverse steps stay in registers
# (g g -> t t~ g: 6 -> 8 slots, 6.1 ms; 8 -> 7 slots, 6.2 ms; 12 -> 6 slots,
# 6.7 ms; 0 -> 9 slots, 46 KB, three waves per CU, 9.4 ms)
ADJ_LDS_SPAN = int(os.environ.get('MG_ADJ_LDS_SPAN', 6))


def _adj_lds(name, prec):
    return (name, prec) in ADJ_LDS


def _fence(prec):
    return int(os.environ.get(f'MG_FENCE_{prec.upper()}', FENCE[prec]))


def _optimised_order(args):
    """Worker: the optimised diagram order of process `name` for `budget`
    (rebuilds the deterministic diagram set and greedy schedule)."""
    name, budget = args
    pd = ProcessDiagrams(name)
    order0, _, need = schedule(pd)
    if schedule_cost(order0, need, budget) <= schedule_cost(order0, need, 10 ** 6):
        return order0
    return optimise_order(order0, need, budget, iters=OPT_ITERS)[0]


def _budget(prec):
    return int(os.environ.get(f'MG_BUDGET_{prec.upper()}', BUDGET[prec]))


def _variant_precs(name):
    return ['f64', 'f32', 'f32m'] + (['a64', 'a32'] if name in GRAD_PROCESSES else [])


def optimised_orders(names):
    """{(process, budget): order} for every budget the processes' variants
    use, the local searches running in parallel processes."""
    import multiprocessing as mp
    jobs = sorted({(n, _budget(p)) for n in names for p in _variant_precs(n)})
    with mp.get_context('fork').Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        res = pool.map(_optimised_order, jobs)
    return dict(zip(jobs, res))


def generate(name, orders=None):
    pd = ProcessDiagrams(name)
    npar = pd.npar
    basis = pd.colour_basis() if pd.gluons else [()]
    ncol = len(basis)
    if pd.gluons:
        cnum, cden = colour_matrix(basis, len(pd.gluons))
    else:
        cnum, cden = [[1]], 1
    coefs = pd.jamp_coefficients()
    order0, bils, need = schedule(pd)
    L = []
    w = L.append
    w(f"// Generated for {name}: do not edit.  {pd.ndiagrams} diagrams, "
      f"{len(pd.diagrams)} amplitude terms, {len(pd.used) - npar} currents, "
      f"{len(bils)} shared bilinears.")
    w(f"namespace gen_{name} {{")
    w(f"constexpr int NPAR = {npar};")
    w(f"constexpr int NCOL = {ncol};")
    w(f"constexpr int NDIAG = {pd.ndiagrams};")
    w(f"constexpr int NAMP = {len(pd.diagrams)};")
    w(f"constexpr int IDEN = {IDEN[name]};")
    w(f"constexpr int CDEN = {cden};")
    w(f"__device__ constexpr int CNUM[{ncol}][{ncol}] = {{")
    for row in cnum:
        w("  {" + ", ".join(str(x) for x in row) + "},")
    w("};")
    f32t, bf16t = colour_mfma_tables(cnum, ncol)
    w("// A operands of the matrix-core colour sum (colour_mfma.h), per K block and lane")
    w(f"__device__ const float CS_A_F32[{len(f32t)}][64] = {{")
    for row in f32t:
        w("  {" + ", ".join(f"{v:.1f}f" for v in row) + "},")
    w("};")
    w(f"__device__ const unsigned CS_A_BF16[{len(bf16t)}][64][4] __attribute__((aligned(16))) = {{")
    for row in bf16t:
        w("  {" + ", ".join("{" + ", ".join(f"0x{x:08x}u" for x in words) + "}" for words in row) + "},")
    w("};")
    w("")
    stats = {}
    variants = [('f64', 'double', 'double', 'double'), ('f32', 'float', 'double', 'float'),
                ('f32m', 'float', 'double', 'float')]
    if orders is None:
        orders = optimised_orders([name])
    for prec, T, Rt, Ct in variants:
        budget = _budget(prec)
        order = orders[(name, budget)]
        body, algo, execd, peak, rec = emit_body(pd, coefs, order, bils, need, budget,
                                                 fence_every=_fence(prec))
        stats[prec] = dict(flops_amp_per_hel=algo, flops_executed_per_hel=execd,
                           peak_live_wavefunctions=peak, recomputed=rec)
        jparam = f"cx<{T}> (&J)[{ncol}]"
        w("// UNI: momenta the same in every lane (scalar registers); BEAM: the two")
        w("// incoming momenta (E,0,0,E) and (E,0,0,-E) with constant zero components")
        w("template <bool UNI = false, bool BEAM = false>")
        w(f"__device__ __forceinline__ void jamps_{prec}({Rt} (&p)[{npar}][4], unsigned hcode,")
        w(f"                                          const Couplings<{Ct}>& c, {jparam}) {{")
        w(f"  using T = {T};")
        w(f"  using R = {Rt};")
        for k in range(ncol):
            w(f"  J[{k}] = cx<T>{{(T)0, (T)0}};")
        L.extend(body)
        w("}")
        w("")
    w("template <typename T, bool UNI = false, bool BEAM = false>")
    w(f"__device__ __forceinline__ void jamps(double (&p)[{npar}][4], unsigned hcode,")
    w(f"                                      const Couplings<T>& c, cx<T> (&J)[{ncol}]) {{")
    w("  if constexpr (sizeof(T) == 8) jamps_f64<UNI, BEAM>(p, hcode, c, J);")
    w("  else jamps_f32<UNI, BEAM>(p, hcode, c, J);")
    w("}")
    w("")
    # colour sum: sum_i J_i^* (sum_j C_ij J_j) using the symmetry of C
    cs_flops = 0
    w("template <typename T>")
    w(f"__device__ __forceinline__ T colour_sum(const cx<T> (&J)[{ncol}]) {{")
    w("  T me = (T)0;")
    for i in range(ncol):
        terms_r = [f"(T){cnum[i][i]} * J[{i}].r"]
        terms_i = [f"(T){cnum[i][i]} * J[{i}].i"]
        for j in range(i + 1, ncol):
            if cnum[i][j]:
                terms_r.append(f"(T){2 * cnum[i][j]} * J[{j}].r")
                terms_i.append(f"(T){2 * cnum[i][j]} * J[{j}].i")
        w(f"  {{ const T zr = {' + '.join(terms_r)};")
        w(f"    const T zi = {' + '.join(terms_i)};")
        w(f"    me += J[{i}].r * zr + J[{i}].i * zi; }}")
        cs_flops += 2 * (2 * len(terms_r) - 1) + 4
    w(f"  return me * (T){1.0 / cden!r};")
    w("}")
    A = []
    if name in GRAD_PROCESSES:
        for prec, T, Ct in (('a64', 'double', 'double'), ('a32', 'float', 'float')):
            budget = _budget(prec)
            order = orders[(name, budget)]
            fwd, algo, execd, peak, rec = emit_body(pd, coefs, order, bils, need, budget,
                                                    fence_every=_fence(prec))
            _, _, _, spans = emit_adjoint_body(pd, coefs, order, bils, need, budget)
            rev, rexec, nslots, _ = emit_adjoint_body(pd, coefs, order, bils, need, budget,
                                                      lds=_adj_lds(name, prec), lds_span=ADJ_LDS_SPAN,
                                                      spans=spans)
            stats[prec] = dict(flops_forward_executed_per_hel=execd, flops_reverse_executed_per_hel=rexec,
                               adjoint_lds_slots=nslots)
            A.append(f"// LDS slots of the adjoint accumulators (0: kept in registers)")
            A.append(f"constexpr int ADJ_SLOTS_{prec} = {nslots};")
            A.append(f"// reverse mode: returns the colour-summed |M|^2 of helicity hcode and adds")
            A.append(f"// its gradient with respect to the momenta of the final-state legs to pb;")
            A.append(f"// ws: the lane's adjoint slots (ws.slot(s), ws.clear(s)) when ADJ_SLOTS > 0;")
            A.append(f"// BEAM: the incoming momenta on the axis with constant zero components")
            A.append(f"template <bool BEAM, class WS>")
            A.append(f"__device__ __forceinline__ double adjoint_{prec}(double (&p)[{npar}][4], unsigned hcode,")
            A.append(f"                                            const Couplings<{Ct}>& c,")
            A.append(f"                                            double (&pb)[{npar}][4], const WS& ws) {{")
            A.append(f"  using T = {T};")
            A.append(f"  using R = double;")
            A.append(f"  constexpr bool UNI = false;")
            A.append(f"  cx<T> J[{ncol}];")
            for k in range(ncol):
                A.append(f"  J[{k}] = cx<T>{{(T)0, (T)0}};")
            A.append("  {")
            A.extend(fwd)
            A.append("  }")
            A.append(f"  const T me = colour_sum<T>(J);")
            A.append(f"  cx<T> Jb[{ncol}];")
            for i in range(ncol):
                tr = " + ".join(f"(T){cnum[i][j]} * J[{j}].r" for j in range(ncol) if cnum[i][j])
                ti = " + ".join(f"(T){cnum[i][j]} * J[{j}].i" for j in range(ncol) if cnum[i][j])
                A.append(f"  Jb[{i}] = cx<T>{{(T){2.0 / cden!r} * ({tr}), (T){2.0 / cden!r} * ({ti})}};")
            A.append("  {")
            A.extend(rev)
            A.append("  }")
            A.append("  return (double)me;")
            A.append("}")
            A.append("")
    L.extend(A)
    w(f"}}  // namespace gen_{name}")
    cs_flops += 1
    meta = {
        'process': name, 'npar': npar, 'ncol': ncol, 'ndiag': pd.ndiagrams,
        'namp': len(pd.diagrams), 'ncurrents': len(pd.used) - npar, 'nbilinears': len(bils),
        'flops_amp_per_hel': stats['f64']['flops_amp_per_hel'],
        'flops_colour_per_hel': cs_flops,
        'schedule': stats,
        'iden': IDEN[name], 'cden': cden,
    }
    return "\n".join(L) + "\n", meta


# One event per wave and one helicity per lane: the processes whose 64
# helicities fill a wave64 (all kept at the benchmark parameters).
HPL_PROCESSES = ('ggttgg',)
# Launches of fewer events than this use the group kernel (one kept helicity
# per lane, several lanes per event) instead of the event-per-lane kernel:
# the crossovers of the events-per-launch sweep (FP64, SIGMAKIN only; group
# against event per lane with the momenta loaded once: e+e- -> mu+mu- 1.4x
# at 4096-16384 events, 1.22x at 2^15, 0.94x at 2^16, 0.77x at 2^20;
# g g -> t t~ 4.0x at 4096, 1.55x at 2^15, 0.96x at 2^16; g g -> t t~ g 8.0x
# at 4096, 1.36x at 2^15, 0.77x at 2^16)
GROUP_MAX_EVENTS = {'eemumu': 1 << 16, 'ggtt': 1 << 16, 'ggttg': 1 << 16}
# Processes whose event-per-lane kernels re-read the momenta for every
# helicity (REREAD_MOMENTA, sigmakin_impl.h): those whose amplitude code
# fills the register file.  The others load them once per event and compute
# the helicity-independent parts once (2^20 events, FP64 / FP32 amplitudes /
# mixed, against re-reading: e+e- -> mu+mu- (2^24) +18 % / - / +14 %,
# g g -> t t~ +3.5 % / +11 % / +9 %, g g -> t t~ g +4.4 % / - / -13 %: the
# mixed kernel then needs 274 registers, one wave per SIMD).
REREAD_MOMENTA = {'sigmakin': ('ggttgg',), 'mixed': ('ggttg', 'ggttgg')}


def _cbool(b):
    return 'true' if b else 'false'


def emit_units(name):
    """{file name: source} of the translation units that instantiate the
    kernels of sigmakin_impl.h and adjoint_impl.h for one process: the
    process traits (amplitude bodies and colour sum of the generated code)
    and the launchers the C ABI calls, per precision."""
    hpl = name in HPL_PROCESSES
    head = (f'// Generated for {name}: do not edit.  Kernels of sigmakin_impl.h for this\n'
            f'// process, {{what}}.\n')
    traits = f'''struct P_{name} {{
  static constexpr bool REREAD_MOMENTA = {{reread}};
  static constexpr int NPAR = gen_{name}::NPAR;
  static constexpr int NCOL = gen_{name}::NCOL;
  static constexpr int CDEN = gen_{name}::CDEN;
  __device__ static __forceinline__ const float* cs_a_f32() {{ return &gen_{name}::CS_A_F32[0][0]; }}
  __device__ static __forceinline__ const unsigned* cs_a_bf16() {{ return &gen_{name}::CS_A_BF16[0][0][0]; }}
  template <typename T, bool UNI = false, bool BEAM = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<T>& c, cx<T> (&J)[NCOL]) {{
    gen_{name}::{{body}}(p, h, c, J);
  }}
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {{
    return gen_{name}::colour_sum<T>(J);
  }}
}};
'''
    sk_args = '(const MeArgs& a, const double* mom, int64_t nevt, double* me, const double* wgt,\n' \
              '    double* evtw, double* mehel, hipStream_t s)'
    units = {}
    for prec, T, c in (('f64', 'double', 'c64'), ('f32', 'float', 'c32')):
        epl = (f'sigmakin_group_launch<P_{name}, {T}, MG_EPL_BLOCK>(a, a.{c}, mom, nevt, me, wgt, evtw,\n'
               f'      mehel, group_max_events({GROUP_MAX_EVENTS.get(name, 0)}), s)')
        if hpl:
            body = (f'#ifdef MG_EVENT_PER_LANE_{prec.upper()}\n'
                    f'  return sigmakin_launch<P_{name}, {T}, 64>(a, a.{c}, mom, nevt, me, wgt, evtw, mehel, s);\n'
                    f'#else\n'
                    f'  return sigmakin_hpl_launch<P_{name}, {T}, 64>(a, a.{c}, mom, nevt, me, wgt, evtw, mehel, s);\n'
                    f'#endif\n')
        else:
            body = f'  return {epl};\n'
        src = head.format(what=f'{T} amplitudes') + '#include "sigmakin_impl.h"\n\nnamespace mg {\n' \
            f'#include "{name}.inc"\n\n' + traits.replace('{body}', 'jamps<T, UNI, BEAM>').replace(
                '{reread}', _cbool(name in REREAD_MOMENTA['sigmakin'])) + '\n' \
            f'int launch_sigmakin_{name}_{prec}{sk_args} {{\n{body}}}\n'
        if prec == 'f64':
            src += (f'\n// FP64 recomputation of the ill-conditioned events of a reduced-precision\n'
                    f'// launch (precision guard of sigmakin_impl.h)\n'
                    f'int launch_sigmakin_{name}_guard(const MeArgs& a, const double* mom, int64_t nevt,\n'
                    f'    double* me, const double* wgt, double* evtw, hipStream_t s) {{\n'
                    f'  return sigmakin_guard_launch<P_{name}>(a, mom, nevt, me, wgt, evtw, s);\n}}\n')
        units[f'sigmakin_{name}_{prec}.hip'] = src + '\n}  // namespace mg\n'
    # mixed: event-per-lane body for the matrix-core colour sum (jamps_f32m)
    # and, for the helicity-per-lane processes, the FP32 body of that kernel
    mt = traits.replace('{body}', 'jamps_f32m<UNI, BEAM>').replace(
        '{reread}', _cbool(name in REREAD_MOMENTA['mixed']))
    mt = mt.replace('const Couplings<T>& c, cx<T> (&J)[NCOL]', 'const Couplings<float>& c, cx<float> (&J)[NCOL]')
    src = head.format(what='FP32 amplitudes and the matrix-core colour sum') + \
        '#include "sigmakin_impl.h"\n\nnamespace mg {\n' + f'#include "{name}.inc"\n\n' + mt
    if hpl:
        src += f'''
struct P_{name}_hpl : P_{name} {{
  template <typename T, bool UNI = false, bool BEAM = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<float>& c, cx<float> (&J)[NCOL]) {{
    gen_{name}::jamps<float, UNI, BEAM>(p, h, c, J);
  }}
}};
'''
    for cs, tag in (('ColourMfmaF32', 'f32'), ('ColourMfmaBf16', 'bf16')):
        call = (f'sigmakin_mixed_hpl_launch<P_{name}, P_{name}_hpl, {cs}>' if hpl
                else f'sigmakin_mixed_launch<P_{name}, {cs}>')
        src += (f'\nint launch_sigmakin_{name}_mfma_{tag}(const MeArgs& a, const double* mom, int64_t nevt,\n'
                f'    double* me, const double* wgt, double* evtw, hipStream_t s) {{\n'
                f'  return {call}(a, mom, nevt, me, wgt, evtw, s);\n}}\n')
    units[f'sigmakin_{name}_mixed.hip'] = src + '\n}  // namespace mg\n'
    if name in GRAD_PROCESSES:
        nf = len(PROCESSES[name]) - 2
        src = (f'// Generated for {name}: do not edit.  Gradient kernels of adjoint_impl.h for\n'
               f'// this process (adjoint_a64: FP64, adjoint_a32: FP32 amplitudes).\n'
               '#include "adjoint_impl.h"\n\nnamespace mg {\n' + f'#include "{name}.inc"\n')
        for prec, T in (('a64', 'double'), ('a32', 'float')):
            src += f'''
struct {prec.upper()}_{name} {{
  static constexpr int SLOTS = gen_{name}::ADJ_SLOTS_{prec};
  template <bool BEAM, class WS>
  __device__ static __forceinline__ double adjoint(double (&p)[gen_{name}::NPAR][4], unsigned h,
                                                   const Couplings<{T}>& c,
                                                   double (&pb)[gen_{name}::NPAR][4], const WS& ws) {{
    return gen_{name}::adjoint_{prec}<BEAM>(p, h, c, pb, ws);
  }}
}};
'''
        src += f'''
int launch_grad_{name}(int prec, const MeArgs& a, const RamboArgs& ra, const double* rnd,
    int64_t nevt, const double* gbar, double* grad_rnd, double* grad_logw, double* mew,
    hipStream_t s) {{
  if (prec == 0)
    return adjoint_launch<A64_{name}, {nf}, double>(a, ra, a.c64, rnd, nevt, gbar, grad_rnd,
                                                   grad_logw, mew, s);
  return adjoint_launch<A32_{name}, {nf}, float>(a, ra, a.c32, rnd, nevt, gbar, grad_rnd,
                                                grad_logw, mew, s);
}}

}}  // namespace mg
'''
        units[f'grad_{name}.hip'] = src
    return units


def _write_if_changed(path, src):
    old = open(path).read() if os.path.exists(path) else None
    if old != src:
        with open(path, 'w') as f:
            f.write(src)


def write_all(outdir):
    os.makedirs(outdir, exist_ok=True)
    metas = {}
    names = ('eemumu', 'ggtt', 'ggttg', 'ggttgg')
    orders = optimised_orders(names)
    for name in names:
        src, meta = generate(name, orders)
        _write_if_changed(os.path.join(outdir, f"{name}.inc"), src)
        for fname, usrc in emit_units(name).items():
            _write_if_changed(os.path.join(outdir, fname), usrc)
        metas[name] = meta
    with open(os.path.join(outdir, 'meta.json'), 'w') as f:
        json.dump(metas, f, indent=1, sort_keys=True)
    return metas


if __name__ == '__main__':
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, '..', 'csrc', 'generated')
    print(json.dumps(write_all(out), indent=1))
