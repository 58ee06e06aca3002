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

from .diagrams import BOSON_MASS, FERMION_MASS, FFV, ProcessDiagrams, colour_matrix, IN

IDEN = {'eemumu': 4, 'ggtt': 256, 'ggttg': 256, 'ggttgg': 512}

# algorithmic flops of each device routine (counted from helas.h)
FLOPS = {
    'vec_in': 22, 'vec_out': 22, 'ubar': 30, 'u': 30, 'v': 30, 'vbar': 30,
    'ffv_amp': 118, 'ffv_cur_v0': 104, 'ffv_cur_vm': 140,
    'ffv_cur_fin': 171, 'ffv_cur_fout': 171,
    'vvv_cur': 187, 'vvvv_cur': 128,
    'jamp_acc': 2,
}


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


def generate(name):
    pd = ProcessDiagrams(name)
    parts = pd.particles
    npar = pd.npar
    basis = pd.colour_basis() if pd.gluons else [()]
    ncol = len(basis)
    if pd.gluons:
        cnum, cden = colour_matrix(basis, len(pd.gluons))
    else:
        cnum, cden = [[1]], 1
    coefs = pd.jamp_coefficients()
    flops = 0
    L = []
    w = L.append
    w(f"// Generated for {name}: do not edit.  {pd.ndiagrams} diagrams, "
      f"{len(pd.diagrams)} amplitude calls, {len(pd.used) - npar} currents.")
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
    w("")
    w("template <typename T>")
    w(f"__device__ __forceinline__ void jamps(const double (&p)[{npar}][4], unsigned hcode,")
    w(f"                                      const Couplings<T>& c, cx<T> (&J)[{ncol}]) {{")
    for k in range(ncol):
        w(f"  J[{k}] = cx<T>{{(T)0, (T)0}};")
    names = {}
    emitted = set()

    def hel(l):
        return f"((hcode >> {npar - 1 - l}) & 1u) ? 1 : -1"

    def emit_node(n):
        nonlocal flops
        if n.idx in emitted:
            return
        op = n.op
        for ch in op[1:]:
            if hasattr(ch, 'idx'):
                emit_node(ch)
        v = f"w{n.idx}"
        names[n.idx] = v
        emitted.add(n.idx)
        if op[0] == 'ext':
            l, routine = op[1], op[2]
            p = f"p[{l}]"
            if routine == 'vec_in':
                w(f"  cx<T> {v}[4]; ext_vector<T>({p}, {hel(l)}, false, {v});")
            elif routine == 'vec_out':
                w(f"  cx<T> {v}[4]; ext_vector<T>({p}, {hel(l)}, true, {v});")
            else:
                mass = {'t': 'c.mt'}.get(n.flav, '0.0')
                fn = {'ubar': ('ext_u', 'true'), 'u': ('ext_u', 'false'),
                      'v': ('ext_v', 'false'), 'vbar': ('ext_v', 'true')}[routine]
                w(f"  cx<T> {v}[4]; {fn[0]}<T>({p}, {mass}, {hel(l)}, {fn[1]}, {v});")
            flops += FLOPS[routine]
            return
        K = _ksum(n.legs, parts)
        if op[0] == 'vvv':
            a, b = op[1], op[2]
            w(f"  cx<T> {v}[4]; {{ const double KA[4] = {_ksum(a.legs, parts)}; "
              f"const double KB[4] = {_ksum(b.legs, parts)}; "
              f"vvv_cur<T>({names[a.idx]}, KA, {names[b.idx]}, KB, c.gs, {v}); }}")
            flops += FLOPS['vvv_cur']
        elif op[0] == 'vvvv':
            s, x, y, z = op[1], op[2], op[3], op[4]
            w(f"  cx<T> {v}[4]; {{ const double K[4] = {K}; "
              f"vvvv_cur<{s}, T>({names[x.idx]}, {names[y.idx]}, {names[z.idx]}, K, c.gs2, {v}); }}")
            flops += FLOPS['vvvv_cur']
        elif op[0] == 'ffv_fout':
            f, vec = op[1], op[2]
            cl, cr = FFV[(f.flav, vec.flav)]
            m, wd = FERMION_MASS[f.flav]
            w(f"  cx<T> {v}[4]; {{ const double K[4] = {K}; "
              f"ffv_cur_fout<T>({names[f.idx]}, {names[vec.idx]}, c.{cl}, c.{cr}, K, c.{m}, c.{wd}, {v}); }}")
            flops += FLOPS['ffv_cur_fout']
        elif op[0] == 'ffv_fin':
            vec, f = op[1], op[2]
            cl, cr = FFV[(f.flav, vec.flav)]
            m, wd = FERMION_MASS[f.flav]
            w(f"  cx<T> {v}[4]; {{ const double K[4] = {K}; "
              f"ffv_cur_fin<T>({names[vec.idx]}, {names[f.idx]}, c.{cl}, c.{cr}, K, c.{m}, c.{wd}, {v}); }}")
            flops += FLOPS['ffv_cur_fin']
        elif op[0] == 'ffv_v':
            fo, fi, boson = op[1], op[2], op[3]
            cl, cr = FFV[(fo.flav, boson)]
            bm = BOSON_MASS[boson]
            if bm is None:
                w(f"  cx<T> {v}[4]; {{ const double K[4] = {K}; "
                  f"ffv_cur_v0<T>({names[fo.idx]}, {names[fi.idx]}, c.{cl}, c.{cr}, K, {v}); }}")
                flops += FLOPS['ffv_cur_v0']
            else:
                w(f"  cx<T> {v}[4]; {{ const double K[4] = {K}; "
                  f"ffv_cur_vm<T>({names[fo.idx]}, {names[fi.idx]}, c.{cl}, c.{cr}, K, c.{bm[0]}, c.{bm[1]}, {v}); }}")
                flops += FLOPS['ffv_cur_vm']
        else:
            raise ValueError(op)

    for d, cf in zip(pd.diagrams, coefs):
        for n in (d.fout, d.vec, d.fin):
            emit_node(n)
        cl, cr = FFV[(d.fin.flav, d.vec.flav)]
        w(f"  {{ const cx<T> a = ffv_amp<T>({names[d.fout.idx]}, {names[d.vec.idx]}, "
          f"{names[d.fin.idx]}, c.{cl}, c.{cr});")
        for k, coef in sorted(cf.items()):
            w(f"    J[{k}] = J[{k}] {_coef_expr(coef, 'a')};")
            flops += FLOPS['jamp_acc']
        w("  }")
        flops += FLOPS['ffv_amp']
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
    w(f"}}  // namespace gen_{name}")
    cs_flops += 1
    meta = {
        'process': name, 'npar': npar, 'ncol': ncol, 'ndiag': pd.ndiagrams,
        'namp': len(pd.diagrams), 'ncurrents': len(pd.used) - npar,
        'flops_amp_per_hel': flops, 'flops_colour_per_hel': cs_flops,
        'iden': IDEN[name], 'cden': cden,
    }
    return "\n".join(L) + "\n", meta


def write_all(outdir):
    os.makedirs(outdir, exist_ok=True)
    metas = {}
    for name in ('eemumu', 'ggtt', 'ggttg', 'ggttgg'):
        src, meta = generate(name)
        path = os.path.join(outdir, f"{name}.inc")
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, 'w') as f:
                f.write(src)
        metas[name] = meta
    with open(os.path.join(outdir, 'meta.json'), 'w') as f:
        json.dump(metas, f, indent=1, sort_keys=True)
    return metas


if __name__ == '__main__':
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, '..', 'csrc', 'generated')
    print(json.dumps(write_all(out), indent=1))
