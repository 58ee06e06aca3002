"""Build the gfx950 shared library libmg5mi.so in-tree.

Steps: run the diagram generator (gen/) to emit csrc/generated/ (the
amplitude code *.inc and the per-process kernel units *.hip), compile every
csrc/*.hip and csrc/generated/*.hip with hipcc for gfx950, link one shared library next to this
file; then build the calibration kernels (calib/) as libmg5cal.so.

    python -m paper_2106_12631_amd.build               build both libraries
    python -m paper_2106_12631_amd.build --resources   print the compiler's
        register, scratch, LDS and occupancy report of every kernel
    python -m paper_2106_12631_amd.build --no-recompute OUT
        a measurement library at OUT whose amplitude code recomputes nothing
        (its executed flops are the algorithmic flops)
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(HERE, '_build')
LIB = os.path.join(HERE, 'libmg5mi.so')
INCLUDE = os.path.join(os.path.dirname(HERE), 'include')
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')

FLAGS = [
    '--offload-arch=gfx950', '-O3', '-std=c++17', '-fPIC',
    # packed FP32 instructions are kept out of every kernel
    '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
    '-ffp-contract=fast',
    '-I', CSRC, '-I', INCLUDE,
]

# Flags of single sources.  The helicity-per-lane mixed kernel runs its
# matrix-core colour sum after the FP32 amplitudes; with the MFMA results in
# VGPRs and no VGPR spills to AGPRs it needs no AGPRs and keeps two waves per
# SIMD.
SOURCE_FLAGS = {
    'sigmakin_ggttgg_mixed.hip': ['-mllvm', '-amdgpu-mfma-vgpr-form',
                                  '-mllvm', '-amdgpu-spill-vgpr-to-agpr=0'],
}

# Flags of the generated per-process units.  Products with components that
# are zero at compile time (the time component of a massless external
# vector, the transverse components of the beams in the beam bodies) fold
# away only when the compiler may disregard signed zeros, infinities and
# NaNs; the results change at most in the sign of a zero.  These units test
# no value for being finite: the kernels that do (count_nonfinite_kernel,
# the cross-section and unweighting kernels) are built without the flags.
GENERATED_FLAGS = ['-fno-signed-zeros', '-ffinite-math-only']


def source_flags(src):
    """Flags of one unit beyond FLAGS (src relative to csrc/)."""
    extra = list(SOURCE_FLAGS.get(os.path.basename(src), ()))
    if os.path.dirname(src) == 'generated':
        extra += GENERATED_FLAGS
    return extra


def sources(csrc=CSRC):
    """Hand-written units of csrc/ and the per-process units the generator
    writes to csrc/generated/ (file names are unique across the two)."""
    gen = os.path.join(csrc, 'generated')
    units = [f for f in os.listdir(csrc) if f.endswith('.hip')]
    if os.path.isdir(gen):
        units += [os.path.join('generated', f) for f in os.listdir(gen) if f.endswith('.hip')]
    return sorted(units)


def build(force=True, verbose=True, extra_flags=(), output=None, csrc=CSRC, objdir=BUILD):
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2106_12631_amd.gen import emit
    emit.write_all(os.path.join(csrc, 'generated'))
    os.makedirs(objdir, exist_ok=True)
    flags = [csrc if f == CSRC else f for f in FLAGS]
    procs = []
    objs = []
    t0 = time.time()
    for src in sources(csrc):
        obj = os.path.join(objdir, os.path.basename(src).replace('.hip', '.o'))
        objs.append(obj)
        cmd = [HIPCC, *flags, *source_flags(src), *extra_flags, '-c',
               os.path.join(csrc, src), '-o', obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors='replace')
        # the host pass does not know the gfx950 target feature: harmless
        lines = [l for l in text.splitlines() if 'packed-fp32-ops' not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            print(f"[build] {src} FAILED\n" + "\n".join(lines[-60:]), file=sys.stderr)
        elif verbose and lines:
            keep = lines if extra_flags else lines[-20:]
            print(f"[build] {src}:\n" + "\n".join(keep), file=sys.stderr)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    lib = output or LIB
    tmp = lib + '.tmp'
    subprocess.check_call([HIPCC, '--offload-arch=gfx950', '-shared', '-fPIC', '-o', tmp, *objs])
    os.replace(tmp, lib)
    if output is None:
        # the calibration kernels (arithmetic peaks), a library of their own
        cal = os.path.join(HERE, 'libmg5cal.so')
        subprocess.check_call([HIPCC, *FLAGS, '-shared', '-o', cal + '.tmp',
                               os.path.join(HERE, 'calib', 'calibrate.hip')],
                              stderr=subprocess.DEVNULL)
        os.replace(cal + '.tmp', cal)
    if verbose:
        print(f"[build] {lib} in {time.time() - t0:.1f}s", file=sys.stderr)
    return lib


# Live-wavefunction budget of the measurement build below: above every
# process's peak (32 for g g -> t t~ g g), so nothing is recomputed.
NO_RECOMPUTE_BUDGET = 1 << 20


def build_without_recomputation(output):
    """A library whose generated amplitude code computes every wavefunction
    once and keeps it until its last use, whatever the register spills: the
    executed flops of its SIGMAKIN kernels (rocprofv3 VALU flop counters) are
    the algorithmic flops of the amplitude code as compiled, after the
    folding of the beam and zero components.  Built from a temporary copy of
    csrc/; the working tree's generated code and library are left as they
    are.  Only the amplitude bodies change (the gradient kernels keep their
    budgets)."""
    import shutil
    import tempfile
    tmp = tempfile.mkdtemp(prefix='mg5mi_norecompute_')
    keys = ('MG_BUDGET_F64', 'MG_BUDGET_F32', 'MG_BUDGET_F32M')
    saved = {k: os.environ.get(k) for k in keys}
    try:
        csrc = os.path.join(tmp, 'csrc')
        shutil.copytree(CSRC, csrc, ignore=shutil.ignore_patterns('generated'))
        for k in keys:
            os.environ[k] = str(NO_RECOMPUTE_BUDGET)
        return build(output=os.path.abspath(output), csrc=csrc, objdir=os.path.join(tmp, 'obj'))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        shutil.rmtree(tmp, ignore_errors=True)


def resource_report():
    """Markdown table of every kernel's registers, scratch, LDS and
    occupancy as the compiler reports them for gfx950
    (-Rpass-analysis=kernel-resource-usage), one row per kernel."""
    import re
    rows = []
    for src in sources():
        cmd = [HIPCC, *FLAGS, *source_flags(src),
               '-Rpass-analysis=kernel-resource-usage', '-c', os.path.join(CSRC, src), '-o',
               os.devnull]
        out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                             text=True).stdout
        cur = None
        for line in out.splitlines():
            m = re.search(r'remark:\s+(Function Name|TotalSGPRs|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|'
                          r'Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s*(\S+)', line)
            if not m:
                continue
            key, val = m.group(1).split(' [')[0], m.group(2)
            if key == 'Function Name':
                cur = {'source': os.path.basename(src), 'kernel': val}
                rows.append(cur)
            elif cur is not None:
                cur[key] = val
    demangled = subprocess.run(['c++filt'], input='\n'.join(r['kernel'] for r in rows),
                               stdout=subprocess.PIPE, text=True).stdout.splitlines()
    lines = ['| source | kernel | VGPRs | AGPRs | SGPRs | scratch B/lane | LDS B/block | waves/SIMD |',
             '|---|---|---|---|---|---|---|---|']
    for r, d in zip(rows, demangled):
        name = re.sub(r'\(.*$', '', d).replace('mg::', '')
        lines.append(f"| {r['source']} | `{name}` | {r.get('VGPRs')} | {r.get('AGPRs')} | "
                     f"{r.get('TotalSGPRs')} | {r.get('ScratchSize')} | {r.get('LDS Size')} | "
                     f"{r.get('Occupancy')} |")
    return '\n'.join(lines)


if __name__ == '__main__':
    if '--resources' in sys.argv:
        print(resource_report())
    elif '--no-recompute' in sys.argv:
        build_without_recomputation(sys.argv[sys.argv.index('--no-recompute') + 1])
    else:
        build()
