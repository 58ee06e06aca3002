"""Build the gfx950 shared library libmg5mi.so in-tree.

Steps: run the diagram generator (gen/) to emit csrc/generated/*.inc, compile
every csrc/*.hip with hipcc for gfx950, link one shared library next to this
file.  Usage: python -m paper_2106_12631_amd.build [--force]
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

# Flags of single sources.  The helicity-per-lane mixed kernel calls its
# matrix-core colour sum out of line; with the MFMA results in VGPRs and the
# callee's saved registers on the stack instead of in AGPRs it needs no AGPRs
# and runs two waves per SIMD.
SOURCE_FLAGS = {
    'sigmakin_ggttgg_mixed.hip': ['-mllvm', '-amdgpu-mfma-vgpr-form',
                                  '-mllvm', '-amdgpu-spill-vgpr-to-agpr=0'],
}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith('.hip'))


def build(force=True, verbose=True, extra_flags=(), output=None):
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2106_12631_amd.gen import emit
    emit.write_all(os.path.join(CSRC, 'generated'))
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    t0 = time.time()
    for src in sources():
        obj = os.path.join(BUILD, src.replace('.hip', '.o'))
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, ()), *extra_flags, '-c',
               os.path.join(CSRC, src), '-o', obj]
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
    if verbose:
        print(f"[build] {lib} in {time.time() - t0:.1f}s", file=sys.stderr)
    return lib


if __name__ == '__main__':
    build()
