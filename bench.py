#!/usr/bin/env python3
"""Throughput of the per-event |M|^2 path on one MI355X.

One step = one pass of the whole path over one batch of synthetic events:
random numbers + RAMBO (fused sampler kernel) and SIGMAKIN (helicity
amplitudes, colour-flow amplitudes, colour sum, helicity sum), for the
gg -> t t~ g g workload (2^19 events, seed 3, sqrt(s) = 1500 GeV).
The headline value is the FP64 path; the FP32-amplitude path is measured
beside it.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matrix elements/sec gg→tt̄gg on 1 GPU, FP64 vs mixed; % FP64/MFMA peak"
PAPER_V100_GGTTGG = 5.2e5      # MEs/s, FP64, 524,288 events per iteration (paper, context)
PEAK_FP64_VALU = 78.6e12       # FLOP/s, MI355X vector FP64 (256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz)
# FLOP/s, MI355X published vector FP32 peak.  The kernels are built without
# packed FP32 instructions, yet their counters show more than one FP32 VALU
# wave instruction per 4 cycles per SIMD, so the FP32 forms are priced
# against the published figure rather than the FP64 rate.
PEAK_FP32_VALU = 157.3e12


# ----------------------------------------------------------------------------- HBM traffic
def kernel_source_hash(proc):
    """sha256 over everything that defines the SIGMAKIN kernels of proc: the
    headers they use, the process's kernel sources, its generated code and
    the compiler flags.  HBM counters recorded under profiles/ are reported only
    while this hash matches the one they were taken with."""
    import hashlib
    sys.path.insert(0, os.path.join(ROOT, 'paper_2106_12631_amd'))
    from paper_2106_12631_amd import build as _build
    csrc = os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc')
    shared = ['colour_mfma.h', 'common.h', 'helas.h', 'internal.h', 'sigmakin_impl.h']
    names = shared + sorted(n for n in os.listdir(csrc)
                            if n.startswith(f'sigmakin_{proc}_') and n.endswith('.hip'))
    h = hashlib.sha256()
    for n in names + [os.path.join('generated', f'{proc}.inc')]:
        h.update(n.encode())
        with open(os.path.join(csrc, n), 'rb') as fh:
            h.update(fh.read())
    h.update(' '.join(a for a in _build.FLAGS if not a.startswith('/')).encode())
    for n in names:
        h.update(' '.join(_build.SOURCE_FLAGS.get(n, ())).encode())
    return h.hexdigest()[:16]


def recorded_traffic(proc, nevt):
    """{precision: HBM bytes per SIGMAKIN launch} from the ```traffic blocks
    of profiles/*.md whose source hash and event count match, else {}."""
    import glob
    import re
    want = kernel_source_hash(proc)
    for path in sorted(glob.glob(os.path.join(ROOT, 'profiles', '*.md'))):
        for blk in re.findall(r"```traffic\n(.*?)```", open(path).read(), re.S):
            rec = json.loads(blk)
            if rec.get('process') == proc and rec.get('nevt') == nevt and \
                    rec.get('source_hash') == want:
                return {k: v['hbm_bytes_per_launch'] for k, v in rec['kernels'].items()}
    return {}


# ----------------------------------------------------------------------------- CPU baseline
def _oracle_chunk(task):
    proc, seed, start, count = task
    import torch
    torch.set_num_threads(1)
    from oracle import me as orc
    t0 = time.perf_counter()
    _, p, _ = orc.sample(proc, seed, start, count)
    orc.matrix_element(proc, p, chunk=64)
    return count, time.perf_counter() - t0


def cpu_baseline(proc, seed, per_worker, workers):
    """Oracle (as it stands) on a bounded sample, one process per core."""
    import multiprocessing as mp
    tasks = [(proc, seed, w * per_worker, per_worker) for w in range(workers)]
    ctx = mp.get_context('fork')
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_chunk, tasks)
    wall = time.perf_counter() - t0
    n = sum(c for c, _ in res)
    per_core = sum(c / t for c, t in res) / len(res)
    cpu_model = ''
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                cpu_model = line.split(':', 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / wall, "unit": "MEs/s", "cores": workers, "kind": "oracle",
            "single_core_value": per_core, "cpu": cpu_model,
            "sample": f"events 0..{n - 1} of the workload (seed {seed}): RNG + RAMBO + |M|^2, "
                      f"{workers} processes x 1 thread, {wall:.1f} s wall"}


# ----------------------------------------------------------------------------- GPU
def _median(x):
    x = sorted(x)
    n = len(x)
    return 0.5 * (x[(n - 1) // 2] + x[n // 2])


def run_gpu(mg, torch, proc, prec, seed, nevt, steps, warmup):
    """Warm-up, then `steps` timed steps (sampler + SIGMAKIN) between two
    device synchronisations; HIP events on the launching stream split each
    step into its kernels.  Afterwards the same number of steps with the
    matrix elements copied to pinned host memory gives the paper's third
    timing scope (compute + device-to-host)."""
    eng = mg.MEEngine(proc, prec)
    dev = eng.device
    mom = eng.empty_mom(nevt)
    wgt = torch.empty(nevt, dtype=torch.float64, device=dev)
    me = torch.empty(nevt, dtype=torch.float64, device=dev)
    host = torch.empty(nevt, dtype=torch.float64, pin_memory=True)

    for _ in range(warmup):
        eng.sample(seed, nevt, mom=mom, wgt=wgt)
        eng.sigmakin(mom, nevt, me=me)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def ev():
        return torch.cuda.Event(enable_timing=True)
    evs = [(ev(), ev(), ev()) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        eng.sample(seed, nevt, mom=mom, wgt=wgt)
        evs[k][1].record(stream)
        eng.sigmakin(mom, nevt, me=me)
        evs[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms = [b.elapsed_time(c) for a, b, c in evs]
    step_ms = [a.elapsed_time(c) for a, b, c in evs]
    nonfinite = eng.count_nonfinite(me)
    evd = [(ev(), ev()) for _ in range(steps)]
    for k in range(steps):
        evd[k][0].record(stream)
        eng.sample(seed, nevt, mom=mom, wgt=wgt)
        eng.sigmakin(mom, nevt, me=me)
        host.copy_(me, non_blocking=True)
        evd[k][1].record(stream)
    torch.cuda.synchronize()
    d2h_ms = [a.elapsed_time(b) for a, b in evd]
    scopes = {
        "sigmakin": nevt / (_median(k_ms) / 1e3),
        "sample_sigmakin": nevt / (_median(step_ms) / 1e3),
        "sample_sigmakin_dtoh": nevt / (_median(d2h_ms) / 1e3),
        "unit": "MEs/s (median over the timed steps)",
    }
    return eng, wall, k_ms, nonfinite, scopes


PEAK_MFMA = {'bf16': 2.5e15, 'f32': 157.3e12}  # dense FLOP/s, MI355X


def mfma_work(ncol, nhel, prec, proc, seconds, nevt):
    """Matrix-core work of the colour sum as executed: per 64 columns (64
    events of one helicity, or the 64 helicities of one event), 2 parts x
    K blocks x 2 tiles of 32x32 outputs."""
    bf16 = prec == 'mixed' and proc == 'ggttgg'
    if bf16:
        kb, k = (3 * ((ncol + 7) // 8) + 1) // 2, 16
    else:
        kb, k = (ncol + 1) // 2, 2
    flops_evt = 2 * kb * 2 * (32 * 32 * k * 2) / 64 * nhel
    achieved = flops_evt * nevt / seconds
    peak = PEAK_MFMA['bf16' if bf16 else 'f32']
    return {"dtype": "bf16" if bf16 else "f32", "flops_per_event": flops_evt,
            "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak}


def run_gradient(mg, torch, prec, nevt, steps, warmup, seed=4):
    """Gradient workload: d(w |M|^2)/dr and d log w/dr for g g -> t t~ g,
    timed beside the forward pass (RAMBO + SIGMAKIN) on the same uniforms."""
    eng = mg.MEEngine('ggttg', prec)
    rnd = eng.rng(seed, nevt)
    mom = eng.empty_mom(nevt)
    wgt = torch.empty(nevt, dtype=torch.float64, device=eng.device)
    me = torch.empty(nevt, dtype=torch.float64, device=eng.device)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    out = {}

    def grad():
        out['g'] = eng.adjoint(rnd, nevt)

    def fwd():
        eng.rambo(rnd, nevt, mom=mom, wgt=wgt)
        eng.sigmakin(mom, nevt, me=me)

    t_grad = timed(grad)
    t_fwd = timed(fwd)
    return {"events_per_s": nevt / t_grad, "ms_per_launch": t_grad * 1e3,
            "forward_ms": t_fwd * 1e3, "gradient_over_forward": t_grad / t_fwd,
            "nonfinite": eng.count_nonfinite(out['g'][0])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=12)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--process', default='ggttgg')
    ap.add_argument('--nevt', type=int, default=1 << 19)
    ap.add_argument('--seed', type=int, default=3)
    ap.add_argument('--precisions', default='fp64,mixed,fp32amp')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-events-per-worker', type=int, default=96)
    ap.add_argument('--no-gradient', action='store_true',
                    help='skip the gradient workload (g g -> t t~ g, 2^18 events)')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='only run a plain 1 GiB device-to-device copy (HBM counter calibration)')
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 27
        src = torch.ones(n, dtype=torch.float64, device='cuda')
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(events are independent: they would shard as one contiguous event range "
              f"per GPU)", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(args.process, args.seed, args.cpu_events_per_worker, workers)

    import torch
    import paper_2106_12631_amd as mg
    meta = json.load(open(os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc', 'generated',
                                       'meta.json')))[args.process]
    traffic = recorded_traffic(args.process, args.nevt)
    results = {}
    for prec in args.precisions.split(','):
        eng, wall, k_ms, nonfinite, scopes = run_gpu(mg, torch, args.process, prec, args.seed,
                                                     args.nevt, args.steps, args.warmup)
        nhel = eng.layout.nhel_good
        flops_evt = (meta['flops_amp_per_hel'] + meta['flops_colour_per_hel']) * nhel
        k_avg = sum(k_ms) / len(k_ms) / 1e3
        achieved = flops_evt * args.nevt / k_avg
        peak = PEAK_FP64_VALU if prec == 'fp64' else PEAK_FP32_VALU
        results[prec] = {
            "value": args.nevt * args.steps / wall,
            "ms_per_step": wall / args.steps * 1e3,
            "sigmakin_ms": k_avg * 1e3,
            "sigmakin_MEs_per_s": args.nevt / k_avg,
            "nonfinite": nonfinite,
            "scopes": scopes,
            "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                         "peak": peak / 1e12, "unit": "TFLOP/s",
                         "frac": achieved / peak, "traffic": traffic.get(prec),
                         "flops_per_event": flops_evt},
        }
        if prec.startswith('mixed'):
            results[prec]["mfma"] = mfma_work(meta['ncol'], nhel, prec, args.process, k_avg,
                                              args.nevt)
    gradient = None
    if not args.no_gradient:
        gradient = {"workload": "ggttg 262144 events seed 4: d(w |M|^2)/dr, d log w/dr "
                                "(12 uniforms per event)"}
        for prec in ('fp64', 'fp32amp'):
            gradient[prec] = run_gradient(mg, torch, prec, 1 << 18, max(1, args.steps // 2), 1)
    head = results.get('fp64') or next(iter(results.values()))
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "MEs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": head["value"] / PAPER_V100_GGTTGG if args.process == 'ggttgg' else None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.process} {args.nevt} events seed {args.seed} "
                               f"sqrt(s)=1500 GeV (Philox + RAMBO + |M|^2)",
                   "process": args.process, "nevt": args.nevt, "seed": args.seed,
                   "parallelism": "1 GPU, one event per wave, one helicity per lane"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "variants": results,
        "gradient": gradient,
    }
    print(json.dumps(line), flush=True)


if __name__ == '__main__':
    main()
