#!/usr/bin/env python3
"""Throughput of the per-event |M|^2 path on one MI355X.

One step = one pass of the whole path over one batch of synthetic events:
random numbers + RAMBO (fused sampler kernel) and SIGMAKIN (helicity
amplitudes, colour-flow amplitudes, colour sum, helicity sum).  The headline
is the gg -> t t~ g g workload (2^19 events, seed 3, sqrt(s) = 1500 GeV) in
FP64; every benchmark workload is measured beside it (`variants`):

  e+e- -> mu+mu-  16384 events, seed 0     FP64
  g g -> t t~     2^20 events, seed 1      FP64, FP32 amplitudes
  g g -> t t~ g   2^20 events, seed 2      mixed (FP32 MFMA colour sum), FP64
  g g -> t t~ g g 2^19 events, seed 3      FP64, mixed (BF16-split MFMA), FP32 amplitudes
  gradient        g g -> t t~ g, 2^18 events, seed 4: d(w |M|^2)/dr, FP64 and FP32 amplitudes
  plateau         e+e- -> mu+mu-, 2^24 events, seed 0, FP64 (throughput plateau)

Three timing scopes per variant (medians over the timed steps, as the
paper's 12 iterations): SIGMAKIN only, sampler + SIGMAKIN, and + the copy of
the matrix elements to pinned host memory.  The oracle is timed per
workload on the host's cores (1 core and P cores, each for a bounded time,
worker start-up and imports excluded), and the GPU results of the same
events are compared with the oracle's (end to end from the uniforms, and on
the oracle's momenta).  Prints one JSON line.
"""
import argparse
import json
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
PEAK_MFMA = {'bf16': 2.5e15, 'f32': 157.3e12}  # dense FLOP/s, MI355X

# (name, process, events, seed, precisions); the first precision of the
# headline workload is the headline value
WORKLOADS = [
    ('eemumu', 'eemumu', 16384, 0, ('fp64',)),
    ('ggtt', 'ggtt', 1 << 20, 1, ('fp64', 'fp32amp')),
    ('ggttg', 'ggttg', 1 << 20, 2, ('mixed', 'fp64')),
    ('ggttgg', 'ggttgg', 1 << 19, 3, ('fp64', 'mixed', 'fp32amp')),
]
HEADLINE = 'ggttgg'
GRADIENT = ('ggttg', 1 << 18, 4, ('fp64', 'fp32amp'))
PLATEAU = ('eemumu', 1 << 24, 0, 'fp64')


# ----------------------------------------------------------------------------- HBM traffic
def kernel_source_hash(proc):
    """sha256 over everything that defines the SIGMAKIN kernels of proc: the
    headers they use, the process's kernel sources, its generated code and
    the compiler flags.  HBM counters recorded under profiles/ are reported only
    while this hash matches the one they were taken with."""
    import hashlib
    from paper_2106_12631_amd import build as _build
    csrc = os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc')
    shared = ['colour_mfma.h', 'common.h', 'helas.h', 'internal.h', 'sigmakin_impl.h']
    gen = os.path.join(csrc, 'generated')
    units = sorted(os.path.join('generated', n) for n in os.listdir(gen)
                   if n.startswith(f'sigmakin_{proc}_') and n.endswith('.hip'))
    names = shared + units
    h = hashlib.sha256()
    for n in names + [os.path.join('generated', f'{proc}.inc')]:
        h.update(n.encode())
        with open(os.path.join(csrc, n), 'rb') as fh:
            h.update(fh.read())
    h.update(' '.join(a for a in _build.FLAGS if not a.startswith('/')).encode())
    for n in names:
        h.update(' '.join(_build.source_flags(n)).encode())
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


def recorded_flops(proc, nhel):
    """Algorithmic flops per event of proc's SIGMAKIN code from the ```flops
    block of profiles/*.md: the executed VALU flops of the FP64 kernel of a
    build whose amplitude code recomputes nothing
    (`python -m paper_2106_12631_amd.build --no-recompute`), i.e. the work of
    the amplitude code as compiled, after the products with the beams' and
    the massless vectors' zero components have folded away.  None when no
    record matches the current sources."""
    import glob
    import re
    want = kernel_source_hash(proc)
    for path in sorted(glob.glob(os.path.join(ROOT, 'profiles', '*.md'))):
        for blk in re.findall(r"```flops\n(.*?)```", open(path).read(), re.S):
            rec = json.loads(blk).get(proc)
            if rec and rec.get('source_hash') == want and rec.get('nhel') == nhel:
                return rec['flops_per_event']
    return None


# ----------------------------------------------------------------------------- CPU baseline
def _oracle_eval(kind, proc, seed, start, count):
    """The oracle on events [start, start + count): RNG + RAMBO + |M|^2
    (kind 'me'), or f = w |M|^2 and its gradient by autograd (kind 'grad').
    Returns arrays to compare the GPU with."""
    from oracle import me as orc
    if kind == 'me':
        _, p, _ = orc.sample(proc, seed, start, count)
        me = orc.matrix_element(proc, p, chunk=64)
        return {'me': me.numpy(), 'p': p.numpy()}
    r, _, _ = orc.sample(proc, seed, start, count)
    f, g, _ = orc.event_weight_and_grad(proc, r)
    return {'f': f.numpy(), 'grad': g.numpy()}


def _oracle_worker(kind, proc, seed, start, tmin, barrier, queue):
    import numpy as np
    import torch
    torch.set_num_threads(1)
    _oracle_eval(kind, proc, seed, start, 1)  # imports and first-call set-up, not timed
    barrier.wait()
    t0 = time.perf_counter()
    n, chunk, parts = 0, 1, []
    while True:
        parts.append(_oracle_eval(kind, proc, seed, start + n, chunk))
        n += chunk
        el = time.perf_counter() - t0
        if el >= tmin:
            break
        # aim the remaining chunks at the time limit
        chunk = max(1, min(4 * chunk, int(n / el * (tmin - el)) + 1, 4096))
    t1 = time.perf_counter()
    out = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    queue.put((start, n, t0, t1, out))


def oracle_timing(kind, proc, seed, workers, tmin, stride):
    """The oracle on `workers` host cores, one process and one thread each,
    every worker for at least tmin seconds on its own event range (worker w
    from event w * stride).  Start-up and imports happen before a barrier;
    the wall time runs from the first worker's start to the last one's
    end.  Returns (events per second, events, wall, per-worker results)."""
    import multiprocessing as mp
    ctx = mp.get_context('fork')
    barrier = ctx.Barrier(workers)
    queue = ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker,
                         args=(kind, proc, seed, w * stride, tmin, barrier, queue))
             for w in range(workers)]
    for p in procs:
        p.start()
    res = [queue.get() for _ in procs]
    for p in procs:
        p.join()
    n = sum(r[1] for r in res)
    wall = max(r[3] for r in res) - min(r[2] for r in res)
    return n / wall, n, wall, res


def host_cores():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_model():
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return ''


def cpu_baselines(tmin, workers):
    """Oracle rates per workload on 1 core and on `workers` cores, and the
    oracle's results on the events it timed (for the GPU comparison)."""
    out = {}
    jobs = [(name, 'me', proc, nevt, seed) for name, proc, nevt, seed, _ in WORKLOADS]
    jobs.append(('gradient', 'grad', GRADIENT[0], GRADIENT[1], GRADIENT[2]))
    for name, kind, proc, nevt, seed in jobs:
        r1, n1, w1, res1 = oracle_timing(kind, proc, seed, 1, tmin, 0)
        stride = max(1, nevt // workers)
        rp, npar, wp, resp = oracle_timing(kind, proc, seed, workers, tmin, stride)
        out[name] = {
            "single_core": {"value": r1, "events": n1, "seconds": w1},
            "all_cores": {"value": rp, "events": npar, "seconds": wp, "cores": workers},
            "results": [(s, n, o) for s, n, _, _, o in res1 + resp],
        }
        print(f"[bench] oracle {name}: {r1:.4g} /s on 1 core, {rp:.4g} /s on {workers} cores",
              file=sys.stderr, flush=True)
    return out


# ----------------------------------------------------------------------------- GPU
def _median(x):
    x = sorted(x)
    n = len(x)
    return 0.5 * (x[(n - 1) // 2] + x[n // 2])


def run_gpu(mg, torch, proc, prec, seed, nevt, steps, warmup):
    """Warm-up, then `steps` timed steps (sampler + SIGMAKIN) between two
    device synchronisations; HIP events on the launching stream (torch's
    current stream, on which the binding enqueues every call) split each
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
    try:
        graph = graph_step(eng, torch, seed, nevt, mom, wgt, me, steps)
    except RuntimeError as e:  # the line does not depend on graph capture
        torch.cuda.synchronize()
        graph = {"step_ms": None, "wall_MEs_per_s": None, "replays_equal_eager": None,
                 "error": str(e)[:200]}
    scopes = {
        "sigmakin": nevt / (_median(k_ms) / 1e3),
        "sample_sigmakin": nevt / (_median(step_ms) / 1e3),
        "sample_sigmakin_dtoh": nevt / (_median(d2h_ms) / 1e3),
        "unit": "MEs/s (median over the timed steps)",
    }
    if graph["step_ms"]:
        scopes["sample_sigmakin_graph"] = nevt / (_median(graph["step_ms"]) / 1e3)
    return eng, wall, k_ms, nonfinite, scopes, me, graph


def graph_step(eng, torch, seed, nevt, mom, wgt, me, steps):
    """The step (sampler + SIGMAKIN) captured once in a HIP graph and
    replayed: one graph launch per step instead of two library calls, for
    the launch-bound workloads.  The library's calls only enqueue kernels on
    the caller's stream (no allocation, no synchronisation), so they capture
    as they are.  Every checked replay must reproduce the eager step's
    matrix elements bit for bit (eager work and synchronisations between
    them).  Returns the per-step HIP-event times and the wall-clock rate of
    back-to-back replays."""
    ref = me.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        eng.sample(seed, nevt, mom=mom, wgt=wgt)
        eng.sigmakin(mom, nevt, me=me)
    stream = torch.cuda.current_stream()
    same = True
    for _ in range(3):
        me.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same = same and bool(torch.equal(me, ref))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        g.replay()
        b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    same = same and bool(torch.equal(me, ref))
    return {"step_ms": [a.elapsed_time(b) for a, b in evs], "wall_MEs_per_s": nevt * steps / wall,
            "replays_equal_eager": same}


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


def _errors(err, n_above=1e-12):
    import numpy as np
    err = np.asarray(err)
    if err.size == 0:
        return None
    return {"max": float(err.max()), "median": float(np.median(err)),
            "above_1e-12": int((err > n_above).sum()), "events": int(err.size)}


def parity_vs_oracle(eng, torch, me_gpu, nevt, orc_res):
    """GPU against the oracle on the events the oracle timed (indices below
    nevt): end to end (the GPU's own sampled events, same seed and index)
    and on the oracle's momenta."""
    import numpy as np
    idx, me_o, p_o = [], [], []
    for start, n, o in orc_res:
        k = max(0, min(n, nevt - start))
        idx.extend(range(start, start + k))
        me_o.append(o['me'][:k])
        p_o.append(o['p'][:k])
    if not idx:
        return None
    me_o = np.concatenate(me_o)
    p_o = torch.from_numpy(np.concatenate(p_o))
    got = me_gpu[torch.tensor(idx, device=me_gpu.device)].cpu().numpy()
    e2e = np.abs(got - me_o) / np.abs(me_o)
    same = eng.sigmakin(eng.events_mom(p_o), len(idx)).cpu().numpy()
    err_same = np.abs(same - me_o) / np.abs(me_o)
    return {"end_to_end": _errors(e2e), "same_momenta": _errors(err_same)}


def run_gradient(mg, torch, prec, nevt, seed, steps, warmup, orc_res):
    """Gradient workload: d(w |M|^2)/dr and d log w/dr for g g -> t t~ g,
    timed beside the forward pass (RAMBO + SIGMAKIN) on the same uniforms;
    the gradients of the oracle's events compared normwise."""
    import numpy as np
    eng = mg.MEEngine(GRADIENT[0], prec)
    rnd = eng.rng(seed, nevt)
    mom = eng.empty_mom(nevt)
    wgt = torch.empty(nevt, dtype=torch.float64, device=eng.device)
    me = torch.empty(nevt, dtype=torch.float64, device=eng.device)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return _median([a.elapsed_time(b) for a, b in evs]) / 1e3

    out = {}

    def grad():
        out['g'] = eng.adjoint(rnd, nevt)

    def fwd():
        eng.rambo(rnd, nevt, mom=mom, wgt=wgt)
        eng.sigmakin(mom, nevt, me=me)

    t_grad = timed(grad)
    t_fwd = timed(fwd)
    res = {"events_per_s": nevt / t_grad, "ms_per_launch": t_grad * 1e3,
           "forward_ms": t_fwd * 1e3, "gradient_over_forward": t_grad / t_fwd,
           "nonfinite": eng.count_nonfinite(out['g'][0])}
    if orc_res:
        g_all = eng.rnd_events(out['g'][0], nevt)
        errs = []
        for start, n, o in orc_res:
            k = max(0, min(n, nevt - start))
            if k:
                g = g_all[start:start + k].cpu().numpy()
                ref = o['grad'][:k]
                errs.append(np.linalg.norm(g - ref, axis=1) / np.linalg.norm(ref, axis=1))
        if errs:
            res["vs_oracle_normwise"] = _errors(np.concatenate(errs))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=12)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--only', default='',
                    help='comma-separated workload names to run (default: all)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-seconds', type=float, default=5.0,
                    help='minimum oracle time per workload, on 1 core and on all cores')
    ap.add_argument('--no-gradient', action='store_true')
    ap.add_argument('--no-plateau', action='store_true')
    ap.add_argument('--no-calibration', action='store_true',
                    help='skip the arithmetic-peak calibration kernels')
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
    only = set(filter(None, args.only.split(',')))
    workloads = [w for w in WORKLOADS if not only or w[0] in only]
    do_grad = not args.no_gradient and (not only or 'gradient' in only)
    do_plateau = not args.no_plateau and (not only or 'plateau' in only)

    # the oracle runs first, in forked worker processes, before this process
    # touches the GPU
    cores = host_cores()
    cpu = cpu_baselines(args.cpu_seconds, cores) if not args.no_cpu_baseline else {}

    import torch
    import paper_2106_12631_amd as mg
    metas = json.load(open(os.path.join(ROOT, 'paper_2106_12631_amd', 'csrc', 'generated',
                                        'meta.json')))
    calibration = None
    if not args.no_calibration:
        from paper_2106_12631_amd import calibrate
        print("[bench] calibration kernels", file=sys.stderr, flush=True)
        calibration = calibrate.run()
    variants = {}
    for name, proc, nevt, seed, precs in workloads:
        meta = metas[proc]
        traffic = recorded_traffic(proc, nevt)
        for prec in precs:
            print(f"[bench] {name} {prec} {nevt} events", file=sys.stderr, flush=True)
            eng, wall, k_ms, nonfinite, scopes, me, graph = run_gpu(mg, torch, proc, prec, seed,
                                                                    nevt, args.steps, args.warmup)
            nhel = eng.layout.nhel_good
            generic = (meta['flops_amp_per_hel'] + meta['flops_colour_per_hel']) * nhel
            flops_evt = recorded_flops(proc, nhel)
            source = "measured: executed flops of the no-recomputation build"
            if flops_evt is None:
                flops_evt = generic
                source = "generic HELAS routine count (no measurement for these sources)"
            k_avg = sum(k_ms) / len(k_ms) / 1e3
            achieved = flops_evt * nevt / k_avg
            peak = PEAK_FP64_VALU if prec == 'fp64' else PEAK_FP32_VALU
            v = {
                "workload": f"{proc} {nevt} events seed {seed}",
                "precision": prec,
                "value": nevt * args.steps / wall,
                "unit": "MEs/s (sampler + SIGMAKIN, wall clock over the timed steps)",
                "ms_per_step": wall / args.steps * 1e3,
                "sigmakin_ms": k_avg * 1e3,
                "nonfinite": nonfinite,
                "scopes": scopes,
                "graph": {"value": graph["wall_MEs_per_s"],
                          "unit": "MEs/s (sampler + SIGMAKIN replayed from one HIP graph, wall clock)",
                          "replays_equal_eager": graph["replays_equal_eager"]},
                "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                             "peak": peak / 1e12, "unit": "TFLOP/s",
                             "frac": achieved / peak, "traffic": traffic.get(prec),
                             "flops_per_event": flops_evt, "flops_source": source,
                             "generic_flops_per_event": generic},
            }
            if calibration:
                # against what a stream of independent FMAs of the same
                # precision reaches on this chip (unpacked FP32: packed FP32
                # instructions are disabled in every build)
                cal = calibration['fp64_vector_fma' if prec == 'fp64'
                                  else 'fp32_vector_fma_unpacked']['achieved_TFLOPs']
                v["roofline"]["calibrated_peak"] = cal
                v["roofline"]["frac_vs_calibrated"] = achieved / 1e12 / cal
            if prec.startswith('mixed'):
                v["mfma"] = mfma_work(meta['ncol'], nhel, prec, proc, k_avg, nevt)
            if name in cpu:
                v["vs_oracle"] = parity_vs_oracle(eng, torch, me, nevt, cpu[name]["results"])
            variants[f"{name}_{prec}"] = v
            del eng, me
            torch.cuda.empty_cache()
    gradient = None
    if do_grad:
        proc, nevt, seed, precs = GRADIENT
        gradient = {"workload": f"{proc} {nevt} events seed {seed}: d(w |M|^2)/dr, d log w/dr "
                                f"({4 * 3} uniforms per event)"}
        for prec in precs:
            print(f"[bench] gradient {prec} {nevt} events", file=sys.stderr, flush=True)
            gradient[prec] = run_gradient(mg, torch, prec, nevt, seed, args.steps, 1,
                                          cpu.get('gradient', {}).get('results'))
    plateau = None
    if do_plateau:
        proc, nevt, seed, prec = PLATEAU
        print(f"[bench] plateau {proc} {nevt} events", file=sys.stderr, flush=True)
        eng, wall, k_ms, nonfinite, scopes, me, graph = run_gpu(mg, torch, proc, prec, seed, nevt,
                                                                args.steps, args.warmup)
        plateau = {"workload": f"{proc} {nevt} events seed {seed}", "precision": prec,
                   "value": nevt * args.steps / wall, "scopes": scopes,
                   "graph": {"value": graph["wall_MEs_per_s"],
                             "replays_equal_eager": graph["replays_equal_eager"]},
                   "sigmakin_ms": sum(k_ms) / len(k_ms), "nonfinite": nonfinite}
        del eng, me
        torch.cuda.empty_cache()

    cpu_line = None
    if HEADLINE in cpu:
        c = cpu[HEADLINE]
        cpu_line = {"value": c["all_cores"]["value"], "unit": "MEs/s", "cores": cores,
                    "kind": "oracle", "single_core_value": c["single_core"]["value"],
                    "cpu": cpu_model(),
                    "sample": (f"events of the headline workload (seed 3) from {cores} disjoint "
                               f"ranges: RNG + RAMBO + |M|^2 by the Python/torch FP64 oracle, "
                               f"{cores} processes x 1 thread for >= {args.cpu_seconds:g} s each "
                               f"({c['all_cores']['events']} events in "
                               f"{c['all_cores']['seconds']:.1f} s; start-up excluded)"),
                    "per_workload": {k: {"single_core": v["single_core"],
                                         "all_cores": v["all_cores"]}
                                     for k, v in cpu.items()}}
    head = variants.get(f"{HEADLINE}_fp64") or (next(iter(variants.values())) if variants else None)
    line = {
        "metric": METRIC,
        "value": head["value"] if head else None,
        "unit": "MEs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"] if head else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (head["value"] / PAPER_V100_GGTTGG
                        if head and head["workload"].startswith('ggttgg ') else None),
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"] + " sqrt(s)=1500 GeV (Philox + RAMBO + |M|^2)"
                   if head else None,
                   "parallelism": "1 GPU, one event per wave, one helicity per lane"},
        "roofline": head["roofline"] if head else None,
        "vs_oracle": head.get("vs_oracle") if head else None,
        "cpu_baseline": cpu_line,
        "calibration": calibration,
        "variants": variants,
        "gradient": gradient,
        "plateau": plateau,
    }
    print(json.dumps(line), flush=True)


if __name__ == '__main__':
    main()
