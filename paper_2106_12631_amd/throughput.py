"""Throughput against the number of events per launch (one GPU).

The paper measures how many events a launch needs before the GPU's matrix-
element throughput reaches its plateau (Sec. IV.b: O(1M) events for
e+e- -> mu+mu-, ~16k for g g -> t t~ g g).  This sweeps events per launch
for one process and precision and prints one JSON line per size with the
median over `steps` launches (HIP events on the launching stream) of the
SIGMAKIN kernel alone and of sampler + SIGMAKIN.

    python -m paper_2106_12631_amd.throughput --process eemumu --max-log2 24
"""
import argparse
import json
import os
import sys


def _median(x):
    x = sorted(x)
    n = len(x)
    return 0.5 * (x[(n - 1) // 2] + x[n // 2])


def sweep(process, precision, sizes, steps=12, warmup=2, seed=0):
    import torch
    import paper_2106_12631_amd as mg
    eng = mg.MEEngine(process, precision)
    stream = torch.cuda.current_stream()
    out = []
    for n in sizes:
        mom = eng.empty_mom(n)
        wgt = torch.empty(n, dtype=torch.float64, device=eng.device)
        me = torch.empty(n, dtype=torch.float64, device=eng.device)
        for _ in range(warmup):
            eng.sample(seed, n, mom=mom, wgt=wgt)
            eng.sigmakin(mom, n, me=me)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for k in range(steps):
            ev[k][0].record(stream)
            eng.sample(seed, n, mom=mom, wgt=wgt)
            ev[k][1].record(stream)
            eng.sigmakin(mom, n, me=me)
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        sk = _median([b.elapsed_time(c) for a, b, c in ev]) / 1e3
        st = _median([a.elapsed_time(c) for a, b, c in ev]) / 1e3
        rec = {"process": process, "precision": precision, "nevt": n,
               "sigmakin_MEs_per_s": n / sk, "sample_sigmakin_MEs_per_s": n / st,
               "sigmakin_ms": sk * 1e3}
        print(json.dumps(rec), flush=True)
        out.append(rec)
        del mom, wgt, me
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--process', default='eemumu')
    ap.add_argument('--precision', default='fp64')
    ap.add_argument('--min-log2', type=int, default=10)
    ap.add_argument('--max-log2', type=int, default=24)
    ap.add_argument('--steps', type=int, default=12)
    args = ap.parse_args()
    sweep(args.process, args.precision,
          [1 << k for k in range(args.min_log2, args.max_log2 + 1)], steps=args.steps)


if __name__ == '__main__':
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
