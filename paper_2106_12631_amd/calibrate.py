"""Calibration of the arithmetic peaks on the device (not part of the path).

Runs the kernels of calib/calibrate.hip (libmg5cal.so): FP64 and FP32
vector FMA streams and BF16, FP32 and FP64 MFMA streams, each on a grid of
16 waves per CU, and reports the FLOP/s each reaches next to the published
MI355X peak it is compared with.

    python -m paper_2106_12631_amd.calibrate
"""
import ctypes
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, 'libmg5cal.so')

# kind: (name, published dense peak FLOP/s, iterations for ~10 ms)
KINDS = {
    0: ('fp64_vector_fma', 78.6e12, 10000),
    1: ('fp32_vector_fma_unpacked', 157.3e12, 10000),
    2: ('bf16_mfma_32x32x16', 2.5e15, 40000),
    3: ('fp32_mfma_32x32x2', 157.3e12, 20000),
    4: ('fp64_mfma_16x16x4', 78.6e12, 20000),
}


def run(blocks=1024):
    import torch
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built: run `python -m paper_2106_12631_amd.build`")
    L = ctypes.CDLL(LIB)
    L.mgcal_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.mgcal_run.restype = ctypes.c_int
    out = torch.empty(blocks * 256, dtype=torch.float64, device='cuda')
    torch.cuda.synchronize()
    res = {}
    for kind, (name, peak, iters) in KINDS.items():
        f, t = ctypes.c_double(), ctypes.c_double()
        rc = L.mgcal_run(kind, blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.byref(f),
                         ctypes.byref(t))
        if rc != 0:
            raise RuntimeError(f"calibration kernel {name} failed ({rc})")
        res[name] = {"achieved_TFLOPs": f.value / 1e12, "published_TFLOPs": peak / 1e12,
                     "frac": f.value / peak, "ms": t.value * 1e3}
    return res


if __name__ == '__main__':
    import sys
    sys.path.insert(0, os.path.dirname(_HERE))
    print(json.dumps(run()), flush=True)
