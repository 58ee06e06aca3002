"""The allocation-free unweighting entry point against mg_unweight (GPU).

mg_unweight_noalloc runs the same three kernels as mg_unweight with the
per-block counts in the library's fixed device array instead of a caller
workspace.  Two calls in a row (the second with a smaller input, so stale
counts of the first call sit in the array) must give exactly the kept
indices and count of mg_unweight on the same inputs; sizes beyond the
array's limit are refused before anything runs.
"""
import ctypes
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12631_amd as mg
    lib = mg.lib()
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    lib.mg_unweight_noalloc.argtypes = [vp, i64, ctypes.c_double, u64, i64, vp, vp, vp]
    lib.mg_unweight_noalloc.restype = ctypes.c_int
    return lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _run(L, f, fmax, seed, off, noalloc):
    n = f.numel()
    dev = f.device
    idx = torch.full((max(n, 1),), -1, dtype=torch.int64, device=dev)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    if noalloc:
        rc = L.mg_unweight_noalloc(_p(f), n, fmax, seed, off, _p(idx), _p(cnt), stream)
    else:
        nb = L.mg_unweight_workspace_bytes(n)
        ws = torch.empty((nb + 7) // 8, dtype=torch.int64, device=dev)
        rc = L.mg_unweight(_p(f), n, fmax, seed, off, _p(idx), _p(cnt), _p(ws), stream)
    assert rc == 0, L.mg_strerror(rc)
    torch.cuda.synchronize(dev)
    c = int(cnt.item())
    return c, idx[:c].cpu()


def test_noalloc_matches_workspace_entry_point(L):
    dev = torch.device('cuda', 0)
    g = torch.Generator().manual_seed(7)
    cases = [(1 << 24, 3.0, 11, 5), (4133, 2.0, 12, 1 << 33)]  # the limit, then smaller
    for n, fmax, seed, off in cases:
        f = (torch.rand(n, generator=g, dtype=torch.float64) * fmax).to(dev)
        f[n // 3] = float('nan')
        say('unweight noalloc', n, fmax, seed, off)
        c1, i1 = _run(L, f, fmax, seed, off, noalloc=True)
        c2, i2 = _run(L, f, fmax, seed, off, noalloc=False)
        assert c1 == c2 and torch.equal(i1, i2)
        assert c1 > 0 and bool((i1[1:] > i1[:-1]).all())
        assert n // 3 not in set(i1.tolist())


def test_noalloc_limits_and_empty_input(L):
    dev = torch.device('cuda', 0)
    f = torch.ones(8, dtype=torch.float64, device=dev)
    idx = torch.empty(8, dtype=torch.int64, device=dev)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=dev)
    limit = 1 << 24
    # beyond the fixed array: refused before any launch (the buffers are too
    # small for such n, which is why nothing may run)
    assert L.mg_unweight_noalloc(_p(f), limit + 1, 1.0, 1, 0, _p(idx), _p(cnt), None) == -7
    assert b'allocation-free' in L.mg_strerror(-7)
    # empty input: count 0
    assert L.mg_unweight_noalloc(None, 0, 1.0, 1, 0, None, _p(cnt), None) == 0
    torch.cuda.synchronize(dev)
    assert int(cnt.item()) == 0
    # invalid arguments
    assert L.mg_unweight_noalloc(_p(f), 8, -1.0, 1, 0, _p(idx), _p(cnt), None) == -1
    assert L.mg_unweight_noalloc(_p(f), 8, 1.0, 1, 0, _p(idx), None, None) == -1
