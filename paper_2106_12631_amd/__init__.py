"""Per-event |M|^2 on AMD MI355X (gfx950): thin binding over libmg5mi.so.

Only argument marshalling lives here: torch supplies device memory and the
current HIP stream, and every step of the path (random numbers, RAMBO,
helicity amplitudes, colour and helicity sums) runs in the library's HIP
kernels through the C ABI of include/mg5mi.h.  There is no CPU fallback: if
the library is missing, construction raises.
"""
import ctypes
import os

import torch

__all__ = ['MEEngine', 'MEWeight', 'PROCESSES', 'PRECISIONS', 'lib', 'library_path', 'engine',
           'sample', 'sigmakin', 'xsec_stats', 'unweight']

_HERE = os.path.dirname(os.path.abspath(__file__))
PROCESSES = {'eemumu': 0, 'ggtt': 1, 'ggttg': 2, 'ggttgg': 3}
PRECISIONS = {'fp64': 0, 'fp32amp': 1, 'mixed': 2, 'mixed_f32mfma': 3}


class Params(ctypes.Structure):
    _fields_ = [('sqrts', ctypes.c_double), ('alpha_inv', ctypes.c_double),
                ('gfermi', ctypes.c_double), ('mZ', ctypes.c_double), ('wZ', ctypes.c_double),
                ('mt', ctypes.c_double), ('wt', ctypes.c_double), ('alphas', ctypes.c_double),
                ('flags', ctypes.c_int)]


# bits of Params.flags (include/mg5mi.h)
FLAG_TCHANNEL_ZERO_WIDTH = 1
FLAG_WEIGHT_2PI = 2
FLAG_NO_PRECISION_GUARD = 4

DEFAULT_PARAMS = dict(sqrts=1500.0, alpha_inv=132.5, gfermi=1.16639e-5, mZ=91.188, wZ=2.441,
                      mt=173.0, wt=1.49, alphas=0.118, flags=0)


class Layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in
                ('npar', 'nparf', 'nrnd', 'nhel', 'nhel_good', 'ncol', 'ndiag', 'neppM', 'neppR',
                 'iden')]


_LIB = None


def library_path():
    """The in-tree library; MG5MI_LIBRARY may name another build of it."""
    return os.environ.get('MG5MI_LIBRARY') or os.path.join(_HERE, 'libmg5mi.so')


def lib():
    """Load libmg5mi.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2106_12631_amd.build`")
    L = ctypes.CDLL(path)
    vp, i64, u64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    sigs = {
        'mg_create': [ci, ci, ctypes.POINTER(Params), ctypes.POINTER(vp)],
        'mg_destroy': [vp],
        'mg_layout': [vp, ctypes.POINTER(Layout)],
        'mg_rng': [vp, u64, i64, i64, vp, vp],
        'mg_rambo': [vp, vp, i64, vp, vp, vp],
        'mg_sample': [vp, u64, i64, i64, vp, vp, vp, vp],
        'mg_sigmakin': [vp, vp, i64, vp, vp, vp, vp],
        'mg_sigmakin_hel': [vp, vp, i64, vp, vp],
        'mg_count_nonfinite': [vp, i64, vp, vp],
        'mg_adjoint': [vp, vp, i64, vp, vp, vp, vp, vp],
        'mg_xsec_stats': [vp, i64, vp, vp, vp],
        'mg_xsec': [vp, vp, i64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
        'mg_unweight': [vp, i64, ctypes.c_double, u64, i64, vp, vp, vp, vp],
        'mg_unweight_noalloc': [vp, i64, ctypes.c_double, u64, i64, vp, vp, vp],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ci
    for name in ('mg_unweight_workspace_bytes', 'mg_xsec_stats_workspace_bytes'):
        getattr(L, name).argtypes = [i64]
        getattr(L, name).restype = i64
    L.mg_strerror.argtypes = [ci]
    L.mg_strerror.restype = ctypes.c_char_p
    _LIB = L
    return L


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed: {lib().mg_strerror(rc).decode()} ({rc})")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class MEEngine:
    """One process at one precision on one device (wraps an mg_handle_t)."""

    def __init__(self, process, precision='fp64', params=None, device='cuda'):
        self.process = process
        self.precision = precision
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device('cuda', torch.cuda.current_device())
        prm = dict(DEFAULT_PARAMS)
        prm.update(params or {})
        self.params = prm
        L = lib()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.mg_create(PROCESSES[process], PRECISIONS[precision],
                               ctypes.byref(Params(**prm)), ctypes.byref(h)), 'mg_create')
        self._h = h
        lay = Layout()
        _check(L.mg_layout(h, ctypes.byref(lay)), 'mg_layout')
        self.layout = lay

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and _LIB is not None:
            _LIB.mg_destroy(h)
            self._h = None

    # ------------------------------------------------------------ buffers
    def _pages(self, nevt, nepp):
        return (nevt + nepp - 1) // nepp

    def empty_mom(self, nevt):
        lay = self.layout
        return torch.empty(self._pages(nevt, lay.neppM) * lay.npar * 4 * lay.neppM,
                           dtype=torch.float64, device=self.device)

    def empty_rnd(self, nevt):
        lay = self.layout
        return torch.empty(self._pages(nevt, lay.neppR) * lay.nrnd * lay.neppR,
                           dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------ layout views
    def mom_events(self, mom, nevt):
        """AoSoA momenta -> (nevt, npar, 4) tensor (copy)."""
        lay = self.layout
        v = mom.view(-1, lay.npar, 4, lay.neppM).permute(0, 3, 1, 2)
        return v.reshape(-1, lay.npar, 4)[:nevt].contiguous()

    def events_mom(self, p):
        """(nevt, npar, 4) tensor -> AoSoA momenta on this device (padded page)."""
        lay = self.layout
        nevt = p.shape[0]
        npg = self._pages(nevt, lay.neppM)
        buf = torch.zeros(npg * lay.neppM, lay.npar, 4, dtype=torch.float64, device=self.device)
        buf[:nevt] = p.to(self.device, torch.float64)
        return buf.view(npg, lay.neppM, lay.npar, 4).permute(0, 2, 3, 1).contiguous().view(-1)

    def rnd_events(self, rnd, nevt):
        lay = self.layout
        v = rnd.view(-1, lay.nrnd, lay.neppR).permute(0, 2, 1)
        return v.reshape(-1, lay.nrnd)[:nevt].contiguous()

    def events_rnd(self, r):
        lay = self.layout
        nevt = r.shape[0]
        npg = self._pages(nevt, lay.neppR)
        buf = torch.full((npg * lay.neppR, lay.nrnd), 0.5, dtype=torch.float64, device=self.device)
        buf[:nevt] = r.to(self.device, torch.float64)
        return buf.view(npg, lay.neppR, lay.nrnd).permute(0, 2, 1).contiguous().view(-1)

    # ------------------------------------------------------------ the path
    def rng(self, seed, nevt, offset=0, out=None):
        rnd = self.empty_rnd(nevt) if out is None else out
        _check(lib().mg_rng(self._h, seed, offset, nevt, _ptr(rnd), _stream(self.device)), 'mg_rng')
        return rnd

    def rambo(self, rnd, nevt, mom=None, wgt=None):
        mom = self.empty_mom(nevt) if mom is None else mom
        wgt = torch.empty(nevt, dtype=torch.float64, device=self.device) if wgt is None else wgt
        _check(lib().mg_rambo(self._h, _ptr(rnd), nevt, _ptr(mom), _ptr(wgt),
                              _stream(self.device)), 'mg_rambo')
        return mom, wgt

    def sample(self, seed, nevt, offset=0, keep_rnd=False, mom=None, wgt=None):
        rnd = self.empty_rnd(nevt) if keep_rnd else None
        mom = self.empty_mom(nevt) if mom is None else mom
        wgt = torch.empty(nevt, dtype=torch.float64, device=self.device) if wgt is None else wgt
        _check(lib().mg_sample(self._h, seed, offset, nevt, _ptr(rnd), _ptr(mom), _ptr(wgt),
                               _stream(self.device)), 'mg_sample')
        return rnd, mom, wgt

    def sigmakin(self, mom, nevt, wgt=None, me=None, evtw=None):
        me = torch.empty(nevt, dtype=torch.float64, device=self.device) if me is None else me
        if wgt is not None and evtw is None:
            evtw = torch.empty(nevt, dtype=torch.float64, device=self.device)
        _check(lib().mg_sigmakin(self._h, _ptr(mom), nevt, _ptr(me), _ptr(wgt), _ptr(evtw),
                                 _stream(self.device)), 'mg_sigmakin')
        return me if wgt is None else (me, evtw)

    def sigmakin_hel(self, mom, nevt):
        out = torch.empty(self.layout.nhel, nevt, dtype=torch.float64, device=self.device)
        _check(lib().mg_sigmakin_hel(self._h, _ptr(mom), nevt, _ptr(out), _stream(self.device)),
               'mg_sigmakin_hel')
        return out

    def adjoint(self, rnd, nevt, gbar=None, want_logw=True, want_f=True):
        """Gradient of f = w |M|^2 with respect to the uniforms (AoSoA like
        rnd), optionally scaled per event by gbar; also d log w / dr and f."""
        grad = torch.empty_like(rnd)
        glogw = torch.empty_like(rnd) if want_logw else None
        f = torch.empty(nevt, dtype=torch.float64, device=self.device) if want_f else None
        _check(lib().mg_adjoint(self._h, _ptr(rnd), nevt, _ptr(gbar), _ptr(grad), _ptr(glogw),
                                _ptr(f), _stream(self.device)), 'mg_adjoint')
        return grad, glogw, f

    def event_weight(self, r):
        """Differentiable f(r) = w(r) |M|^2(p(r)) for event-major uniforms
        r of shape (nevt, nrnd) (see MEWeight)."""
        return MEWeight.apply(r, self)

    def cross_section(self, evtw, nevt):
        """(sigma [pb], Monte Carlo error [pb], stats) from the weighted
        events evtw = w |M|^2 (mg_xsec_stats on the device, mg_xsec on the
        host; stats = sum, sum of squares, max, finite count)."""
        st = xsec_stats(evtw[:nevt])
        host = st.cpu()
        sig, err = ctypes.c_double(), ctypes.c_double()
        _check(lib().mg_xsec(self._h, ctypes.c_void_p(host.data_ptr()), nevt, ctypes.byref(sig),
                             ctypes.byref(err)), 'mg_xsec')
        return sig.value, err.value, host

    def count_nonfinite(self, x):
        cnt = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().mg_count_nonfinite(_ptr(x), x.numel(), _ptr(cnt), _stream(self.device)),
               'mg_count_nonfinite')
        return int(cnt.item())


class MEWeight(torch.autograd.Function):
    """f(r) = w(r) |M|^2(p(r)) per event as a differentiable torch function.

    forward: RAMBO and SIGMAKIN kernels (mg_rambo, mg_sigmakin);
    backward: the gradient kernel (mg_adjoint) with gbar = grad_output,
    so r.grad[i, j] = grad_output[i] * df_i/dr_ij.
    r: float64 device tensor (nevt, nrnd) of uniforms in (0, 1).
    """

    @staticmethod
    def forward(ctx, r, engine):
        nevt = r.shape[0]
        rnd = engine.events_rnd(r.detach())
        mom, wgt = engine.rambo(rnd, nevt)
        _, evtw = engine.sigmakin(mom, nevt, wgt=wgt)
        ctx.engine = engine
        ctx.save_for_backward(r.detach())
        return evtw

    @staticmethod
    def backward(ctx, gout):
        (r,) = ctx.saved_tensors
        eng = ctx.engine
        nevt = r.shape[0]
        grad, _, _ = eng.adjoint(eng.events_rnd(r), nevt, gbar=gout.contiguous().to(torch.float64),
                                 want_logw=False, want_f=False)
        return eng.rnd_events(grad, nevt), None


# ----------------------------------------------------------------------------- shortcuts
_ENGINES = {}


def engine(process='ggttgg', precision='fp64', device=None):
    """A cached MEEngine per (process, precision, device) with default params."""
    dev = torch.device('cuda', torch.cuda.current_device()) if device is None else torch.device(device)
    key = (process, precision, str(dev))
    if key not in _ENGINES:
        _ENGINES[key] = MEEngine(process, precision, device=dev)
    return _ENGINES[key]


def sample(seed, nevt, process='ggttgg', offset=0, keep_rnd=True):
    """Random numbers and RAMBO events: (rnd AoSoA or None, mom AoSoA, wgt)."""
    return engine(process).sample(seed, nevt, offset=offset, keep_rnd=keep_rnd)


def sigmakin(mom, nevt, wgt=None, process='ggttgg', precision='fp64'):
    """|M|^2 per event for AoSoA momenta (and w |M|^2 if wgt is given)."""
    return engine(process, precision).sigmakin(mom, nevt, wgt=wgt)


def xsec_stats(f):
    """Device tensor (4,) = (sum, sum of squares, max, count) of the finite f."""
    f = f.contiguous()
    out = torch.empty(4, dtype=torch.float64, device=f.device)
    nb = lib().mg_xsec_stats_workspace_bytes(f.numel())
    ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=f.device)
    _check(lib().mg_xsec_stats(_ptr(f), f.numel(), _ptr(out), _ptr(ws), _stream(f.device)),
           'mg_xsec_stats')
    return out


def unweight(f, fmax, seed, evt_offset=0):
    """Hit-or-miss unweighting: device int64 tensor of the kept event indices
    (increasing): event i is kept iff u_i fmax < f[i] (mg_unweight)."""
    f = f.contiguous()
    n = f.numel()
    idx = torch.empty(max(n, 1), dtype=torch.int64, device=f.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=f.device)
    nb = lib().mg_unweight_workspace_bytes(n)
    ws = torch.empty((nb + 7) // 8, dtype=torch.int64, device=f.device)
    _check(lib().mg_unweight(_ptr(f), n, float(fmax), int(seed), int(evt_offset), _ptr(idx),
                             _ptr(cnt), _ptr(ws), _stream(f.device)), 'mg_unweight')
    return idx[:int(cnt.item())]
