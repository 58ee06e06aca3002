"""Gradient-based phase-space adaptation on top of the gradient kernel.

The paper's sampler is flat RAMBO on uniform random numbers (Sec. IV.a);
its event weights w |M|^2 vary over many decades, which costs Monte Carlo
efficiency.  Here a differentiable map of the uniforms, x = g(u), is
trained so that the integrand seen by the sampler,

    F(u) = f(g(u)) |dg/du|,      f = w |M|^2  (MEWeight: RAMBO + SIGMAKIN),

has a small relative second moment E[F^2] / E[F]^2 (the variance of the
cross-section estimate per event, up to a constant).  The gradient of F with
respect to the map's parameters needs df/dx, which the gradient kernel
(mg_adjoint, the backward pass of MEWeight) provides.  E[F] is the same
integral for every map, so the adapted sampler stays unbiased.

Without cuts a process with a final-state gluon has an infrared-divergent
cross section (soft and beam-collinear gluons): E[F] grows with the sample
and no map gives a finite variance.  The adaptation therefore takes an
optional generator-level cut, pT > ptmin for chosen final-state particles,
applied to the RAMBO momenta of each point (the integrand is f times the
cut's indicator; the indicator is piecewise constant and carries no
gradient).

Two maps:
  WarpMap       separable: per uniform, a monotone piecewise-linear warp of
                (0, 1) with nbins equal input bins whose output widths are
                softmax(logits) (a VEGAS-like grid trained by gradient
                descent instead of by histogram refinement);
  CouplingFlow  non-separable: a stack of piecewise-linear coupling layers
                (the normalising-flow construction of neural importance
                sampling: each layer warps half of the uniforms with bin
                widths that a small network computes from the other half),
                able to follow the correlations that RAMBO's boost puts
                between the uniforms and the physical angles and energies.
Both are torch arithmetic on the device; the matrix elements and their
gradients come from the library's kernels.
"""
import math

import torch


class WarpMap(torch.nn.Module):
    """Per-dimension monotone piecewise-linear map of (0, 1) onto itself."""

    def __init__(self, ndim, nbins=32, device=None, dtype=torch.float64, floor=0.0):
        super().__init__()
        self.ndim, self.nbins, self.floor = ndim, nbins, floor
        self.logits = torch.nn.Parameter(torch.zeros(ndim, nbins, dtype=dtype, device=device))

    def forward(self, u):
        """x = g(u) and the Jacobian |dg/du| per event; u: (N, ndim) in (0, 1)."""
        K = self.nbins
        # output bin widths (ndim, K); `floor` mixes in the uniform map so that
        # no bin is compressed below floor / K (bounds the weights' growth)
        w = (1.0 - self.floor) * torch.softmax(self.logits, dim=-1) + self.floor / K
        x, d = _pwl(u, w.unsqueeze(0))
        tiny = torch.finfo(u.dtype).eps
        return x.clamp(tiny, 1.0 - tiny), d.prod(dim=-1)

    def inverse(self, x):
        """u = g^-1(x) and the Jacobian |dg/du| at u."""
        K = self.nbins
        w = (1.0 - self.floor) * torch.softmax(self.logits, dim=-1) + self.floor / K
        u, d = _pwl_inverse(x, w.unsqueeze(0))
        return u, d.prod(dim=-1)


def _onehot(k, K, dtype):
    return (k.unsqueeze(-1) == torch.arange(K, device=k.device)).to(dtype)


# The bin lookups below select with one-hot masks and sums instead of
# gather / advanced indexing: the backward pass of those scatters into the
# widths with atomic additions on the device, whose order (and so the
# rounding of the trained map) changes from run to run.  Masked sums reduce
# in a fixed order, so training is reproducible bit for bit.
def _pwl(u, w):
    """Monotone piecewise-linear map of (0, 1) with equal input bins and
    output bin widths w (..., K), summing to 1: x and dx/du per entry."""
    K = w.shape[-1]
    t = u * K
    k = t.detach().floor().clamp(0, K - 1)
    oh = _onehot(k.long(), K, w.dtype)
    left = torch.cumsum(w, dim=-1) - w
    wk = (oh * w).sum(-1)
    x = (oh * left).sum(-1) + (t - k) * wk
    return x, K * wk


def _pwl_inverse(x, w):
    """Inverse of _pwl: u with _pwl(u, w) = x, and dx/du at u."""
    K = w.shape[-1]
    right = torch.cumsum(w, dim=-1)
    # the output bin of x: the number of right edges at or below x
    k = (right.detach() <= x.detach().unsqueeze(-1)).sum(-1).clamp(0, K - 1)
    oh = _onehot(k, K, w.dtype)
    wk = (oh * w).sum(-1)
    left = (oh * (right - w)).sum(-1)
    u = (k.to(x.dtype) + (x - left) / wk) / K
    return u, K * wk


class CouplingFlow(torch.nn.Module):
    """Stack of piecewise-linear coupling layers on (0, 1)^ndim.

    Layer l splits the dimensions by bit (l // 2) of their index (the
    complement on odd l, so every dimension is transformed and every pair of
    dimensions is split by some layer); the transformed half is warped as in
    _pwl with widths (1 - floor) softmax(net_l(identity half)) + floor / K.
    The last linear layer of every network starts at zero: the flow starts
    as the identity map."""

    def __init__(self, ndim, nbins=32, layers=None, hidden=64, device=None,
                 dtype=torch.float64, floor=0.0):
        super().__init__()
        self.ndim, self.nbins, self.floor = ndim, nbins, floor
        nbits = max(1, (ndim - 1).bit_length())
        layers = 2 * nbits if layers is None else layers
        self.masks = []
        self.nets = torch.nn.ModuleList()
        for l in range(layers):
            bit = (l // 2) % nbits
            m = [((d >> bit) & 1) == (l % 2) for d in range(ndim)]
            if all(m) or not any(m):
                m = [d % 2 == l % 2 for d in range(ndim)]
            ia = [d for d in range(ndim) if not m[d]]   # identity half
            ib = [d for d in range(ndim) if m[d]]       # transformed half
            self.masks.append((ia, ib))
            net = torch.nn.Sequential(
                torch.nn.Linear(len(ia), hidden, dtype=dtype, device=device), torch.nn.ReLU(),
                torch.nn.Linear(hidden, hidden, dtype=dtype, device=device), torch.nn.ReLU(),
                torch.nn.Linear(hidden, len(ib) * nbins, dtype=dtype, device=device))
            torch.nn.init.zeros_(net[-1].weight)
            torch.nn.init.zeros_(net[-1].bias)
            self.nets.append(net)

    def forward(self, u):
        """x = g(u) and the Jacobian |dg/du| per event; u: (N, ndim) in (0, 1)."""
        K = self.nbins
        x = u
        jac = torch.ones(u.shape[0], dtype=u.dtype, device=u.device)
        for (ia, ib), net in zip(self.masks, self.nets):
            logits = net(x[:, ia]).view(-1, len(ib), K)
            w = (1.0 - self.floor) * torch.softmax(logits, dim=-1) + self.floor / K
            xb, db = _pwl(x[:, ib], w)
            x = x.index_copy(1, torch.tensor(ib, device=u.device), xb)
            jac = jac * db.prod(dim=-1)
        tiny = torch.finfo(u.dtype).eps
        return x.clamp(tiny, 1.0 - tiny), jac

    def inverse(self, x):
        """u = g^-1(x) and the Jacobian |dg/du| at u (layers in reverse; the
        identity half of a layer is the same before and after it)."""
        K = self.nbins
        u = x
        jac = torch.ones(x.shape[0], dtype=x.dtype, device=x.device)
        for (ia, ib), net in zip(reversed(self.masks), reversed(self.nets)):
            logits = net(u[:, ia]).view(-1, len(ib), K)
            w = (1.0 - self.floor) * torch.softmax(logits, dim=-1) + self.floor / K
            ub, db = _pwl_inverse(u[:, ib], w)
            u = u.index_copy(1, torch.tensor(ib, device=x.device), ub)
            jac = jac * db.prod(dim=-1)
        return u, jac


MAPS = {'warp': WarpMap, 'coupling': CouplingFlow}


def pt_cut(engine, particles, ptmin):
    """Indicator of pT > ptmin for every particle in `particles` (0-based
    indices in the process's particle order) at the RAMBO momenta of the
    event-major uniforms r: a function r -> (N,) float64 tensor of 0 / 1."""
    particles = list(particles)

    def mask(r):
        n = r.shape[0]
        with torch.no_grad():
            mom, _ = engine.rambo(engine.events_rnd(r.detach()), n)
            p = engine.mom_events(mom, n)[:, particles]
            pt = torch.hypot(p[..., 1], p[..., 2])
            return (pt > ptmin).all(dim=-1).to(r.dtype)
    return mask


def relative_second_moment(F):
    m = F.mean()
    return (F * F).mean() / (m * m)


def estimate(F):
    """Mean, its standard error and the relative variance of a weight sample."""
    n = F.numel()
    m = float(F.mean())
    v = float(F.var(unbiased=True))
    return m, math.sqrt(v / n), v / (m * m)


def sample_weights(m, fn, u, mix=0.0):
    """Weights F = f(x) / q(x) of a batch drawn from the defensive mixture
    q = mix + (1 - mix) q_g of the flat density and the map's density
    q_g = 1 / |dg/du| (Hesterberg's defensive importance sampling: F <= f / mix
    wherever the map thins out).  The first round(mix N) rows of u are used
    as flat points x = u, the others through the map, x = g(u); the mean of F
    estimates the integral of f for any map.  mix = 0: F = f(g(u)) |dg/du|."""
    nf = int(round(mix * u.shape[0])) if mix > 0 else 0
    xg, jg = m(u[nf:])
    if nf:
        xf = u[:nf]
        _, jf = m.inverse(xf)
        x, jac = torch.cat([xf, xg]), torch.cat([jf, jg])
    else:
        x, jac = xg, jg
    return fn(x) / (mix + (1.0 - mix) / jac)


def train(fn, ndim, uniforms, iters=200, batch=1 << 14, nbins=32, lr=0.05, device=None,
          log=None, clip=0.995, floor=0.0, flow='warp', mix=0.0):
    """Train a map for the integrand fn (a differentiable torch function
    of (N, ndim) points in (0, 1) returning (N,) weights); uniforms(i, n)
    returns the i-th batch of n uniforms.  The loss is the relative second
    moment E[F^2]/E[F]^2 of the weights capped at the batch's `clip`
    quantile; floor: see WarpMap; flow: 'warp'
    (WarpMap) or 'coupling' (CouplingFlow); mix: the flat share of the
    defensive mixture (see sample_weights), trained as it is evaluated.
    Returns the map and the loss history."""
    m = MAPS[flow](ndim, nbins, device=device, floor=floor)
    opt = torch.optim.Adam(m.parameters(), lr=lr)
    hist = []
    for it in range(iters):
        F = sample_weights(m, fn, uniforms(it, batch), mix)
        F = F[torch.isfinite(F)]
        # the weights are heavy-tailed: the training loss caps them at the
        # batch's `clip` quantile (the estimates always use the raw weights)
        cap = torch.quantile(F.detach(), clip) if clip < 1.0 else None
        value = relative_second_moment(torch.minimum(F, cap) if cap is not None else F)
        opt.zero_grad()
        value.backward()
        torch.nn.utils.clip_grad_norm_(m.parameters(), 1.0)
        opt.step()
        hist.append(float(value.detach()))
        if log and (it % max(1, iters // 10) == 0 or it == iters - 1):
            log(f"iter {it} variance loss {hist[-1]:.4g}")
    return m, hist


def adapt_process(engine, seed=4, iters=200, batch=1 << 14, nbins=32, lr=0.05, eval_batch=1 << 18,
                  log=None, cut=None, clip=0.995, floor=0.0, flow='warp', mix=0.0):
    """Adapt the uniforms of engine's process and compare with flat sampling.

    cut: None or a function r -> (N,) indicator (see pt_cut) multiplying
    the integrand; mix: flat share of the defensive mixture (sample_weights).  Training batches use Philox(seed) event ranges
    [i batch, (i+1) batch); the two evaluations use disjoint ranges of
    Philox(seed + 1).  Returns a dict with both estimates of <w |M|^2 cut>,
    their errors, relative variances and the variance reduction."""
    nr = engine.layout.nrnd

    def uniforms(i, n, s=seed):
        return engine.rnd_events(engine.rng(s, n, offset=i * n), n)

    def fn(x):
        f = engine.event_weight(x)
        return f if cut is None else f * cut(x)

    m, hist = train(fn, nr, uniforms, iters, batch, nbins, lr, device=engine.device, log=log,
                    clip=clip, floor=floor, flow=flow, mix=mix)
    with torch.no_grad():
        u = uniforms(0, eval_batch, seed + 1)
        flat = fn(u)
        adapted = sample_weights(m, fn, uniforms(1, eval_batch, seed + 1), mix)
    flat = flat[torch.isfinite(flat)]
    adapted = adapted[torch.isfinite(adapted)]
    ef, ea = estimate(flat), estimate(adapted)
    # the raw relative variance is dominated by a few extreme weights; the
    # capped one (both samples capped at the flat sample's 99.9% quantile)
    # shows the bulk of the distribution
    cap = torch.quantile(flat, 0.999)
    cf = estimate(torch.minimum(flat, cap))[2]
    ca = estimate(torch.minimum(adapted, cap))[2]
    return {"flat": {"mean": ef[0], "error": ef[1], "relative_variance": ef[2],
                     "capped_relative_variance": cf},
            "adapted": {"mean": ea[0], "error": ea[1], "relative_variance": ea[2],
                        "capped_relative_variance": ca},
            "variance_reduction": ef[2] / ea[2], "capped_variance_reduction": cf / ca,
            "loss_history": hist, "map": m}
