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

The map is separable: per uniform, a monotone piecewise-linear warp of
(0, 1) with nbins equal input bins whose output widths are softmax(logits)
(a VEGAS-like grid trained by gradient descent instead of by histogram
refinement).  It is elementwise torch arithmetic on the device; the matrix
elements and their gradients come from the library's kernels.
"""
import math

import torch


class WarpMap(torch.nn.Module):
    """Per-dimension monotone piecewise-linear map of (0, 1) onto itself."""

    def __init__(self, ndim, nbins=32, device=None, dtype=torch.float64):
        super().__init__()
        self.ndim, self.nbins = ndim, nbins
        self.logits = torch.nn.Parameter(torch.zeros(ndim, nbins, dtype=dtype, device=device))

    def forward(self, u):
        """x = g(u) and the Jacobian |dg/du| per event; u: (N, ndim) in (0, 1)."""
        K = self.nbins
        w = torch.softmax(self.logits, dim=-1)              # output bin widths (ndim, K)
        left = torch.cumsum(w, dim=-1) - w                   # output left edges
        t = u * K
        k = t.detach().floor().clamp(0, K - 1).long()        # input bin per (event, dim)
        frac = t - k
        dims = torch.arange(self.ndim, device=u.device).expand_as(k)
        wk = w[dims, k]
        x = left[dims, k] + frac * wk
        tiny = torch.finfo(u.dtype).eps
        x = x.clamp(tiny, 1.0 - tiny)
        jac = (K * wk).prod(dim=-1)
        return x, jac


def relative_second_moment(F):
    m = F.mean()
    return (F * F).mean() / (m * m)


def kl_divergence(F):
    """KL(p || q) up to a constant for the target density p = f / I and the
    sampling density q = 1 / |dg/du| of the map: E_u[(F/I) log(F/I)] with
    I estimated by the batch mean (held fixed in the gradient)."""
    r = F / F.mean().detach()
    return (r * torch.log(r.clamp_min(1e-300))).mean()


LOSSES = {'variance': relative_second_moment, 'kl': kl_divergence}


def estimate(F):
    """Mean, its standard error and the relative variance of a weight sample."""
    n = F.numel()
    m = float(F.mean())
    v = float(F.var(unbiased=True))
    return m, math.sqrt(v / n), v / (m * m)


def train(fn, ndim, uniforms, iters=200, batch=1 << 14, nbins=32, lr=0.05, device=None,
          log=None, clip=0.995, loss='variance'):
    """Train a WarpMap for the integrand fn (a differentiable torch function
    of (N, ndim) points in (0, 1) returning (N,) weights); uniforms(i, n)
    returns the i-th batch of n uniforms.  loss: 'variance' (relative second
    moment E[F^2]/E[F]^2) or 'kl' (KL divergence of the sampling density from
    the integrand), both on weights capped at the batch's `clip` quantile.
    Returns the map and the loss history."""
    m = WarpMap(ndim, nbins, device=device)
    opt = torch.optim.Adam(m.parameters(), lr=lr)
    hist = []
    for it in range(iters):
        u = uniforms(it, batch)
        x, jac = m(u)
        F = fn(x) * jac
        F = F[torch.isfinite(F)]
        # the weights are heavy-tailed: the training loss caps them at the
        # batch's `clip` quantile (the estimates always use the raw weights)
        cap = torch.quantile(F.detach(), clip) if clip < 1.0 else None
        value = LOSSES[loss](torch.minimum(F, cap) if cap is not None else F)
        opt.zero_grad()
        value.backward()
        torch.nn.utils.clip_grad_norm_(m.parameters(), 1.0)
        opt.step()
        hist.append(float(value.detach()))
        if log and (it % max(1, iters // 10) == 0 or it == iters - 1):
            log(f"iter {it} {loss} loss {hist[-1]:.4g}")
    return m, hist


def adapt_process(engine, seed=4, iters=200, batch=1 << 14, nbins=32, lr=0.05, eval_batch=1 << 18,
                  log=None):
    """Adapt the uniforms of engine's process and compare with flat sampling.

    Training batches use Philox(seed) event ranges [i batch, (i+1) batch);
    the two evaluations use disjoint ranges of Philox(seed + 1).  Returns a
    dict with both estimates of sum-of-weights (w |M|^2 means), their errors,
    relative variances and the variance reduction."""
    nr = engine.layout.nrnd

    def uniforms(i, n, s=seed):
        return engine.rnd_events(engine.rng(s, n, offset=i * n), n)

    def fn(x):
        return engine.event_weight(x)

    m, hist = train(fn, nr, uniforms, iters, batch, nbins, lr, device=engine.device, log=log)
    with torch.no_grad():
        u = uniforms(0, eval_batch, seed + 1)
        flat = fn(u)
        u2 = uniforms(1, eval_batch, seed + 1)
        x, jac = m(u2)
        adapted = fn(x) * jac
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
