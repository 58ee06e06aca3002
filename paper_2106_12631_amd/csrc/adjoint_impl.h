// Gradient of the event weight f(r) = |M|^2(p(r)) w(r) with respect to the
// uniforms r of one event, and of log w (the differentiable event weight of
// a phase-space adaptation built on RAMBO and SIGMAKIN).
//
// Forward mode: for each of the 4 nparf uniforms the kernel seeds that
// uniform's derivative, carries value and derivative through RAMBO (the
// Newton rescaling by the implicit-function theorem) and through the
// generated helicity amplitudes and colour sum (instantiated on dual
// numbers), and reads df/dr_j and dw/dr_j off the result.  Per event this
// costs 4 nparf dual passes, which is cheaper in registers than storing
// every intermediate wavefunction for a reverse sweep.  The helicity sum and
// /IDEN are in FP64 (dual<double>); the amplitudes in dual<double> or
// dual<float> (mixed).
#pragma once
#include "common.h"
#include "internal.h"
#include "rambo.h"

namespace mg {

template <class P, int NF, typename TD>
__global__ void __launch_bounds__(64)
    grad_kernel(const double* __restrict__ rnd, int64_t nevt, RamboArgs ra, HelList hl,
                Couplings<base_t<TD>> c, double inv_iden, const double* __restrict__ gbar,
                double* __restrict__ grad_rnd, double* __restrict__ grad_logw,
                double* __restrict__ mew) {
  using D = dual<double>;
  constexpr int NR = 4 * NF;
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= nevt) return;
  double r[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) r[k] = rnd[aosoa_rnd(i, k, NR)];
  const double g = gbar ? gbar[i] : 1.0;
  double fval = 0.0;
#pragma nounroll
  for (int j = 0; j < NR; ++j) {
    D w;
    {
      D rd[NR], p[NF + 2][4];
#pragma unroll
      for (int k = 0; k < NR; ++k) rd[k] = D(r[k], k == j ? 1.0 : 0.0);
      rambo<NF>(rd, ra, p, w);
    }
    D me = 0.0;
#pragma nounroll
    for (int h = 0; h < hl.n; ++h) {
      // RAMBO is re-run per helicity from opaque copies of the uniforms: it
      // is cheap, and keeping the dual momenta live across the helicity loop
      // is not.
      D rq[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        double rv = r[k];
        opaque(rv);
        rq[k] = D(rv, k == j ? 1.0 : 0.0);
      }
      D p[NF + 2][4], wq;
      rambo<NF>(rq, ra, p, wq);
      cx<TD> J[P::NCOL];
      P::jamps(p, hl.code[h], c, J);
      me += D(P::colour_sum(J));
    }
    const D f = me * inv_iden * w;
    grad_rnd[aosoa_rnd(i, j, NR)] = g * f.d;
    if (grad_logw) grad_logw[aosoa_rnd(i, j, NR)] = w.d / w.v;
    fval = f.v;
  }
  if (mew) mew[i] = fval;
}

template <class P, int NF, typename TD>
int grad_launch(const MeArgs& a, const RamboArgs& ra, const Couplings<base_t<TD>>& c,
                const double* rnd, int64_t nevt, const double* gbar, double* grad_rnd,
                double* grad_logw, double* mew, hipStream_t s) {
  const unsigned g = (unsigned)((nevt + 63) / 64);
  grad_kernel<P, NF, TD><<<g, 64, 0, s>>>(rnd, nevt, ra, a.hel, c, a.inv_iden, gbar, grad_rnd,
                                          grad_logw, mew);
  return 0;
}

}  // namespace mg
