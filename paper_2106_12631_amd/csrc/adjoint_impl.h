// Gradient of the event weight f(r) = |M|^2(p(r)) w(r) with respect to the
// uniforms r of one event, and of log w (the differentiable event weight of
// a phase-space adaptation built on RAMBO and SIGMAKIN).
//
// Reverse mode: per helicity the generated
// code runs the amplitudes forward, forms the colour-flow adjoints
// Jb = 2 C J / den from the colour sum, and sweeps back through the
// amplitude terms and currents (helas_adj.h) to the final-state momenta,
// accumulating d|M|^2/dp over helicities.  The momenta depend on the
// uniforms only through RAMBO, whose Jacobian dp/dr_j (and dw/dr_j) comes
// from one cheap dual-number RAMBO pass per uniform; then
//   df/dr_j = (1/IDEN) (w sum_{leg,mu} d|M|^2/dp dp/dr_j + |M|^2 dw/dr_j).
// The helicity sum, the momentum adjoints and /IDEN are in FP64; the
// amplitudes and their adjoints in FP64 or FP32 (mixed).
#pragma once
#include "common.h"
#include "helas_adj.h"
#include "internal.h"
#include "rambo.h"

namespace mg {

// Adjoint accumulators of the reverse sweep in LDS (when the generated code
// has slots): slot s of a lane is 4 complex values at base + s * SLOT, with
// the lanes of a slot LANE bytes apart (8 bytes of padding per lane spread
// the accesses of consecutive lanes over the banks; 16 bytes run as fast but
// take 11 % more LDS).  Every access launders the address, so the compiler
// keeps no accumulator in registers across the sweep: the registers stay
// with the recomputed forward values.  The slots of a 64-lane block must
// leave room for four blocks per CU (40 KB each).
typedef __attribute__((address_space(3))) char lds_char;

#ifndef MG_ADJ_LANE_PAD
#define MG_ADJ_LANE_PAD 8
#endif
template <typename T>
struct AdjSlots {
  static constexpr int LANE = 4 * (int)sizeof(cx<T>) + MG_ADJ_LANE_PAD;
  static constexpr int SLOT = 64 * LANE;
  lds_char* base;  // this lane's slot 0
  __device__ __forceinline__ cx<T>* slot(int s) const {
    int off = s * SLOT;
    asm volatile("" : "+v"(off));
    return (cx<T>*)(base + off);
  }
  __device__ __forceinline__ void clear(int s) const {
    cx<T>* w = slot(s);
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = cx<T>{(T)0, (T)0};
  }
};

template <class P, int NF, typename T>
__global__ void __launch_bounds__(64)
    adjoint_kernel(const double* __restrict__ rnd, int64_t nevt, RamboArgs ra, HelList hl,
                   Couplings<T> c, double inv_iden, const double* __restrict__ gbar,
                   double* __restrict__ grad_rnd, double* __restrict__ grad_logw,
                   double* __restrict__ mew) {
  using D = dual<double>;
  constexpr int NR = 4 * NF, NP = NF + 2;
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= nevt) return;
  double r[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) r[k] = rnd[aosoa_rnd(i, k, NR)];
  double p[NP][4], w;
  rambo<NF>(r, ra, p, w);
  set_beams(p);  // RAMBO's incoming momenta, on the axis: the beam body
  double pb[NP][4];
#pragma unroll
  for (int l = 0; l < NP; ++l)
#pragma unroll
    for (int m = 0; m < 4; ++m) pb[l][m] = 0.0;
  double me = 0.0;
  static_assert(P::SLOTS * AdjSlots<T>::SLOT <= 40 * 1024, "adjoint slots: four blocks per CU");
  __shared__ char slots[P::SLOTS > 0 ? P::SLOTS * AdjSlots<T>::SLOT : 1];
  const AdjSlots<T> ws{(lds_char*)(slots + threadIdx.x * AdjSlots<T>::LANE)};
#pragma nounroll
  for (int h = 0; h < hl.n; ++h) me += P::template adjoint<true>(p, hl.code[h], c, pb, ws);
  const double g = gbar ? gbar[i] : 1.0;
  // the uniforms are read again rather than kept live across the helicity
  // loop (an opaque index keeps the compiler from reusing the first loads)
  int64_t ir = i;
  asm volatile("" : "+v"(ir));
#pragma unroll
  for (int k = 0; k < NR; ++k) r[k] = rnd[aosoa_rnd(ir, k, NR)];
#pragma nounroll
  for (int j = 0; j < NR; ++j) {
    D rd[NR], pd[NP][4], wd;
#pragma unroll
    for (int k = 0; k < NR; ++k) rd[k] = D(r[k], k == j ? 1.0 : 0.0);
    rambo<NF>(rd, ra, pd, wd);
    double s = 0.0;
#pragma unroll
    for (int l = 2; l < NP; ++l)
#pragma unroll
      for (int m = 0; m < 4; ++m) s += pb[l][m] * pd[l][m].d;
    const double df = inv_iden * (w * s + me * wd.d);
    grad_rnd[aosoa_rnd(i, j, NR)] = g * df;
    if (grad_logw) grad_logw[aosoa_rnd(i, j, NR)] = wd.d / wd.v;
  }
  if (mew) mew[i] = me * inv_iden * w;
}

template <class P, int NF, typename T>
int adjoint_launch(const MeArgs& a, const RamboArgs& ra, const Couplings<T>& c, const double* rnd,
                   int64_t nevt, const double* gbar, double* grad_rnd, double* grad_logw,
                   double* mew, hipStream_t s) {
  const unsigned g = (unsigned)((nevt + 63) / 64);
  adjoint_kernel<P, NF, T><<<g, 64, 0, s>>>(rnd, nevt, ra, a.hel, c, a.inv_iden, gbar, grad_rnd,
                                            grad_logw, mew);
  return 0;
}

}  // namespace mg
