// SIGMAKIN kernels for one process (Sec. II, Sec. IV.b).  Per helicity the
// generated straight-line code builds the colour-flow amplitudes and the
// colour sum gives the helicity's |M|^2; the helicity sum is in FP64.
//   sigmakin_kernel          one event per lane, the loop over the kept
//                            helicities inside the lane (the paper's layout);
//   sigmakin_hpl_kernel      one event per wave, one helicity per lane (64
//                            helicities): wave-uniform momenta in scalar
//                            registers, helicity sum by wave reduction;
//   sigmakin_mixed_kernel    event per lane with the colour sum on the
//                            matrix cores (colour_mfma.h);
//   sigmakin_mixed_hpl_kernel  one event per wave, one helicity per lane,
//                            the 64 helicities' amplitudes as the 64 columns
//                            of the matrix-core colour sum.
#pragma once
#include "colour_mfma.h"
#include "common.h"
#include "internal.h"

// Threads per block of the event-per-lane kernel (e+e- -> mu+mu-, g g -> t
// t~, g g -> t t~ g); -DMG_EPL_BLOCK=n builds another block size.
#ifndef MG_EPL_BLOCK
#define MG_EPL_BLOCK 256
#endif

// Launches of fewer events than a per-process threshold (written by the
// generator) use several lanes per event (one kept helicity per lane,
// sigmakin_group_kernel) in the event-per-lane processes;
// -DMG_GROUP_MAX_EVENTS=n sets one threshold for all of them.
constexpr int64_t group_max_events(int64_t per_process) {
#ifdef MG_GROUP_MAX_EVENTS
  return (int64_t)(MG_GROUP_MAX_EVENTS) + 0 * per_process;
#else
  return per_process;
#endif
}

namespace mg {

// Workgroups are handed to the 8 XCDs of the chip in turn (block b to XCD
// b % 8), each with its own L2.  With one event per block, consecutive
// events share the 64-byte lines of the AoSoA momenta, so the event of
// block b is chosen to give XCD x one contiguous range of events, walked in
// dispatch order: a bijection of [0, nblocks).
__device__ __forceinline__ int64_t xcd_event(int64_t b, int64_t nblocks) {
  constexpr int NXCD = 8;
  const int64_t q = nblocks / NXCD, r = nblocks % NXCD;
  const int64_t x = b % NXCD, k = b / NXCD;
  return x * q + (x < r ? x : r) + k;
}

template <class P>
__device__ __forceinline__ void load_event(const double* __restrict__ mom, int64_t i,
                                           double (&p)[P::NPAR][4]) {
#pragma unroll
  for (int ip = 0; ip < P::NPAR; ++ip)
#pragma unroll
    for (int m = 0; m < 4; ++m) p[ip][m] = mom[aosoa_mom(i, ip, m, P::NPAR)];
}

// The momenta of event i for one pass of a helicity loop.  With REREAD they
// are read again (cache hits) through an event index the compiler cannot see
// through, so that no helicity-independent subexpression (momentum sums,
// propagator denominators) is hoisted out of the loop and kept live across
// it: for the processes whose amplitude code fills the register file,
// recomputing them is cheap and keeping them is not.  Otherwise the copy q0
// loaded before the loop is used and those parts are computed once per
// event.  (The generator sets REREAD_MOMENTA per process and kernel.)
template <class P, bool REREAD>
__device__ __forceinline__ void event_momenta(const double* __restrict__ mom, int64_t i,
                                              const double (&q0)[P::NPAR][4],
                                              double (&q)[P::NPAR][4]) {
  if constexpr (REREAD) {
    int64_t iq = i;
    asm volatile("" : "+v"(iq));
    load_event<P>(mom, iq, q);
  } else {
#pragma unroll
    for (int ip = 0; ip < P::NPAR; ++ip)
#pragma unroll
      for (int m = 0; m < 4; ++m) q[ip][m] = q0[ip][m];
  }
}

// me[i] = inv_iden * sum_k |M|^2(helicity hl.code[k]); with mehel != null the
// per-helicity values are also stored at mehel[hl.code[k] * nevt + i].
template <class P, typename T, int BS>
__global__ void __launch_bounds__(BS)
    sigmakin_kernel(const double* __restrict__ mom, int64_t nevt, double* __restrict__ me,
                    const double* __restrict__ wgt, double* __restrict__ evtw,
                    double* __restrict__ mehel, HelList hl, Couplings<T> c, double inv_iden) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= nevt) return;
  double q0[P::NPAR][4];
  load_event<P>(mom, i, q0);
  auto hel_sum = [&](auto beam) {
    constexpr bool B = decltype(beam)::value;
    double acc = 0.0;
#pragma nounroll
    for (int k = 0; k < hl.n; ++k) {
      double q[P::NPAR][4];
      event_momenta<P, P::REREAD_MOMENTA>(mom, i, q0, q);
      if constexpr (B) set_beams(q);
      cx<T> J[P::NCOL];
      P::template jamps<T, false, B>(q, hl.code[k], c, J);
      const double v = (double)P::template colour_sum<T>(J);
      if (mehel) mehel[(int64_t)hl.code[k] * nevt + i] = v;
      acc += v;
    }
    return acc;
  };
  // the beam body when every active lane of the wave has its beams on the axis
  const double acc = __all(beams_on_axis(q0)) ? hel_sum(Beam<true>{}) : hel_sum(Beam<false>{});
  const double m = acc * inv_iden;
  if (me) me[i] = m;
  if (evtw) evtw[i] = m * wgt[i];
}

// Mixed precision: FP32 amplitudes, colour sum on the matrix cores (CS =
// ColourMfmaF32 or ColourMfmaBf16), FP64 helicity sum.  One wave per block;
// lanes past nevt compute a copy of the last event and store nothing, so
// every lane takes part in the wave-wide MFMA exchange.
template <class P, template <int> class CS>
__global__ void __launch_bounds__(64)
    sigmakin_mixed_kernel(const double* __restrict__ mom, int64_t nevt, double* __restrict__ me,
                          const double* __restrict__ wgt, double* __restrict__ evtw, HelList hl,
                          Couplings<float> c, double inv_iden) {
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool valid = i < nevt;
  const int64_t il = valid ? i : nevt - 1;
  // the matrix-core A operands (the colour matrix) wait in LDS while the
  // amplitude code runs and are reloaded for each colour sum
  using CSN = CS<P::NCOL>;
  __shared__ typename CSN::Word tab[CSN::KB * 64];
  CSN cs;
  cs.init(CSN::template table<P>(), lane);
  cs.save(tab, lane);
  const double scale = inv_iden / P::CDEN;
  double q0[P::NPAR][4];
  load_event<P>(mom, il, q0);
  auto hel_sum = [&](auto beam) {
    constexpr bool B = decltype(beam)::value;
    double acc = 0.0;
#pragma nounroll
    for (int k = 0; k < hl.n; ++k) {
      double q[P::NPAR][4];
      event_momenta<P, P::REREAD_MOMENTA>(mom, il, q0, q);
      if constexpr (B) set_beams(q);
      cx<float> J[P::NCOL];
      P::template jamps<float, false, B>(q, hl.code[k], c, J);
      int lt = lane;
      asm volatile("" : "+v"(lt));
      cs.restore(tab, lt);
      acc += (double)cs.sum(J, lane);
    }
    return acc;
  };
  const double acc = __all(beams_on_axis(q0)) ? hel_sum(Beam<true>{}) : hel_sum(Beam<false>{});
  if (valid) {
    const double m = acc * scale;
    if (me) me[i] = m;
    if (evtw) evtw[i] = m * wgt[i];
  }
}

template <class P, template <int> class CS>
int sigmakin_mixed_launch(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                          const double* wgt, double* evtw, hipStream_t s) {
  const unsigned g = (unsigned)((nevt + 63) / 64);
  sigmakin_mixed_kernel<P, CS><<<g, 64, 0, s>>>(mom, nevt, me, wgt, evtw, a.hel, a.c32, a.inv_iden);
  return 0;
}

template <class P, typename T, int BS>
int sigmakin_launch(const MeArgs& a, const Couplings<T>& c, const double* mom, int64_t nevt,
                    double* me, const double* wgt, double* evtw, double* mehel, hipStream_t s) {
  const unsigned g = (unsigned)((nevt + BS - 1) / BS);
  HelList hl = a.hel;
  if (mehel) {  // every helicity
    hl.n = 1 << P::NPAR;
    for (int k = 0; k < hl.n; ++k) hl.code[k] = (uint8_t)k;
  }
  sigmakin_kernel<P, T, BS><<<g, BS, 0, s>>>(mom, nevt, me, wgt, evtw, mehel, hl, c, a.inv_iden);
  return 0;
}

// One event per wave, one helicity per lane: for a process with 64
// helicities, all kept, lane h of block i computes helicity h of event i.
// The momenta are the same in every lane and stay in scalar registers (the
// generated code is instantiated with uniform momenta), which leaves the
// vector registers to the wavefunctions and colour-flow amplitudes; the
// helicity sum is a wave reduction.  The grid has exactly nevt blocks.
template <class P, typename T>
__global__ void __launch_bounds__(64)
    sigmakin_hpl_kernel(const double* __restrict__ mom, int64_t nevt, double* __restrict__ me,
                        const double* __restrict__ wgt, double* __restrict__ evtw,
                        double* __restrict__ mehel, Couplings<T> c, double inv_iden) {
  static_assert((1 << P::NPAR) == 64, "one helicity per lane of a wave64");
  const int64_t i = xcd_event(blockIdx.x, nevt);
  const unsigned h = threadIdx.x;
  double q[P::NPAR][4];
  load_event<P>(mom, i, q);
  cx<T> J[P::NCOL];
  if (beams_on_axis(q)) {  // wave-uniform
    set_beams(q);
    P::template jamps<T, true, true>(q, h, c, J);
  } else {
    P::template jamps<T, true, false>(q, h, c, J);
  }
  double v = (double)P::template colour_sum<T>(J);
  if (mehel) mehel[(int64_t)h * nevt + i] = v;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (h == 0) {
    const double m = v * inv_iden;
    if (me) me[i] = m;
    if (evtw) evtw[i] = m * wgt[i];
  }
}

// Several lanes per event, one kept helicity per lane: for L = hl.n kept
// helicities (a power of two up to 64), 64 / L events per wave, lane k of an
// event's group computing helicity hl.code[k]; the helicity sum is a
// butterfly over the group.  Every lane loads its event's momenta (the
// group's lanes read the same lines).  For small launches it spreads the
// helicity loop of the event-per-lane kernel over L times more lanes.  The
// groups of events past nevt return whole, so every butterfly stays inside
// active lanes.
template <class P, typename T, int BS>
__global__ void __launch_bounds__(BS)
    sigmakin_group_kernel(const double* __restrict__ mom, int64_t nevt, double* __restrict__ me,
                          const double* __restrict__ wgt, double* __restrict__ evtw, HelList hl,
                          Couplings<T> c, double inv_iden, int lanes_log2) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t i = t >> lanes_log2;
  const int L = 1 << lanes_log2;
  const int k = (int)(t & (L - 1));
  if (i >= nevt) return;
  double q[P::NPAR][4];
  load_event<P>(mom, i, q);
  cx<T> J[P::NCOL];
  if (__all(beams_on_axis(q))) {
    set_beams(q);
    P::template jamps<T, false, true>(q, hl.code[k], c, J);
  } else {
    P::template jamps<T, false, false>(q, hl.code[k], c, J);
  }
  double v = (double)P::template colour_sum<T>(J);
  for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (k == 0) {
    const double m = v * inv_iden;
    if (me) me[i] = m;
    if (evtw) evtw[i] = m * wgt[i];
  }
}

// the group kernel when the kept helicities are a power of two and the
// launch has fewer than `max_events` events (where the event-per-lane kernel
// leaves compute units idle), else the event-per-lane kernel
template <class P, typename T, int BS>
int sigmakin_group_launch(const MeArgs& a, const Couplings<T>& c, const double* mom, int64_t nevt,
                          double* me, const double* wgt, double* evtw, double* mehel,
                          int64_t max_events, hipStream_t s) {
  const int n = a.hel.n;
  if (!mehel && nevt > 0 && nevt < max_events && n > 1 && n <= 64 && (n & (n - 1)) == 0) {
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    const int64_t threads = nevt << lg;
    const unsigned g = (unsigned)((threads + BS - 1) / BS);
    sigmakin_group_kernel<P, T, BS><<<g, BS, 0, s>>>(mom, nevt, me, wgt, evtw, a.hel, c,
                                                     a.inv_iden, lg);
    return 0;
  }
  return sigmakin_launch<P, T, BS>(a, c, mom, nevt, me, wgt, evtw, mehel, s);
}

// Matrix-core colour sum of one helicity per lane.  The amplitudes reach it
// through LDS, jl[(2 k + part) * 64 + lane] (each lane reads back only its
// own values, so no barrier is needed): with the MFMA results in VGPRs
// (-amdgpu-mfma-vgpr-form, a flag of the mixed sources) the kernel keeps the
// register allocation of the FP32 amplitude body, 253 VGPRs, no AGPRs and
// no scratch: two waves per SIMD.  (Out of line behind a call it needed a
// 72-byte stack frame per lane and ran 1.8 % slower; with the amplitudes
// passed in registers instead of LDS, 0.4 % slower.)
typedef __attribute__((address_space(3))) float lds_float;

template <template <int> class CS, int NCOL>
__device__ __forceinline__ float colour_sum_mfma_lds(const lds_float* jl,
                                                     const typename CS<NCOL>::Word* tab,
                                                     int lane) {
  CS<NCOL> cs;
  cs.init(tab, lane);
  return cs.sum_parts([&](int part, int k) { return jl[(2 * k + part) * 64 + lane]; },
                      [&](int kb) { return cs.a[kb]; }, lane);
}

// Mixed precision with one helicity per lane: the 64 helicities of one event
// are the 64 columns of the matrix-core colour sum (the same product as for
// 64 events), whose per-lane results are summed over the wave in FP64.
template <class P, template <int> class CS>
__global__ void __launch_bounds__(64)
    sigmakin_mixed_hpl_kernel(const double* __restrict__ mom, int64_t nevt,
                              double* __restrict__ me, const double* __restrict__ wgt,
                              double* __restrict__ evtw, Couplings<float> c, double inv_iden) {
  static_assert((1 << P::NPAR) == 64, "one helicity per lane of a wave64");
  const int64_t i = xcd_event(blockIdx.x, nevt);
  const int lane = threadIdx.x;
  double q[P::NPAR][4];
  load_event<P>(mom, i, q);
  cx<float> J[P::NCOL];
  if (beams_on_axis(q)) {  // wave-uniform
    set_beams(q);
    P::template jamps<float, true, true>(q, (unsigned)lane, c, J);
  } else {
    P::template jamps<float, true, false>(q, (unsigned)lane, c, J);
  }
__shared__ float jl[2 * P::NCOL * 64];
#pragma unroll
  for (int k = 0; k < P::NCOL; ++k) {
    jl[(2 * k) * 64 + lane] = J[k].r;
    jl[(2 * k + 1) * 64 + lane] = J[k].i;
  }
  double v = (double)colour_sum_mfma_lds<CS, P::NCOL>(
      (const lds_float*)jl, CS<P::NCOL>::template table<P>(), lane);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) {
    const double m = v * (inv_iden / P::CDEN);
    if (me) me[i] = m;
    if (evtw) evtw[i] = m * wgt[i];
  }
}

// Precision guard of the reduced-precision forms.  |M|^2 is ill-conditioned
// in its invariants when kappa = s / min_{i<j} |2 p_i.p_j| is large (a soft
// or collinear gluon): single Feynman-gauge diagrams ~ 1/s_ij cancel to an
// amplitude ~ 1/sqrt(s_ij), so FP32 rounding of the diagram sums grows like
// eps32 sqrt(kappa).  The guard recomputes in FP64 the events with
// kappa > kmax after a reduced-precision launch.  One wave scans 64 events
// (one per lane) and evaluates each flagged event with one helicity per lane
// (wave-uniform momenta, helicity sum by wave reduction), overwriting me and
// evtw; the scan finds none in most waves.
template <int NPAR>
__device__ __forceinline__ bool ill_conditioned(const double (&p)[NPAR][4], double kmax) {
  double m = __DBL_MAX__;
#pragma unroll
  for (int i = 0; i < NPAR; ++i)
#pragma unroll
    for (int j = i + 1; j < NPAR; ++j) {
      const double d = 2.0 * (p[i][0] * p[j][0] - p[i][1] * p[j][1] - p[i][2] * p[j][2] -
                              p[i][3] * p[j][3]);
      m = fmin(m, fabs(d));
    }
  const double E = p[0][0] + p[1][0], X = p[0][1] + p[1][1], Y = p[0][2] + p[1][2],
               Z = p[0][3] + p[1][3];
  return E * E - X * X - Y * Y - Z * Z > kmax * m;
}

template <class P>
__global__ void __launch_bounds__(64)
    sigmakin_guard_kernel(const double* __restrict__ mom, int64_t nevt, double* __restrict__ me,
                          const double* __restrict__ wgt, double* __restrict__ evtw, HelList hl,
                          Couplings<double> c, double inv_iden, double kmax) {
  const int lane = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  bool flag = false;
  if (i0 + lane < nevt) {
    double q[P::NPAR][4];
    load_event<P>(mom, i0 + lane, q);
    flag = ill_conditioned<P::NPAR>(q, kmax);
  }
  uint64_t pending = __ballot(flag);
  while (pending) {
    const int l = __ffsll((unsigned long long)pending) - 1;
    pending &= pending - 1;
    const int64_t e = i0 + l;
    double q[P::NPAR][4];
    load_event<P>(mom, e, q);
    double v = 0.0;
    for (int k = lane; k < hl.n; k += 64) {
      cx<double> J[P::NCOL];
      P::template jamps<double, true>(q, hl.code[k], c, J);
      v += P::template colour_sum<double>(J);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) {
      const double m = v * inv_iden;
      me[e] = m;
      if (evtw) evtw[e] = m * wgt[e];
    }
  }
}

template <class P>
int sigmakin_guard_launch(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                          const double* wgt, double* evtw, hipStream_t s) {
  if (!(a.guard_kappa > 0.0) || nevt <= 0) return 0;
  const unsigned g = (unsigned)((nevt + 63) / 64);
  sigmakin_guard_kernel<P><<<g, 64, 0, s>>>(mom, nevt, me, wgt, evtw, a.hel, a.c64, a.inv_iden,
                                            a.guard_kappa);
  return 0;
}

// helicity-per-lane mixed launch when every helicity is kept, else the
// event-per-lane mixed kernel (PH: the traits of the helicity-per-lane body)
template <class P, class PH, template <int> class CS>
int sigmakin_mixed_hpl_launch(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, hipStream_t s) {
  if (a.hel.n == (1 << P::NPAR) && nevt > 0 && nevt <= 0x7FFFFFFF) {
    sigmakin_mixed_hpl_kernel<PH, CS><<<(unsigned)nevt, 64, 0, s>>>(mom, nevt, me, wgt, evtw,
                                                                   a.c32, a.inv_iden);
    return 0;
  }
  return sigmakin_mixed_launch<P, CS>(a, mom, nevt, me, wgt, evtw, s);
}

// helicity-per-lane launch when every helicity is kept, else the
// event-per-lane kernel
template <class P, typename T, int BS>
int sigmakin_hpl_launch(const MeArgs& a, const Couplings<T>& c, const double* mom, int64_t nevt,
                        double* me, const double* wgt, double* evtw, double* mehel,
                        hipStream_t s) {
  if ((mehel || a.hel.n == (1 << P::NPAR)) && nevt > 0 && nevt <= 0x7FFFFFFF) {
    sigmakin_hpl_kernel<P, T><<<(unsigned)nevt, 64, 0, s>>>(mom, nevt, me, wgt, evtw, mehel, c,
                                                           a.inv_iden);
    return 0;
  }
  return sigmakin_launch<P, T, BS>(a, c, mom, nevt, me, wgt, evtw, mehel, s);
}

}  // namespace mg
