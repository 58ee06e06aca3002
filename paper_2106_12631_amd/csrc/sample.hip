// Random numbers and RAMBO phase space on gfx950 (one event per lane).
//
// Random numbers (Sec. IV.b): Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11) with key = seed and counter = (global event index, block j), so
// every event's uniforms depend only on (seed, event): the reproducibility
// the paper obtains from identical host/device cuRAND sequences (Sec. III).
// Slot s of an event uses block s/2; the 64-bit word is
// x[2(s%2)] + 2^32 x[2(s%2)+1] and u = ((w >> 11) + 1/2) 2^-53.
//
// Phase space: RAMBO (rambo.h) on the uniforms of each event.
#include "common.h"
#include "internal.h"
#include "philox.h"
#include "rambo.h"

namespace mg {

template <int NRND>
__device__ __forceinline__ void event_uniforms(uint64_t seed, uint64_t ievt, double (&u)[NRND]) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int j = 0; j < (NRND + 1) / 2; ++j) {
    uint32_t c0 = (uint32_t)ievt, c1 = (uint32_t)(ievt >> 32), c2 = (uint32_t)j, c3 = 0u;
    philox10(c0, c1, c2, c3, k0, k1);
    u[2 * j] = bits_to_u(c0, c1);
    if (2 * j + 1 < NRND) u[2 * j + 1] = bits_to_u(c2, c3);
  }
}

template <int NRND>
__global__ void __launch_bounds__(256) rng_kernel(uint64_t seed, int64_t off, int64_t nevt,
                                                  double* __restrict__ rnd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  double u[NRND];
  event_uniforms<NRND>(seed, (uint64_t)(off + i), u);
#pragma unroll
  for (int k = 0; k < NRND; ++k) rnd[aosoa_rnd(i, k, NRND)] = u[k];
}

template <int NF>
__device__ __forceinline__ void store_event(int64_t i, const double (&p)[NF + 2][4], double w,
                                            double* __restrict__ mom, double* __restrict__ wgt) {
#pragma unroll
  for (int ip = 0; ip < NF + 2; ++ip)
#pragma unroll
    for (int m = 0; m < 4; ++m) mom[aosoa_mom(i, ip, m, NF + 2)] = p[ip][m];
  wgt[i] = w;
}

template <int NF>
__global__ void __launch_bounds__(256) rambo_kernel(const double* __restrict__ rnd, int64_t nevt,
                                                    RamboArgs a, double* __restrict__ mom,
                                                    double* __restrict__ wgt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  double r[4 * NF];
#pragma unroll
  for (int k = 0; k < 4 * NF; ++k) r[k] = rnd[aosoa_rnd(i, k, 4 * NF)];
  double p[NF + 2][4], w;
  rambo<NF>(r, a, p, w);
  store_event<NF>(i, p, w, mom, wgt);
}

template <int NF>
__global__ void __launch_bounds__(256) sample_kernel(uint64_t seed, int64_t off, int64_t nevt,
                                                     RamboArgs a, double* __restrict__ rnd,
                                                     double* __restrict__ mom,
                                                     double* __restrict__ wgt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  double r[4 * NF];
  event_uniforms<4 * NF>(seed, (uint64_t)(off + i), r);
  if (rnd) {
#pragma unroll
    for (int k = 0; k < 4 * NF; ++k) rnd[aosoa_rnd(i, k, 4 * NF)] = r[k];
  }
  double p[NF + 2][4], w;
  rambo<NF>(r, a, p, w);
  store_event<NF>(i, p, w, mom, wgt);
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int launch_rng(int nrnd, uint64_t seed, int64_t off, int64_t nevt, double* rnd, hipStream_t s) {
  const unsigned g = blocks_for(nevt, 256);
  switch (nrnd) {
    case 8: rng_kernel<8><<<g, 256, 0, s>>>(seed, off, nevt, rnd); break;
    case 12: rng_kernel<12><<<g, 256, 0, s>>>(seed, off, nevt, rnd); break;
    case 16: rng_kernel<16><<<g, 256, 0, s>>>(seed, off, nevt, rnd); break;
    default: return -1;
  }
  return 0;
}

int launch_rambo(int nf, const double* rnd, int64_t nevt, const RamboArgs& a, double* mom,
                 double* wgt, hipStream_t s) {
  const unsigned g = blocks_for(nevt, 256);
  switch (nf) {
    case 2: rambo_kernel<2><<<g, 256, 0, s>>>(rnd, nevt, a, mom, wgt); break;
    case 3: rambo_kernel<3><<<g, 256, 0, s>>>(rnd, nevt, a, mom, wgt); break;
    case 4: rambo_kernel<4><<<g, 256, 0, s>>>(rnd, nevt, a, mom, wgt); break;
    default: return -1;
  }
  return 0;
}

int launch_sample(int nf, uint64_t seed, int64_t off, int64_t nevt, const RamboArgs& a,
                  double* rnd, double* mom, double* wgt, hipStream_t s) {
  const unsigned g = blocks_for(nevt, 256);
  switch (nf) {
    case 2: sample_kernel<2><<<g, 256, 0, s>>>(seed, off, nevt, a, rnd, mom, wgt); break;
    case 3: sample_kernel<3><<<g, 256, 0, s>>>(seed, off, nevt, a, rnd, mom, wgt); break;
    case 4: sample_kernel<4><<<g, 256, 0, s>>>(seed, off, nevt, a, rnd, mom, wgt); break;
    default: return -1;
  }
  return 0;
}

}  // namespace mg
