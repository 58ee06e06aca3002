// Random numbers and RAMBO phase space on gfx950 (one event per lane).
//
// Random numbers (Sec. IV.b): Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11) with key = seed and counter = (global event index, block j), so
// every event's uniforms depend only on (seed, event): the reproducibility
// the paper obtains from identical host/device cuRAND sequences (Sec. III).
// Slot s of an event uses block s/2; the 64-bit word is
// x[2(s%2)] + 2^32 x[2(s%2)+1] and u = ((w >> 11) + 1/2) 2^-53.
//
// Phase space (Sec. IV.a/IV.b; Kleiss, Stirling, Ellis, CPC 40 (1986) 359):
// four uniforms per final-state particle give an isotropic massless q_i
// with energy -ln(r2 r3); the q_i are boosted to the rest frame of their sum
// and scaled to sqrt(s); masses are introduced by a Newton solve for the
// common scale xi of the three-momenta, in FP64.
#include "common.h"
#include "internal.h"

namespace mg {

constexpr uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    const uint32_t hi0 = __umulhi(PHILOX_M0, c0), lo0 = PHILOX_M0 * c0;
    const uint32_t hi1 = __umulhi(PHILOX_M1, c2), lo1 = PHILOX_M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

__device__ __forceinline__ double bits_to_u(uint32_t lo, uint32_t hi) {
  const uint64_t w = ((uint64_t)hi << 32) | lo;
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

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

// RAMBO for NF final-state particles.  p[0], p[1] are the incoming momenta
// along +z and -z; returns false if the Newton solve did not converge.
template <int NF>
__device__ __forceinline__ bool rambo(const double (&r)[4 * NF], const RamboArgs& a,
                                      double (&p)[NF + 2][4], double& w) {
  const double twopi = 6.283185307179586476925286766559;
  double q[NF][4];
  double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const double c = 2.0 * r[4 * i] - 1.0;
    const double st = sqrt(1.0 - c * c);
    double sph, cph;
    sincos(twopi * r[4 * i + 1], &sph, &cph);
    const double q0 = -log(r[4 * i + 2] * r[4 * i + 3]);
    q[i][0] = q0;
    q[i][1] = q0 * st * cph;
    q[i][2] = q0 * st * sph;
    q[i][3] = q0 * c;
#pragma unroll
    for (int m = 0; m < 4; ++m) Q[m] += q[i][m];
  }
  const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b1 = -Q[1] / M, b2 = -Q[2] / M, b3 = -Q[3] / M;
  const double gam = Q[0] / M;
  const double aa = 1.0 / (1.0 + gam);
  const double x = a.sqrts / M;
  const double h = 0.5 * a.sqrts;
  p[0][0] = h; p[0][1] = 0.0; p[0][2] = 0.0; p[0][3] = h;
  p[1][0] = h; p[1][1] = 0.0; p[1][2] = 0.0; p[1][3] = -h;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const double bq = b1 * q[i][1] + b2 * q[i][2] + b3 * q[i][3];
    p[i + 2][0] = x * (gam * q[i][0] + bq);
    p[i + 2][1] = x * (q[i][1] + b1 * q[i][0] + aa * bq * b1);
    p[i + 2][2] = x * (q[i][2] + b2 * q[i][0] + aa * bq * b2);
    p[i + 2][3] = x * (q[i][3] + b3 * q[i][0] + aa * bq * b3);
  }
  w = a.w0;
  if (!a.massive) return true;
  // Newton solve of sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s)
  double xi = a.xi0;
  bool ok = false;
  for (int it = 0; it <= 50; ++it) {
    double f = -a.sqrts, fp = 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const double E = p[i + 2][0];
      const double root = sqrt(a.m2[i] + xi * xi * E * E);
      f += root;
      fp += xi * E * E / root;
    }
    if (fabs(f) <= 1e-14 * a.sqrts) {
      ok = true;
      break;
    }
    if (it == 50) break;
    xi -= f / fp;
  }
  double prod = 1.0, den = 0.0;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const double E = p[i + 2][0];
    const double k0 = sqrt(a.m2[i] + xi * xi * E * E);
    const double kx = xi * p[i + 2][1], ky = xi * p[i + 2][2], kz = xi * p[i + 2][3];
    const double kabs = sqrt(kx * kx + ky * ky + kz * kz);
    prod *= kabs / k0;
    den += kabs * kabs / k0;
    p[i + 2][0] = k0;
    p[i + 2][1] = kx;
    p[i + 2][2] = ky;
    p[i + 2][3] = kz;
  }
  double xin = 1.0;
#pragma unroll
  for (int k = 0; k < 2 * NF - 3; ++k) xin *= xi;
  w = a.w0 * xin * prod * a.sqrts / den;
  if (!ok) w = __builtin_nan("");
  return ok;
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
