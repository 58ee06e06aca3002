// RAMBO phase space for one event (Sec. IV.a/IV.b phase-space sampler;
// R. Kleiss, W.J. Stirling, S.D. Ellis, Comput. Phys. Commun. 40 (1986) 359).
//
// Four uniforms per final-state particle give an isotropic massless q_i
// with energy -ln(r2 r3); the q_i are boosted to the rest frame of their sum
// and scaled to sqrt(s); masses are introduced by a Newton solve for the
// common scale xi of the three-momenta, in FP64.  The boost is written with
// the pairwise Minkowski products of the q_i (identical to the published
// boost in exact arithmetic; its direct form loses ~gamma^2 of the digits,
// gamma = Q^0/M, when the q_i are nearly collinear).  Templated on the real
// type R: double, or dual<double> to carry the derivative with respect to
// one uniform (forward mode).  For duals the Newton solve runs on the values
// and xi's derivative follows from the implicit-function theorem applied to
// sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s), whose partial derivatives are
// xi^2 E_i / k_i^0 (in E_i) and sum_i xi E_i^2 / k_i^0 (in xi):
//   dxi = -xi (sum_i E_i dE_i / k_i^0) / (sum_i E_i^2 / k_i^0).
#pragma once
#include "helas.h"
#include "internal.h"

namespace mg {

__device__ __forceinline__ double with_xi_derivative(double xi, const double*, const double*,
                                                     const RamboArgs&, int) {
  return xi;
}
template <typename F>
__device__ __forceinline__ dual<F> with_xi_derivative(double xi, const dual<F>* E, const double*,
                                                      const RamboArgs& a, int nf) {
  F num = 0, den = 0;
  for (int i = 0; i < nf; ++i) {
    const double Ev = E[i].v;
    const double k0 = sqrt(a.m2[i] + xi * xi * Ev * Ev);
    num += Ev * E[i].d / k0;
    den += Ev * Ev / k0;
  }
  return dual<F>(xi, -xi * num / den);
}

// A quiet NaN hidden from the optimiser: the gradient units, which run RAMBO
// inside their kernel, are built with -ffinite-math-only.
__device__ __forceinline__ double failed_weight() {
  uint64_t bits = 0x7FF8000000000000ull;
  asm volatile("" : "+v"(bits));
  return __builtin_bit_cast(double, bits);
}

// p[0], p[1] are the incoming momenta along +z and -z; returns false (and a
// NaN weight) if the Newton solve did not converge.
template <int NF, typename R>
__device__ __forceinline__ bool rambo(const R (&r)[4 * NF], const RamboArgs& a,
                                      R (&p)[NF + 2][4], R& w) {
  const double twopi = 6.283185307179586476925286766559;
  R q0[NF], n[NF][3];
  R Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const R c = 2.0 * r[4 * i] - 1.0;
    const R st = sqrt(1.0 - c * c);
    R sph, cph;
    sincos(twopi * r[4 * i + 1], &sph, &cph);
    q0[i] = -log(r[4 * i + 2] * r[4 * i + 3]);
    n[i][0] = st * cph;
    n[i][1] = st * sph;
    n[i][2] = c;
    Q[0] += q0[i];
#pragma unroll
    for (int m = 0; m < 3; ++m) Q[m + 1] += q0[i] * n[i][m];
  }
  // Boost to the rest frame of Q from the Minkowski products of the massless
  // q_i, q_i.q_j = q_i^0 q_j^0 |n_i - n_j|^2 / 2 (exact for nearly collinear
  // q_i, where Q^0^2 - |Q|^2 cancels): M^2 = sum_{i != j} q_i.q_j, rest-frame
  // energies E_i = q_i.Q / M, three-momenta q_i - Q (q_i^0 + E_i)/(Q^0 + M).
  R EM[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) EM[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = i + 1; j < NF; ++j) {
      const R d0 = n[i][0] - n[j][0], d1 = n[i][1] - n[j][1], d2 = n[i][2] - n[j][2];
      const R dij = 0.5 * q0[i] * q0[j] * (d0 * d0 + d1 * d1 + d2 * d2);
      EM[i] += dij;
      EM[j] += dij;
    }
  R M2 = 0.0;
#pragma unroll
  for (int i = 0; i < NF; ++i) M2 += EM[i];
  const R M = sqrt(M2);
  const R x = a.sqrts / M;
  const R Q0M = Q[0] + M;
  const double h = 0.5 * a.sqrts;
  p[0][0] = h; p[0][1] = 0.0; p[0][2] = 0.0; p[0][3] = h;
  p[1][0] = h; p[1][1] = 0.0; p[1][2] = 0.0; p[1][3] = -h;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const R E = EM[i] / M;
    const R t = (q0[i] + E) / Q0M;
    p[i + 2][0] = x * E;
#pragma unroll
    for (int m = 0; m < 3; ++m) p[i + 2][m + 1] = x * (q0[i] * n[i][m] - Q[m + 1] * t);
  }
  w = a.w0;
  if (!a.massive) return true;
  // Newton solve of sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s) on the values
  double xiv = a.xi0;
  bool ok = false;
  for (int it = 0; it <= 50; ++it) {
    double f = -a.sqrts, fp = 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const double E = val(p[i + 2][0]);
      const double root = sqrt(a.m2[i] + xiv * xiv * E * E);
      f += root;
      fp += xiv * E * E / root;
    }
    if (fabs(f) <= 1e-14 * a.sqrts) {
      ok = true;
      break;
    }
    if (it == 50) break;
    xiv -= f / fp;
  }
  R E[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) E[i] = p[i + 2][0];
  const R xi = with_xi_derivative(xiv, E, a.m2, a, NF);
  R prod = 1.0, den = 0.0;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const R k0 = sqrt(a.m2[i] + xi * xi * E[i] * E[i]);
    const R kx = xi * p[i + 2][1], ky = xi * p[i + 2][2], kz = xi * p[i + 2][3];
    const R kabs = sqrt(kx * kx + ky * ky + kz * kz);
    prod = prod * (kabs / k0);
    den = den + kabs * kabs / k0;
    p[i + 2][0] = k0;
    p[i + 2][1] = kx;
    p[i + 2][2] = ky;
    p[i + 2][3] = kz;
  }
  R xin = 1.0;
#pragma unroll
  for (int k = 0; k < 2 * NF - 3; ++k) xin = xin * xi;
  w = a.w0 * xin * prod * a.sqrts / den;
  if (!ok) w = failed_weight();
  return ok;
}

}  // namespace mg
