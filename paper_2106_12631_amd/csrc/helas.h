// Device routines of the helicity-amplitude method for gfx950.
//
// The paper computes each matrix element with three kinds of routines used
// in sequence (Sec. II, Fig. 1): "external particle" wavefunctions from a
// momentum and a helicity, "internal particle" off-shell currents at a
// vertex with one unknown leg, and "amplitude" routines at a vertex whose
// legs are all known.  These are written here from the Feynman rules in the
// chiral (Weyl) representation, where gamma^mu = [[0, s^mu], [sb^mu, 0]] with
// s^mu = (1, sigma), sb^mu = (1, -sigma), so that every gamma-matrix product
// reduces to 2x2 blocks:
//
//   spinor     (L0, L1, R0, R1): upper = left-handed
//   vertex     i gamma^mu (cL P_L + cR P_R)   (gluon: cL = cR = g_s, colour
//              factor T^a handled by the generated code)
//   g g g      g_s [g^{mu nu}(k1-k2)^rho + g^{nu rho}(k2-k3)^mu + g^{rho mu}(k3-k1)^nu]
//   g g g g    -i g_s^2 x one of three Lorentz structures (one per f f term)
//   propagators  vector -i g/K^2 (massless) or -i (g - K K/M^2)/(K^2 - M^2 + i M W),
//                fermion i (P-slash + m)/(P^2 - m^2 + i m w)
//
// Two scalar types: R for momenta (double, or dual<double> when the
// routines are differentiated in forward mode) and T for the amplitudes
// (double or float, or their duals).  Every momentum-only quantity -- square
// roots of the external momenta and the propagator denominators -- is
// formed in R and rounded to T afterwards.  Couplings are plain reals of the
// base type of T.
#pragma once
#include <hip/hip_runtime.h>

namespace mg {

// the dual-number overloads below must not hide the real ones
using ::fabs;
using ::log;
using ::sincos;
using ::sqrt;

// ---------------------------------------------------------------------------
// forward-mode dual numbers: value and one directional derivative
// ---------------------------------------------------------------------------
template <typename F>
struct dual {
  F v, d;
  dual() = default;
  __host__ __device__ constexpr dual(F value) : v(value), d(F(0)) {}
  __host__ __device__ constexpr dual(F value, F deriv) : v(value), d(deriv) {}
  template <typename G>
  __host__ __device__ explicit constexpr dual(const dual<G>& o) : v(F(o.v)), d(F(o.d)) {}
};

template <typename F>
__device__ __forceinline__ dual<F> operator+(dual<F> a, dual<F> b) { return {a.v + b.v, a.d + b.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator-(dual<F> a, dual<F> b) { return {a.v - b.v, a.d - b.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator-(dual<F> a) { return {-a.v, -a.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator*(dual<F> a, dual<F> b) {
  return {a.v * b.v, a.v * b.d + a.d * b.v};
}
template <typename F>
__device__ __forceinline__ dual<F> operator/(dual<F> a, dual<F> b) {
  const F q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <typename F>
__device__ __forceinline__ dual<F> operator+(dual<F> a, F b) { return {a.v + b, a.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator+(F a, dual<F> b) { return {a + b.v, b.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator-(dual<F> a, F b) { return {a.v - b, a.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator-(F a, dual<F> b) { return {a - b.v, -b.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator*(dual<F> a, F b) { return {a.v * b, a.d * b}; }
template <typename F>
__device__ __forceinline__ dual<F> operator*(F a, dual<F> b) { return {a * b.v, a * b.d}; }
template <typename F>
__device__ __forceinline__ dual<F> operator/(dual<F> a, F b) { return {a.v / b, a.d / b}; }
template <typename F>
__device__ __forceinline__ dual<F> operator/(F a, dual<F> b) {
  const F q = a / b.v;
  return {q, -q * b.d / b.v};
}
template <typename F>
__device__ __forceinline__ dual<F>& operator+=(dual<F>& a, dual<F> b) { return a = a + b; }
template <typename F>
__device__ __forceinline__ dual<F>& operator-=(dual<F>& a, dual<F> b) { return a = a - b; }
template <typename F>
__device__ __forceinline__ dual<F>& operator*=(dual<F>& a, dual<F> b) { return a = a * b; }
// sqrt with derivative 0 at exactly 0: only constant momenta (the incoming
// beams along the z axis) reach it, with a zero tangent.
template <typename F>
__device__ __forceinline__ dual<F> sqrt(dual<F> a) {
  const F r = sqrt(a.v);
  return {r, r > F(0) ? a.d / (F(2) * r) : F(0)};
}
template <typename F>
__device__ __forceinline__ dual<F> log(dual<F> a) { return {log(a.v), a.d / a.v}; }
template <typename F>
__device__ __forceinline__ dual<F> fabs(dual<F> a) { return a.v < F(0) ? -a : a; }
template <typename F>
__device__ __forceinline__ void sincos(dual<F> a, dual<F>* s, dual<F>* c) {
  F sv, cv;
  sincos(a.v, &sv, &cv);
  *s = {sv, cv * a.d};
  *c = {cv, -sv * a.d};
}

template <typename X>
struct base_of {
  using type = X;
};
template <typename F>
struct base_of<dual<F>> {
  using type = F;
};
template <typename X>
using base_t = typename base_of<X>::type;

__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ float val(float x) { return x; }
template <typename F>
__device__ __forceinline__ F val(dual<F> x) { return x.v; }

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
  T r, i;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <typename F>
__device__ __forceinline__ cx<dual<F>> operator*(F s, cx<dual<F>> a) { return {s * a.r, s * a.i}; }
template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }

// Fused forms: c + a b and c - a b as four fused multiply-adds (real T), so
// that sums of products do not round every product separately and take
// one instruction per term.  Dual numbers fall back to the operators.
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) { return a * b + c; }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T>
__device__ __forceinline__ cx<T> cmadd(cx<T> a, cx<T> b, cx<T> c) {
  return {fmadd(a.r, b.r, fmadd(-a.i, b.i, c.r)), fmadd(a.r, b.i, fmadd(a.i, b.r, c.i))};
}
template <typename T>
__device__ __forceinline__ cx<T> cmsub(cx<T> a, cx<T> b, cx<T> c) {
  return {fmadd(-a.r, b.r, fmadd(a.i, b.i, c.r)), fmadd(-a.r, b.i, fmadd(-a.i, b.r, c.i))};
}
// real scalar s: c + s a, c - s a
template <typename T>
__device__ __forceinline__ cx<T> rmadd(T s, cx<T> a, cx<T> c) {
  return {fmadd(s, a.r, c.r), fmadd(s, a.i, c.i)};
}
template <typename T>
__device__ __forceinline__ cx<T> rmsub(T s, cx<T> a, cx<T> c) {
  return {fmadd(-s, a.r, c.r), fmadd(-s, a.i, c.i)};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.r, -a.i}; }

// Reciprocal of a propagator denominator: the hardware estimate refined by
// two Newton steps r <- r + r (1 - x r), within an ulp or two of 1/x for the
// finite, non-zero, normal x that reach it (squared momentum sums minus
// squared masses).  Other real types (dual numbers) divide.
template <typename R>
__device__ __forceinline__ R recip(R x) { return R(1.0) / x; }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// 1 / (re + i im) formed in R, rounded to T
template <typename T, typename R>
__device__ __forceinline__ cx<T> inv_den(R re, R im) {
  const R n = recip(re * re + im * im);
  return cx<T>{(T)(re * n), (T)(-im * n)};
}

// Opaque copy: the compiler must assume the four components changed, so a
// wavefunction recomputed from it is not merged with an earlier computation.
// Components that are constants after inlining (the zero time component of
// a massless external vector, the zeros of a beam's wavefunction) stay
// visible: merging cannot happen through them, and the recomputation folds
// the products with them as the first computation did.
__device__ __forceinline__ void opaque(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(float& x) { asm volatile("" : "+v"(x)); }
template <typename F>
__device__ __forceinline__ void opaque(dual<F>& x) {
  opaque(x.v);
  opaque(x.d);
}
template <typename T>
__device__ __forceinline__ void opaque4(cx<T> (&w)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!__builtin_constant_p(w[k].r)) opaque(w[k].r);
    if (!__builtin_constant_p(w[k].i)) opaque(w[k].i);
  }
}

// Scheduling fence between groups of amplitude terms: the momenta are made
// opaque (so momentum sums of one group are not merged with identical ones
// of another group and kept live in between) and the machine scheduler may
// not move instructions across the fence.  The generated code orders its
// work to bound the number of live wavefunctions; the fence keeps that order.
// With UNI the momenta are the same in every lane of the wave (one event per
// wave) and stay in scalar registers.  With BEAM the two incoming momenta
// are (E,0,0,E) and (E,0,0,-E) with their zero components written as
// constants (set_beams in the kernels): they stay visible, so products with
// those zeros fold away in every group.
__device__ __forceinline__ void opaque_uniform(double& x) { asm volatile("" : "+s"(x)); }

template <bool UNI = false, bool BEAM = false, int N, typename R>
__device__ __forceinline__ void fence(R (&p)[N][4]) {
#pragma unroll
  for (int k = BEAM ? 2 : 0; k < N; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if constexpr (UNI) opaque_uniform(p[k][m]);
      else opaque(p[k][m]);
    }
  __builtin_amdgcn_sched_barrier(0);
}

// Colour-flow amplitude accumulation (the generated code's jamp += c amp)
template <typename T>
__device__ __forceinline__ void jacc(cx<T>& j, cx<T> v) { j = j + v; }

// ---------------------------------------------------------------------------
// external wavefunctions
// ---------------------------------------------------------------------------

// Polarisation vector eps^mu(p, lam) of a massless vector boson; conj = true
// gives eps* (outgoing).  eps = (-lam e1 - i e2)/sqrt2 with
// e1 = (0, cth cph, cth sph, -sth), e2 = (0, -sph, cph, 0); phi = 0 when pT = 0.
template <typename T, typename R>
__device__ __forceinline__ void ext_vector(const R p[4], int lam, bool conjugate, cx<T> w[4]) {
  const R kt2 = p[1] * p[1] + p[2] * p[2];
  const R K = sqrt(kt2 + p[3] * p[3]);
  const R kt = sqrt(kt2);
  const R iK = 1.0 / K;
  const R cth = p[3] * iK, sth = kt * iK;
  R cph = 1.0, sph = 0.0;
  if (val(kt) > 0.0) {
    const R ikt = 1.0 / kt;
    cph = p[1] * ikt;
    sph = p[2] * ikt;
  }
  const double r2 = 0.70710678118654752440;
  const double a = -lam * r2;             // coefficient of e1 (real part)
  const double b = conjugate ? r2 : -r2;  // coefficient of e2 (imaginary part)
  w[0] = cx<T>{(T)0.0, (T)0.0};
  w[1] = cx<T>{(T)(a * cth * cph), (T)(-b * sph)};
  w[2] = cx<T>{(T)(a * cth * sph), (T)(b * cph)};
  w[3] = cx<T>{(T)(-a * sth), (T)0.0};
}

// Two-component helicity state for the direction of p.  P + pz is formed as
// pT^2 / (P - pz) when pz < 0 to avoid cancellation; along -z the limit
// theta = pi, phi = 0 gives chi+ = (0, 1), chi- = (-1, 0).
template <typename R>
__device__ __forceinline__ void helicity_chi(const R p[4], int lam, R& c0r, R& c0i, R& c1r, R& c1i) {
  const R pt2 = p[1] * p[1] + p[2] * p[2];
  const R P = sqrt(pt2 + p[3] * p[3]);
  R ppz;
  if (val(p[3]) >= 0.0) {
    ppz = P + p[3];
  } else {
    const R d = P - p[3];
    ppz = val(d) > 0.0 ? pt2 / d : R(0.0);
  }
  if (!(val(ppz) > 0.0)) {  // along -z
    c0i = 0.0;
    c1i = 0.0;
    if (lam > 0) { c0r = 0.0; c1r = 1.0; }
    else { c0r = -1.0; c1r = 0.0; }
    return;
  }
  const R nrm = 1.0 / sqrt(2.0 * P * ppz);
  if (lam > 0) {  // (P + pz, px + i py) / nrm
    c0r = ppz * nrm; c0i = 0.0;
    c1r = p[1] * nrm; c1i = p[2] * nrm;
  } else {        // (-(px - i py), P + pz) / nrm
    c0r = -p[1] * nrm; c0i = p[2] * nrm;
    c1r = ppz * nrm; c1i = 0.0;
  }
}

// (sqrt(E - lam P), sqrt(E + lam P)); E - P = m^2 / (E + P), exactly 0 if m = 0
template <typename R>
__device__ __forceinline__ void omegas(const R p[4], double m, int lam, R& wm, R& wp) {
  const R P = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  const R epp = p[0] + P;
  const R emp = (m == 0.0) ? R(0.0) : m * m / epp;
  const R se = sqrt(emp), sp = sqrt(epp);
  if (lam > 0) { wm = se; wp = sp; } else { wm = sp; wp = se; }
}

// u(p, lam) = (sqrt(E - lam P) chi_lam, sqrt(E + lam P) chi_lam); bar = u^dagger gamma^0
template <typename T, typename R>
__device__ __forceinline__ void ext_u(const R p[4], double m, int lam, bool barred, cx<T> w[4]) {
  R wm, wp, c0r, c0i, c1r, c1i;
  omegas(p, m, lam, wm, wp);
  helicity_chi(p, lam, c0r, c0i, c1r, c1i);
  const double s = barred ? -1.0 : 1.0;  // conjugation flips the imaginary parts
  const cx<T> L0{(T)(wm * c0r), (T)(s * wm * c0i)}, L1{(T)(wm * c1r), (T)(s * wm * c1i)};
  const cx<T> R0{(T)(wp * c0r), (T)(s * wp * c0i)}, R1{(T)(wp * c1r), (T)(s * wp * c1i)};
  if (barred) { w[0] = R0; w[1] = R1; w[2] = L0; w[3] = L1; }  // gamma^0 swaps the blocks
  else { w[0] = L0; w[1] = L1; w[2] = R0; w[3] = R1; }
}

// v(p, lam) = (sqrt(E + lam P) chi_-lam, -sqrt(E - lam P) chi_-lam)
template <typename T, typename R>
__device__ __forceinline__ void ext_v(const R p[4], double m, int lam, bool barred, cx<T> w[4]) {
  R wm, wp, c0r, c0i, c1r, c1i;
  omegas(p, m, lam, wm, wp);
  helicity_chi(p, -lam, c0r, c0i, c1r, c1i);
  const double s = barred ? -1.0 : 1.0;
  const cx<T> L0{(T)(wp * c0r), (T)(s * wp * c0i)}, L1{(T)(wp * c1r), (T)(s * wp * c1i)};
  const cx<T> R0{(T)(-wm * c0r), (T)(-s * wm * c0i)}, R1{(T)(-wm * c1r), (T)(-s * wm * c1i)};
  if (barred) { w[0] = R0; w[1] = R1; w[2] = L0; w[3] = L1; }
  else { w[0] = L0; w[1] = L1; w[2] = R0; w[3] = R1; }
}

// ---------------------------------------------------------------------------
// 2x2 blocks of V-slash for a complex vector V (contravariant components)
//   sV  = s^mu V_mu  = [[V0 - V3, -(V1 - i V2)], [-(V1 + i V2), V0 + V3]]
//   sbV = sb^mu V_mu = [[V0 + V3,   V1 - i V2 ], [  V1 + i V2,  V0 - V3]]
// ---------------------------------------------------------------------------
template <typename T>
struct blk {
  cx<T> a, b, c, d;  // [[a, b], [c, d]]
};

template <typename T>
__device__ __forceinline__ void slash_blocks(const cx<T> V[4], blk<T>& s, blk<T>& sb) {
  const cx<T> v0p3 = V[0] + V[3], v0m3 = V[0] - V[3];
  const cx<T> v1mi2 = V[1] - times_i(V[2]), v1pi2 = V[1] + times_i(V[2]);
  s = blk<T>{v0m3, -v1mi2, -v1pi2, v0p3};
  sb = blk<T>{v0p3, v1mi2, v1pi2, v0m3};
}

// column: M x
template <typename T>
__device__ __forceinline__ void mcol(const blk<T>& m, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  y0 = cmadd(m.b, x1, m.a * x0);
  y1 = cmadd(m.d, x1, m.c * x0);
}
// row: x M
template <typename T>
__device__ __forceinline__ void mrow(const blk<T>& m, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  y0 = cmadd(x1, m.c, x0 * m.a);
  y1 = cmadd(x1, m.d, x0 * m.b);
}

// column: (s.K) x with s.K = [[K0-K3, -(K1 - i K2)], [-(K1 + i K2), K0+K3]]
template <typename T>
__device__ __forceinline__ void sK_col(const T K[4], cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> m01{-K[1], K[2]}, m10{-K[1], -K[2]};
  y0 = cmadd(m01, x1, (K[0] - K[3]) * x0);
  y1 = cmadd(m10, x0, (K[0] + K[3]) * x1);
}
// column: (sb.K) x with sb.K = [[K0+K3, K1 - i K2], [K1 + i K2, K0-K3]]
template <typename T>
__device__ __forceinline__ void sbK_col(const T K[4], cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> m01{K[1], -K[2]}, m10{K[1], K[2]};
  y0 = cmadd(m01, x1, (K[0] + K[3]) * x0);
  y1 = cmadd(m10, x0, (K[0] - K[3]) * x1);
}
// row: x (s.K)
template <typename T>
__device__ __forceinline__ void sK_row(const T K[4], cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> m01{-K[1], K[2]}, m10{-K[1], -K[2]};
  y0 = cmadd(x1, m10, (K[0] - K[3]) * x0);
  y1 = cmadd(x0, m01, (K[0] + K[3]) * x1);
}
// row: x (sb.K)
template <typename T>
__device__ __forceinline__ void sbK_row(const T K[4], cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  const cx<T> m01{K[1], -K[2]}, m10{K[1], K[2]};
  y0 = cmadd(x1, m10, (K[0] + K[3]) * x0);
  y1 = cmadd(x0, m01, (K[0] - K[3]) * x1);
}

template <typename T, typename R>
__device__ __forceinline__ void to_T(const R K[4], T k[4]) {
  k[0] = (T)K[0]; k[1] = (T)K[1]; k[2] = (T)K[2]; k[3] = (T)K[3];
}

template <typename R>
__device__ __forceinline__ R msq(const R K[4]) {
  return K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3];
}

template <typename T>
__device__ __forceinline__ cx<T> mdot(const cx<T> a[4], const cx<T> b[4]) {
  return cmsub(a[3], b[3], cmsub(a[2], b[2], cmsub(a[1], b[1], a[0] * b[0])));
}
template <typename T>
__device__ __forceinline__ cx<T> mdot(const T k[4], const cx<T> b[4]) {
  return rmsub(k[3], b[3], rmsub(k[2], b[2], rmsub(k[1], b[1], k[0] * b[0])));
}

// ---------------------------------------------------------------------------
// f f V : amplitude, vector current, flow-in and flow-out fermion currents
// ---------------------------------------------------------------------------

// bilinear J^mu = F gamma^mu (cL P_L + cR P_R) G for row F, column G
template <typename T>
__device__ __forceinline__ void ffv_bilinear(const cx<T> F[4], const cx<T> G[4], base_t<T> cL,
                                             base_t<T> cR, cx<T> J[4]) {
  // a = F_L s^mu G_R, b = F_R sb^mu G_L (sb^mu = (1, -sigma))
  const cx<T> a00 = F[0] * G[2], a11 = F[1] * G[3], a01 = F[0] * G[3], a10 = F[1] * G[2];
  const cx<T> b00 = F[2] * G[0], b11 = F[3] * G[1], b01 = F[2] * G[1], b10 = F[3] * G[0];
  // s^mu bilinear x^T s^mu y: (x0y0 + x1y1, x0y1 + x1y0, i(x1y0 - x0y1), x0y0 - x1y1)
  J[0] = cR * (a00 + a11) + cL * (b00 + b11);
  J[1] = cR * (a01 + a10) - cL * (b01 + b10);
  J[2] = cR * times_i(a10 - a01) - cL * times_i(b10 - b01);
  J[3] = cR * (a00 - a11) - cL * (b00 - b11);
}

// amplitude i F V-slash (cL P_L + cR P_R) G
template <typename T>
__device__ __forceinline__ cx<T> ffv_amp(const cx<T> F[4], const cx<T> V[4], const cx<T> G[4],
                                         base_t<T> cL, base_t<T> cR) {
  cx<T> J[4];
  ffv_bilinear(F, G, cL, cR, J);
  return times_i(mdot(J, V));
}

// Vector-like vertices (cL = cR = g: gluon, photon).  The bilinear without
// the coupling, F gamma^mu G, and the amplitude with g applied once to the
// result instead of to every component.
template <typename T>
__device__ __forceinline__ void ffv_bilinear_v(const cx<T> F[4], const cx<T> G[4], cx<T> J[4]) {
  const cx<T> a00 = F[0] * G[2], a11 = F[1] * G[3], a01 = F[0] * G[3], a10 = F[1] * G[2];
  const cx<T> b00 = F[2] * G[0], b11 = F[3] * G[1], b01 = F[2] * G[1], b10 = F[3] * G[0];
  J[0] = (a00 + a11) + (b00 + b11);
  J[1] = (a01 + a10) - (b01 + b10);
  J[2] = times_i((a10 - a01) - (b10 - b01));
  J[3] = (a00 - a11) - (b00 - b11);
}

template <typename T>
__device__ __forceinline__ cx<T> ffv_amp_v(const cx<T> F[4], const cx<T> V[4], const cx<T> G[4],
                                           base_t<T> g) {
  cx<T> J[4];
  ffv_bilinear_v(F, G, J);
  return g * times_i(mdot(J, V));
}

// vector current from F, G through a massless (photon, gluon) propagator:
// (-i/K^2) i J^mu = J^mu / K^2
template <typename T, typename R>
__device__ __forceinline__ void ffv_cur_v0(const cx<T> F[4], const cx<T> G[4], base_t<T> cL,
                                           base_t<T> cR, const R K[4], cx<T> out[4]) {
  cx<T> J[4];
  ffv_bilinear(F, G, cL, cR, J);
  const T rk = (T)recip(msq(K));
  for (int m = 0; m < 4; ++m) out[m] = rk * J[m];
}

// vector current through a massive propagator in unitary gauge:
// (J - K (K.J)/M^2) / (K^2 - M^2 + i M W)
template <typename T, typename R>
__device__ __forceinline__ void ffv_cur_vm(const cx<T> F[4], const cx<T> G[4], base_t<T> cL,
                                           base_t<T> cR, const R K[4], double mass, double width,
                                           cx<T> out[4]) {
  cx<T> J[4];
  ffv_bilinear(F, G, cL, cR, J);
  T k[4];
  to_T(K, k);
  const cx<T> kj = (T)recip(mass * mass) * mdot(k, J);
  const cx<T> d = inv_den<T>(msq(K) - mass * mass, R(mass * width));
  for (int m = 0; m < 4; ++m) out[m] = d * rmsub(k[m], kj, J[m]);
}

// flow-in fermion current: i(K-slash + m)/D * i V-slash (cL P_L + cR P_R) G
template <typename T, typename R>
__device__ __forceinline__ void ffv_cur_fin(const cx<T> V[4], const cx<T> G[4], base_t<T> cL,
                                            base_t<T> cR, const R K[4], double m, double w,
                                            cx<T> out[4]) {
  blk<T> s, sb;
  slash_blocks(V, s, sb);
  // phi = V-slash (cL G_L, cR G_R) = (sV cR G_R, sbV cL G_L)
  cx<T> f0, f1, f2, f3;
  mcol(s, cR * G[2], cR * G[3], f0, f1);
  mcol(sb, cL * G[0], cL * G[1], f2, f3);
  // (K-slash + m) phi = (sK phi_R + m phi_L, sbK phi_L + m phi_R)
  T k[4];
  to_T(K, k);
  const T mm = (T)m;
  cx<T> y0, y1, y2, y3;
  sK_col(k, f2, f3, y0, y1);
  sbK_col(k, f0, f1, y2, y3);
  const cx<T> d = -inv_den<T>(msq(K) - m * m, R(m * w));  // i * i = -1
  out[0] = d * rmadd(mm, f0, y0);
  out[1] = d * rmadd(mm, f1, y1);
  out[2] = d * rmadd(mm, f2, y2);
  out[3] = d * rmadd(mm, f3, y3);
}

// flow-out fermion current: F i V-slash (cL P_L + cR P_R) * i(-K-slash + m)/D
template <typename T, typename R>
__device__ __forceinline__ void ffv_cur_fout(const cx<T> F[4], const cx<T> V[4], base_t<T> cL,
                                             base_t<T> cR, const R K[4], double m, double w,
                                             cx<T> out[4]) {
  blk<T> s, sb;
  slash_blocks(V, s, sb);
  // row phi = F [[0, sV cR], [sbV cL, 0]] = (F_R sbV cL, F_L sV cR)
  cx<T> f0, f1, f2, f3;
  mrow(sb, F[2], F[3], f0, f1);
  mrow(s, F[0], F[1], f2, f3);
  f0 = cL * f0; f1 = cL * f1; f2 = cR * f2; f3 = cR * f3;
  // phi (-K-slash + m) = (m phi_L - phi_R sbK, -phi_L sK + m phi_R)
  T k[4];
  to_T(K, k);
  const T mm = (T)m;
  cx<T> y0, y1, y2, y3;
  sbK_row(k, f2, f3, y0, y1);
  sK_row(k, f0, f1, y2, y3);
  const cx<T> d = -inv_den<T>(msq(K) - m * m, R(m * w));
  out[0] = d * rmadd(mm, f0, -y0);
  out[1] = d * rmadd(mm, f1, -y1);
  out[2] = d * rmadd(mm, f2, -y2);
  out[3] = d * rmadd(mm, f3, -y3);
}

// ffv_cur_fin and ffv_cur_fout for a vector-like vertex (cL = cR = g): the
// coupling joins the propagator factor instead of every component
template <typename T, typename R>
__device__ __forceinline__ void ffv_cur_fin_v(const cx<T> V[4], const cx<T> G[4], base_t<T> g,
                                              const R K[4], double m, double w, cx<T> out[4]) {
  blk<T> s, sb;
  slash_blocks(V, s, sb);
  cx<T> f0, f1, f2, f3;
  mcol(s, G[2], G[3], f0, f1);
  mcol(sb, G[0], G[1], f2, f3);
  T k[4];
  to_T(K, k);
  const T mm = (T)m;
  cx<T> y0, y1, y2, y3;
  sK_col(k, f2, f3, y0, y1);
  sbK_col(k, f0, f1, y2, y3);
  const cx<T> d = -g * inv_den<T>(msq(K) - m * m, R(m * w));
  out[0] = d * rmadd(mm, f0, y0);
  out[1] = d * rmadd(mm, f1, y1);
  out[2] = d * rmadd(mm, f2, y2);
  out[3] = d * rmadd(mm, f3, y3);
}

template <typename T, typename R>
__device__ __forceinline__ void ffv_cur_fout_v(const cx<T> F[4], const cx<T> V[4], base_t<T> g,
                                               const R K[4], double m, double w, cx<T> out[4]) {
  blk<T> s, sb;
  slash_blocks(V, s, sb);
  cx<T> f0, f1, f2, f3;
  mrow(sb, F[2], F[3], f0, f1);
  mrow(s, F[0], F[1], f2, f3);
  T k[4];
  to_T(K, k);
  const T mm = (T)m;
  cx<T> y0, y1, y2, y3;
  sbK_row(k, f2, f3, y0, y1);
  sK_row(k, f0, f1, y2, y3);
  const cx<T> d = -g * inv_den<T>(msq(K) - m * m, R(m * w));
  out[0] = d * rmadd(mm, f0, -y0);
  out[1] = d * rmadd(mm, f1, -y1);
  out[2] = d * rmadd(mm, f2, -y2);
  out[3] = d * rmadd(mm, f3, -y3);
}

// ---------------------------------------------------------------------------
// gluon self-couplings (colour handled by the generated code)
// ---------------------------------------------------------------------------

// three-gluon current with legs (out, A, B), colour f^{out A B}:
// (-i/K^2) g [A (-(2kA + kB).B) + (A.B)(kA - kB) + B ((kA + 2kB).A)]
template <typename T, typename R>
__device__ __forceinline__ void vvv_cur(const cx<T> A[4], const R KA[4], const cx<T> B[4],
                                        const R KB[4], base_t<T> g, cx<T> out[4]) {
  R qa[4], qb[4], dk[4], K[4];
  for (int m = 0; m < 4; ++m) {
    qa[m] = -(2.0 * KA[m] + KB[m]);
    qb[m] = KA[m] + 2.0 * KB[m];
    dk[m] = KA[m] - KB[m];
    K[m] = KA[m] + KB[m];
  }
  T tqa[4], tqb[4], tdk[4];
  to_T(qa, tqa);
  to_T(qb, tqb);
  to_T(dk, tdk);
  const cx<T> ca = mdot(tqa, B), cb = mdot(tqb, A), ab = mdot(A, B);
  // (-i g / K^2) [...]
  const T pim = (T)(-recip(msq(K))) * g;
  for (int m = 0; m < 4; ++m) out[m] = pim * times_i(rmadd(tdk[m], ab, cmadd(B[m], cb, A[m] * ca)));
}

// four-gluon current, structure s (1, 2, 3), legs (out, X, Y, Z):
//   s=1: Y (X.Z) - Z (X.Y)   s=2: X (Y.Z) - Z (X.Y)   s=3: X (Y.Z) - Y (X.Z)
// times (-i g^2)(-i/K^2) = -g^2/K^2
template <int S, typename T, typename R>
__device__ __forceinline__ void vvvv_cur(const cx<T> X[4], const cx<T> Y[4], const cx<T> Z[4],
                                         const R K[4], base_t<T> g2, cx<T> out[4]) {
  const T pre = (T)(-recip(msq(K))) * g2;
  if (S == 1) {
    const cx<T> xz = pre * mdot(X, Z), xy = pre * mdot(X, Y);
    for (int m = 0; m < 4; ++m) out[m] = cmsub(Z[m], xy, Y[m] * xz);
  } else if (S == 2) {
    const cx<T> yz = pre * mdot(Y, Z), xy = pre * mdot(X, Y);
    for (int m = 0; m < 4; ++m) out[m] = cmsub(Z[m], xy, X[m] * yz);
  } else {
    const cx<T> yz = pre * mdot(Y, Z), xz = pre * mdot(X, Z);
    for (int m = 0; m < 4; ++m) out[m] = cmsub(Y[m], xz, X[m] * yz);
  }
}

}  // namespace mg
