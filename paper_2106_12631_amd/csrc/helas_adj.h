// Reverse-mode (adjoint) versions of the routines of helas.h.
//
// Convention: for a real function L of complex values z, the adjoint is
// zb = dL/d(Re z) + i dL/d(Im z).  Then for w = f(z) holomorphic,
// zb += conj(f'(z)) wb, and for a real parameter t of w, tb += Re(conj(wb)
// dw/dt).  Every routine here takes the forward inputs and the adjoint of
// the output, and ADDS the adjoints of its inputs (wavefunctions, and the
// real momentum sums K whose derivative flows back to the external momenta)
// to the accumulators passed in.
//
// The K dependence of the currents enters through the propagator
// denominator and, for massive vectors, fermions and the three-gluon vertex,
// through the numerator.  The denominator term needs <wb, out> (sum of
// conj(wb) out over components); since every current is linear in each of
// its wavefunction inputs, <wb, out> equals <Xb, X> for the adjoint
// contribution Xb to any one input X, which is what the routines use
// instead of recomputing the output.
#pragma once
#include "helas.h"

namespace mg {

// sum_c conj(a_c) b_c over four components (no metric)
template <typename T>
__device__ __forceinline__ cx<T> cdot4(const cx<T> a[4], const cx<T> b[4]) {
  cx<T> s = conj(a[0]) * b[0];
#pragma unroll
  for (int c = 1; c < 4; ++c) s = s + conj(a[c]) * b[c];
  return s;
}
// Re(conj(a) b)
template <typename T>
__device__ __forceinline__ T redot(cx<T> a, cx<T> b) { return a.r * b.r + a.i * b.i; }

__device__ __forceinline__ constexpr double metric(int m) { return m == 0 ? 1.0 : -1.0; }

// bilinear J = F Gamma^mu (cL P_L + cR P_R) G (ffv_bilinear): from Jb add
// Fb and Gb
template <typename T>
__device__ __forceinline__ void adj_bilinear(const cx<T> F[4], const cx<T> G[4], base_t<T> cL,
                                             base_t<T> cR, const cx<T> Jb[4], cx<T> Fb[4],
                                             cx<T> Gb[4]) {
  const cx<T> ia = times_i(Jb[2]);
  const cx<T> a00 = cR * (Jb[0] + Jb[3]), a11 = cR * (Jb[0] - Jb[3]);
  const cx<T> a01 = cR * (Jb[1] + ia), a10 = cR * (Jb[1] - ia);
  const cx<T> b00 = cL * (Jb[0] - Jb[3]), b11 = cL * (Jb[0] + Jb[3]);
  const cx<T> b01 = -(cL * (Jb[1] + ia)), b10 = -(cL * (Jb[1] - ia));
  Fb[0] = Fb[0] + conj(G[2]) * a00 + conj(G[3]) * a01;
  Fb[1] = Fb[1] + conj(G[3]) * a11 + conj(G[2]) * a10;
  Fb[2] = Fb[2] + conj(G[0]) * b00 + conj(G[1]) * b01;
  Fb[3] = Fb[3] + conj(G[1]) * b11 + conj(G[0]) * b10;
  Gb[0] = Gb[0] + conj(F[2]) * b00 + conj(F[3]) * b10;
  Gb[1] = Gb[1] + conj(F[3]) * b11 + conj(F[2]) * b01;
  Gb[2] = Gb[2] + conj(F[0]) * a00 + conj(F[1]) * a10;
  Gb[3] = Gb[3] + conj(F[1]) * a11 + conj(F[0]) * a01;
}

// a = i mdot(B, V): add Bb and Vb
template <typename T>
__device__ __forceinline__ void adj_mdot_i(const cx<T> B[4], const cx<T> V[4], cx<T> ab,
                                           cx<T> Bb[4], cx<T> Vb[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T g = (T)metric(m);
    Bb[m] = Bb[m] - g * times_i(conj(V[m]) * ab);
    Vb[m] = Vb[m] - g * times_i(conj(B[m]) * ab);
  }
}

// amplitude a = i F V-slash (cL P_L + cR P_R) G (ffv_amp)
template <typename T>
__device__ __forceinline__ void adj_ffv_amp(const cx<T> F[4], const cx<T> V[4], const cx<T> G[4],
                                            base_t<T> cL, base_t<T> cR, cx<T> ab, cx<T> Fb[4],
                                            cx<T> Vb[4], cx<T> Gb[4]) {
  cx<T> J[4];
  ffv_bilinear(F, G, cL, cR, J);
  cx<T> Jb[4] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};
  adj_mdot_i(J, V, ab, Jb, Vb);
  adj_bilinear(F, G, cL, cR, Jb, Fb, Gb);
}

// d(K^2)/dK^mu = 2 g_mu K^mu: Kb += s * 2 g_mu K^mu
template <typename T, typename R>
__device__ __forceinline__ void add_msq_grad(const R K[4], T s, T Kb[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) Kb[m] += (T)(2.0 * metric(m)) * (T)K[m] * s;
}

// vector current through a massless propagator, out = J(F, G) / K^2
template <typename T, typename R>
__device__ __forceinline__ void adj_ffv_cur_v0(const cx<T> F[4], const cx<T> G[4], base_t<T> cL,
                                               base_t<T> cR, const R K[4], const cx<T> ob[4],
                                               cx<T> Fb[4], cx<T> Gb[4], T Kb[4]) {
  const R rkR = 1.0 / msq(K);
  const T rk = (T)rkR;
  cx<T> Jb[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) Jb[m] = rk * ob[m];
  cx<T> fl[4] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};
  adj_bilinear(F, G, cL, cR, Jb, fl, Gb);
  // <ob, out> = <fl, F>;  d(1/K^2) = -(1/K^2)^2 d(K^2)
  const T s = -rk * cdot4(fl, F).r;
  add_msq_grad(K, s, Kb);
#pragma unroll
  for (int m = 0; m < 4; ++m) Fb[m] = Fb[m] + fl[m];
}

// massive vector current, out = d (J - k (k.J)/M^2), d = 1/(K^2 - M^2 + i M W)
template <typename T, typename R>
__device__ __forceinline__ void adj_ffv_cur_vm(const cx<T> F[4], const cx<T> G[4], base_t<T> cL,
                                               base_t<T> cR, const R K[4], double mass,
                                               double width, const cx<T> ob[4], cx<T> Fb[4],
                                               cx<T> Gb[4], T Kb[4]) {
  cx<T> J[4];
  ffv_bilinear(F, G, cL, cR, J);
  T k[4];
  to_T(K, k);
  const T im2 = (T)(1.0 / (mass * mass));
  const cx<T> d = inv_den<T>(msq(K) - mass * mass, R(mass * width));
  const cx<T> kj = im2 * mdot(k, J);
  cx<T> ub[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) ub[m] = conj(d) * ob[m];
  // sum_rho k^rho ub^rho (no metric) and sum_rho conj(ub^rho) k^rho
  cx<T> kub = k[0] * ub[0];
#pragma unroll
  for (int m = 1; m < 4; ++m) kub = kub + k[m] * ub[m];
  cx<T> Jb[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) Jb[m] = ub[m] - ((T)metric(m) * im2 * k[m]) * kub;
  cx<T> fl[4] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};
  adj_bilinear(F, G, cL, cR, Jb, fl, Gb);
  // denominator: Kb^mu += -2 g_mu K^mu Re(d <ob, out>), <ob, out> = <fl, F>
  const T s = -(d * cdot4(fl, F)).r;
  add_msq_grad(K, s, Kb);
  // numerator: Kb^mu += -Re[conj(ub^mu) (k.J) + conj(kub) g_mu J^mu] / M^2
#pragma unroll
  for (int m = 0; m < 4; ++m)
    Kb[m] -= redot(ub[m], kj) + (T)metric(m) * im2 * redot(kub, J[m]);
#pragma unroll
  for (int m = 0; m < 4; ++m) Fb[m] = Fb[m] + fl[m];
}

// M^H x for a 2x2 block (column form) and x M^H (row form)
template <typename T>
__device__ __forceinline__ void mcolH(const blk<T>& m, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  y0 = conj(m.a) * x0 + conj(m.c) * x1;
  y1 = conj(m.b) * x0 + conj(m.d) * x1;
}
template <typename T>
__device__ __forceinline__ void mrowH(const blk<T>& m, cx<T> x0, cx<T> x1, cx<T>& y0, cx<T>& y1) {
  y0 = x0 * conj(m.a) + x1 * conj(m.b);
  y1 = x0 * conj(m.c) + x1 * conj(m.d);
}

// V-slash acting on (x0, x1) through the block pattern of s (upper) or sb
// (lower): adjoint with respect to V of y = sV x (sgn = -1) or sbV x
// (sgn = +1), column form, given yb: Vb += ...
template <typename T>
__device__ __forceinline__ void adj_slash_V_col(cx<T> x0, cx<T> x1, cx<T> yb0, cx<T> yb1, T sgn,
                                                cx<T> Vb[4]) {
  // sV  = [[V0 - V3, -(V1 - i V2)], [-(V1 + i V2), V0 + V3]]
  // sbV = [[V0 + V3,   V1 - i V2 ], [  V1 + i V2,  V0 - V3]]
  const cx<T> c0 = conj(x0), c1 = conj(x1);
  Vb[0] = Vb[0] + c0 * yb0 + c1 * yb1;
  Vb[3] = Vb[3] + sgn * (c0 * yb0 - c1 * yb1);
  Vb[1] = Vb[1] + sgn * (c1 * yb0 + c0 * yb1);
  Vb[2] = Vb[2] - sgn * times_i(c0 * yb1 - c1 * yb0);
}
// the same for the row form y = x sV (sgn = -1) or x sbV (sgn = +1)
template <typename T>
__device__ __forceinline__ void adj_slash_V_row(cx<T> x0, cx<T> x1, cx<T> yb0, cx<T> yb1, T sgn,
                                                cx<T> Vb[4]) {
  // (x M)_0 = x0 a + x1 c, (x M)_1 = x0 b + x1 d
  const cx<T> c0 = conj(x0), c1 = conj(x1);
  Vb[0] = Vb[0] + c0 * yb0 + c1 * yb1;
  Vb[3] = Vb[3] + sgn * (c0 * yb0 - c1 * yb1);
  Vb[1] = Vb[1] + sgn * (c1 * yb0 + c0 * yb1);
  Vb[2] = Vb[2] - sgn * times_i(c1 * yb0 - c0 * yb1);
}

// Kb from the numerator K-slash: column form, num_U = sK phiR, num_D = sbK phiL
// (times sign sg), with ob = conj(d) outb
template <typename T>
__device__ __forceinline__ void adj_kslash_col(cx<T> pR0, cx<T> pR1, cx<T> pL0, cx<T> pL1,
                                               cx<T> oU0, cx<T> oU1, cx<T> oD0, cx<T> oD1, T sg,
                                               T Kb[4]) {
  // sK = [[K0-K3, -K1+iK2], [-K1-iK2, K0+K3]], sbK = [[K0+K3, K1-iK2], [K1+iK2, K0-K3]]
  Kb[0] += sg * (redot(oU0, pR0) + redot(oU1, pR1) + redot(oD0, pL0) + redot(oD1, pL1));
  Kb[3] += sg * (-redot(oU0, pR0) + redot(oU1, pR1) + redot(oD0, pL0) - redot(oD1, pL1));
  Kb[1] += sg * (-redot(oU0, pR1) - redot(oU1, pR0) + redot(oD0, pL1) + redot(oD1, pL0));
  Kb[2] += sg * (redot(oU0, times_i(pR1)) - redot(oU1, times_i(pR0)) -
                 redot(oD0, times_i(pL1)) + redot(oD1, times_i(pL0)));
}

// flow-in fermion current (ffv_cur_fin): out = -(1/D) (K-slash + m) V-slash (cL P_L + cR P_R) G
template <typename T, typename R>
__device__ __forceinline__ void adj_ffv_cur_fin(const cx<T> V[4], const cx<T> G[4], base_t<T> cL,
                                                base_t<T> cR, const R K[4], double m, double w,
                                                const cx<T> ob[4], cx<T> Vb[4], cx<T> Gb[4],
                                                T Kb[4]) {
  blk<T> s, sb;
  slash_blocks(V, s, sb);
  const cx<T> g2 = cR * G[2], g3 = cR * G[3], g0 = cL * G[0], g1 = cL * G[1];
  cx<T> f0, f1, f2, f3;  // phiL = (f0, f1) = sV cR G_R, phiR = (f2, f3) = sbV cL G_L
  mcol(s, g2, g3, f0, f1);
  mcol(sb, g0, g1, f2, f3);
  T k[4];
  to_T(K, k);
  const T mm = (T)m;
  const cx<T> d = -inv_den<T>(msq(K) - m * m, R(m * w));
  const cx<T> o0 = conj(d) * ob[0], o1 = conj(d) * ob[1], o2 = conj(d) * ob[2],
              o3 = conj(d) * ob[3];
  // out_U = d (sK phiR + m phiL), out_D = d (sbK phiL + m phiR); sK, sbK Hermitian
  cx<T> pL0, pL1, pR0, pR1;
  sbK_col(k, o2, o3, pL0, pL1);
  sK_col(k, o0, o1, pR0, pR1);
  pL0 = pL0 + mm * o0; pL1 = pL1 + mm * o1;
  pR0 = pR0 + mm * o2; pR1 = pR1 + mm * o3;
  adj_kslash_col(f2, f3, f0, f1, o0, o1, o2, o3, (T)1, Kb);
  // phiL = sV (g2, g3), phiR = sbV (g0, g1)
  cx<T> gl[4];
  mcolH(s, pL0, pL1, gl[2], gl[3]);
  mcolH(sb, pR0, pR1, gl[0], gl[1]);
  gl[0] = cL * gl[0]; gl[1] = cL * gl[1]; gl[2] = cR * gl[2]; gl[3] = cR * gl[3];
  adj_slash_V_col(g2, g3, pL0, pL1, (T)-1, Vb);
  adj_slash_V_col(g0, g1, pR0, pR1, (T)1, Vb);
  // denominator: d(-1/D) = (1/D^2) dD = d^2 dD -> Kb += 2 g K Re(d <ob, out>)
  const T sden = (d * cdot4(gl, G)).r;
  add_msq_grad(K, sden, Kb);
#pragma unroll
  for (int c = 0; c < 4; ++c) Gb[c] = Gb[c] + gl[c];
}

// flow-out fermion current (ffv_cur_fout): out = -(1/D) F V-slash (cL P_L + cR P_R) (-K-slash + m)
template <typename T, typename R>
__device__ __forceinline__ void adj_ffv_cur_fout(const cx<T> F[4], const cx<T> V[4], base_t<T> cL,
                                                 base_t<T> cR, const R K[4], double m, double w,
                                                 const cx<T> ob[4], cx<T> Fb[4], cx<T> Vb[4],
                                                 T Kb[4]) {
  blk<T> s, sb;
  slash_blocks(V, s, sb);
  const cx<T> x0 = cL * F[2], x1 = cL * F[3], y0 = cR * F[0], y1 = cR * F[1];
  cx<T> f0, f1, f2, f3;  // phiL = (F_R sbV) cL, phiR = (F_L sV) cR
  mrow(sb, x0, x1, f0, f1);
  mrow(s, y0, y1, f2, f3);
  T k[4];
  to_T(K, k);
  const T mm = (T)m;
  const cx<T> d = -inv_den<T>(msq(K) - m * m, R(m * w));
  const cx<T> o0 = conj(d) * ob[0], o1 = conj(d) * ob[1], o2 = conj(d) * ob[2],
              o3 = conj(d) * ob[3];
  // out_U = d (m phiL - phiR sbK), out_D = d (-phiL sK + m phiR)
  cx<T> pL0, pL1, pR0, pR1;
  sK_row(k, o2, o3, pL0, pL1);
  sbK_row(k, o0, o1, pR0, pR1);
  pL0 = mm * o0 - pL0; pL1 = mm * o1 - pL1;
  pR0 = mm * o2 - pR0; pR1 = mm * o3 - pR1;
  // numerator: num_U = -(phiR sbK): the row products have the same K
  // derivatives as the column ones with the off-diagonal entries swapped
  Kb[0] -= redot(o0, f2) + redot(o1, f3) + redot(o2, f0) + redot(o3, f1);
  Kb[3] -= redot(o0, f2) - redot(o1, f3) - redot(o2, f0) + redot(o3, f1);
  Kb[1] -= redot(o0, f3) + redot(o1, f2) - redot(o2, f1) - redot(o3, f0);
  Kb[2] -= redot(o0, times_i(f3)) - redot(o1, times_i(f2)) - redot(o2, times_i(f1)) +
           redot(o3, times_i(f0));
  cx<T> fl[4];
  mrowH(sb, pL0, pL1, fl[2], fl[3]);
  mrowH(s, pR0, pR1, fl[0], fl[1]);
  fl[0] = cR * fl[0]; fl[1] = cR * fl[1]; fl[2] = cL * fl[2]; fl[3] = cL * fl[3];
  adj_slash_V_row(x0, x1, pL0, pL1, (T)1, Vb);
  adj_slash_V_row(y0, y1, pR0, pR1, (T)-1, Vb);
  const T sden = (d * cdot4(fl, F)).r;
  add_msq_grad(K, sden, Kb);
#pragma unroll
  for (int c = 0; c < 4; ++c) Fb[c] = Fb[c] + fl[c];
}

// u = A (B.C) for complex four-vectors (metric dot): given ub add Ab, Bb, Cb
template <typename T>
__device__ __forceinline__ void adj_vec_times_dot(const cx<T> A[4], const cx<T> B[4],
                                                  const cx<T> C[4], const cx<T> ub[4], T sign,
                                                  cx<T> Ab[4], cx<T> Bb[4], cx<T> Cb[4]) {
  const cx<T> bc = mdot(B, C);
  const cx<T> au = cdot4(A, ub);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T g = sign * (T)metric(m);
    Ab[m] = Ab[m] + sign * (conj(bc) * ub[m]);
    Bb[m] = Bb[m] + g * (conj(C[m]) * au);
    Cb[m] = Cb[m] + g * (conj(B[m]) * au);
  }
}

// three-gluon current (vvv_cur), out = (-i g / K^2) [A (qa.B) + dk (A.B) + B (qb.A)]
// with qa = -(2KA + KB), qb = KA + 2KB, dk = KA - KB, K = KA + KB
template <typename T, typename R>
__device__ __forceinline__ void adj_vvv_cur(const cx<T> A[4], const R KA[4], const cx<T> B[4],
                                            const R KB[4], base_t<T> g, const cx<T> ob[4],
                                            cx<T> Ab[4], T KAb[4], cx<T> Bb[4], T KBb[4]) {
  R K[4];
  T qa[4], qb[4], dk[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    qa[m] = (T)(-(2.0 * KA[m] + KB[m]));
    qb[m] = (T)(KA[m] + 2.0 * KB[m]);
    dk[m] = (T)(KA[m] - KB[m]);
    K[m] = KA[m] + KB[m];
  }
  const T rk = (T)(1.0 / msq(K));
  // ub = conj(pre) ob with pre = -i g / K^2
  cx<T> ub[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) ub[m] = (rk * g) * times_i(ob[m]);
  const cx<T> ca = mdot(qa, B), cb = mdot(qb, A), ab = mdot(A, B);
  const cx<T> Au = cdot4(A, ub), Bu = cdot4(B, ub);
  cx<T> dku = dk[0] * ub[0];
#pragma unroll
  for (int m = 1; m < 4; ++m) dku = dku + dk[m] * ub[m];
  cx<T> al[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T gm = (T)metric(m);
    al[m] = conj(ca) * ub[m] + gm * (conj(B[m]) * dku) + (gm * qb[m]) * Bu;
    Bb[m] = Bb[m] + conj(cb) * ub[m] + gm * (conj(A[m]) * dku) + (gm * qa[m]) * Au;
  }
  // momenta: qa, qb, dk in the numerator, 1/K^2 in the prefactor
  T qab[4], qbb[4], dkb[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const T gm = (T)metric(m);
    qab[m] = gm * redot(Au, B[m]);
    qbb[m] = gm * redot(Bu, A[m]);
    dkb[m] = redot(ub[m], ab);
  }
  const T sden = -rk * cdot4(al, A).r;
  T Kb[4] = {(T)0, (T)0, (T)0, (T)0};
  add_msq_grad(K, sden, Kb);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    KAb[m] += -2 * qab[m] + qbb[m] + dkb[m] + Kb[m];
    KBb[m] += -qab[m] + 2 * qbb[m] - dkb[m] + Kb[m];
    Ab[m] = Ab[m] + al[m];
  }
}

// four-gluon current (vvvv_cur), structure S, out = (-g^2/K^2) u with
//   S=1: u = Y (X.Z) - Z (X.Y)   S=2: u = X (Y.Z) - Z (X.Y)   S=3: u = X (Y.Z) - Y (X.Z)
template <int S, typename T, typename R>
__device__ __forceinline__ void adj_vvvv_cur(const cx<T> X[4], const cx<T> Y[4], const cx<T> Z[4],
                                             const R K[4], base_t<T> g2, const cx<T> ob[4],
                                             cx<T> Xb[4], cx<T> Yb[4], cx<T> Zb[4], T Kb[4]) {
  const T pre = (T)(-1.0 / msq(K)) * g2;
  cx<T> ub[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) ub[m] = pre * ob[m];
  cx<T> xl[4] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};
  if (S == 1) {
    adj_vec_times_dot(Y, X, Z, ub, (T)1, Yb, xl, Zb);
    adj_vec_times_dot(Z, X, Y, ub, (T)-1, Zb, xl, Yb);
  } else if (S == 2) {
    adj_vec_times_dot(X, Y, Z, ub, (T)1, xl, Yb, Zb);
    adj_vec_times_dot(Z, X, Y, ub, (T)-1, Zb, xl, Yb);
  } else {
    adj_vec_times_dot(X, Y, Z, ub, (T)1, xl, Yb, Zb);
    adj_vec_times_dot(Y, X, Z, ub, (T)-1, Yb, xl, Zb);
  }
  // <ob, out> = <xl, X>; d(-1/K^2) = (1/K^2)^2 d(K^2)
  const T s = -((T)(1.0 / msq(K))) * cdot4(xl, X).r;
  add_msq_grad(K, s, Kb);
#pragma unroll
  for (int m = 0; m < 4; ++m) Xb[m] = Xb[m] + xl[m];
}

// external wavefunctions: pb += Re sum_c conj(wb_c) dw_c/dp, from four
// forward-mode passes (one per momentum component) of the routine
template <typename T, typename F>
__device__ __forceinline__ void adj_ext_accum(const cx<dual<F>> w[4], const cx<T> wb[4], double& pbm) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += (double)wb[c].r * (double)w[c].r.d + (double)wb[c].i * (double)w[c].i.d;
  pbm += s;
}

template <typename T>
__device__ __forceinline__ void adj_ext_vector(const double p[4], int lam, bool conjugate,
                                               const cx<T> wb[4], double pb[4]) {
  using D = dual<double>;
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    D pd[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) pd[m] = D(p[m], m == mu ? 1.0 : 0.0);
    cx<dual<T>> w[4];
    ext_vector<dual<T>>(pd, lam, conjugate, w);
    adj_ext_accum(w, wb, pb[mu]);
  }
}

template <typename T>
__device__ __forceinline__ void adj_ext_u(const double p[4], double m, int lam, bool barred,
                                          const cx<T> wb[4], double pb[4]) {
  using D = dual<double>;
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    D pd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pd[k] = D(p[k], k == mu ? 1.0 : 0.0);
    cx<dual<T>> w[4];
    ext_u<dual<T>>(pd, m, lam, barred, w);
    adj_ext_accum(w, wb, pb[mu]);
  }
}

template <typename T>
__device__ __forceinline__ void adj_ext_v(const double p[4], double m, int lam, bool barred,
                                          const cx<T> wb[4], double pb[4]) {
  using D = dual<double>;
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    D pd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pd[k] = D(p[k], k == mu ? 1.0 : 0.0);
    cx<dual<T>> w[4];
    ext_v<dual<T>>(pd, m, lam, barred, w);
    adj_ext_accum(w, wb, pb[mu]);
  }
}

}  // namespace mg
