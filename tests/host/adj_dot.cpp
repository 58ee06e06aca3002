// Dot-product tests of the hand-written reverse-mode HELAS routines
// (helas_adj.h), compiled for the host by test_helas_adjoint_host.py.
//
// For a routine out = f(x) and any output adjoint ob, the reverse routine
// returns xb with  Re<ob, df/dx . dx> = Re<xb, dx>  for every tangent dx
// (<a, b> = sum conj(a) b; real momenta K pair with plain products).  The
// left side comes from the forward routine of helas.h instantiated with
// forward-mode dual numbers (the tangent carried by every input), the right
// side from the adjoint routine, so a wrong term or sign in either shows up
// as a mismatch.  The external wavefunction adjoints are checked against
// fourth-order central differences of the plain forward routine instead.
//
// Prints one line per routine: name, number of random trials, max relative
// mismatch |lhs - rhs| / (|lhs| + |rhs| + tiny).
#include <cstdio>
#include <cmath>
#include <random>

#include "helas_adj.h"

using namespace mg;
using D = dual<double>;
using C = cx<double>;
using CD = cx<D>;

static std::mt19937_64 rng(20240917);
static double U(double a = -1.0, double b = 1.0) {
  return std::uniform_real_distribution<double>(a, b)(rng);
}
static C rc() { return C{U(), U()}; }
static void rvec(C v[4]) {
  for (int k = 0; k < 4; ++k) v[k] = rc();
}
// momentum sum with K^2 well away from the pole of any propagator
static void rmom(double K[4]) {
  for (;;) {
    for (int k = 1; k < 4; ++k) K[k] = U(-300.0, 300.0);
    K[0] = U(-800.0, 800.0);
    const double m2 = K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3];
    if (std::fabs(m2) > 2.0e4 && std::fabs(m2 - 173.0 * 173.0) > 2.0e4 &&
        std::fabs(m2 - 91.188 * 91.188) > 2.0e4)
      return;
  }
}
static void tie(const C x[4], const C dx[4], CD out[4]) {
  for (int k = 0; k < 4; ++k) out[k] = CD{D(x[k].r, dx[k].r), D(x[k].i, dx[k].i)};
}
static void tieK(const double K[4], const double dK[4], D out[4]) {
  for (int k = 0; k < 4; ++k) out[k] = D(K[k], dK[k]);
}
// Re<a, b> over four components
static double re4(const C a[4], const C b[4]) {
  double s = 0;
  for (int k = 0; k < 4; ++k) s += a[k].r * b[k].r + a[k].i * b[k].i;
  return s;
}
static double re4d(const C ob[4], const CD out[4]) {
  double s = 0;
  for (int k = 0; k < 4; ++k) s += ob[k].r * out[k].r.d + ob[k].i * out[k].i.d;
  return s;
}
static double kdot(const double a[4], const double b[4]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}
static void zero(C v[4]) {
  for (int k = 0; k < 4; ++k) v[k] = C{0, 0};
}
static double mism(double a, double b) { return std::fabs(a - b) / (std::fabs(a) + std::fabs(b) + 1e-300); }

struct Report {
  const char* name;
  int n = 0;
  double worst = 0;
  void add(double lhs, double rhs) {
    ++n;
    worst = std::fmax(worst, mism(lhs, rhs));
  }
  ~Report() { std::printf("%s %d %.3e\n", name, n, worst); }
};

static const int NTRIAL = 200;
static const double CL = -0.37, CR = 0.81, G = 1.21;

static void test_bilinear() {
  Report r{"adj_bilinear"};
  for (int t = 0; t < NTRIAL; ++t) {
    C F[4], G_[4], dF[4], dG[4], Jb[4];
    rvec(F); rvec(G_); rvec(dF); rvec(dG); rvec(Jb);
    CD Fd[4], Gd[4], J[4];
    tie(F, dF, Fd); tie(G_, dG, Gd);
    ffv_bilinear<D>(Fd, Gd, CL, CR, J);
    C Fb[4], Gb[4];
    zero(Fb); zero(Gb);
    adj_bilinear<double>(F, G_, CL, CR, Jb, Fb, Gb);
    r.add(re4d(Jb, J), re4(Fb, dF) + re4(Gb, dG));
  }
}

static void test_mdot_i() {
  Report r{"adj_mdot_i"};
  for (int t = 0; t < NTRIAL; ++t) {
    C B[4], V[4], dB[4], dV[4];
    rvec(B); rvec(V); rvec(dB); rvec(dV);
    const C ab = rc();
    CD Bd[4], Vd[4];
    tie(B, dB, Bd); tie(V, dV, Vd);
    const CD a = times_i(mdot(Bd, Vd));
    C Bb[4], Vb[4];
    zero(Bb); zero(Vb);
    adj_mdot_i<double>(B, V, ab, Bb, Vb);
    r.add(ab.r * a.r.d + ab.i * a.i.d, re4(Bb, dB) + re4(Vb, dV));
  }
}

static void test_ffv_amp() {
  Report r{"adj_ffv_amp"};
  for (int t = 0; t < NTRIAL; ++t) {
    C F[4], V[4], G_[4], dF[4], dV[4], dG[4];
    rvec(F); rvec(V); rvec(G_); rvec(dF); rvec(dV); rvec(dG);
    const C ab = rc();
    CD Fd[4], Vd[4], Gd[4];
    tie(F, dF, Fd); tie(V, dV, Vd); tie(G_, dG, Gd);
    const CD a = ffv_amp<D>(Fd, Vd, Gd, CL, CR);
    C Fb[4], Vb[4], Gb[4];
    zero(Fb); zero(Vb); zero(Gb);
    adj_ffv_amp<double>(F, V, G_, CL, CR, ab, Fb, Vb, Gb);
    r.add(ab.r * a.r.d + ab.i * a.i.d, re4(Fb, dF) + re4(Vb, dV) + re4(Gb, dG));
  }
}

static void test_cur_v0() {
  Report r{"adj_ffv_cur_v0"};
  for (int t = 0; t < NTRIAL; ++t) {
    C F[4], G_[4], dF[4], dG[4], ob[4];
    double K[4], dK[4];
    rvec(F); rvec(G_); rvec(dF); rvec(dG); rvec(ob); rmom(K);
    for (int k = 0; k < 4; ++k) dK[k] = U();
    CD Fd[4], Gd[4], out[4];
    D Kd[4];
    tie(F, dF, Fd); tie(G_, dG, Gd); tieK(K, dK, Kd);
    ffv_cur_v0<D, D>(Fd, Gd, CL, CR, Kd, out);
    C Fb[4], Gb[4];
    double Kb[4] = {0, 0, 0, 0};
    zero(Fb); zero(Gb);
    adj_ffv_cur_v0<double, double>(F, G_, CL, CR, K, ob, Fb, Gb, Kb);
    r.add(re4d(ob, out), re4(Fb, dF) + re4(Gb, dG) + kdot(Kb, dK));
  }
}

static void test_cur_vm() {
  Report r{"adj_ffv_cur_vm"};
  for (int t = 0; t < NTRIAL; ++t) {
    C F[4], G_[4], dF[4], dG[4], ob[4];
    double K[4], dK[4];
    rvec(F); rvec(G_); rvec(dF); rvec(dG); rvec(ob); rmom(K);
    for (int k = 0; k < 4; ++k) dK[k] = U();
    CD Fd[4], Gd[4], out[4];
    D Kd[4];
    tie(F, dF, Fd); tie(G_, dG, Gd); tieK(K, dK, Kd);
    ffv_cur_vm<D, D>(Fd, Gd, CL, CR, Kd, 91.188, 2.441, out);
    C Fb[4], Gb[4];
    double Kb[4] = {0, 0, 0, 0};
    zero(Fb); zero(Gb);
    adj_ffv_cur_vm<double, double>(F, G_, CL, CR, K, 91.188, 2.441, ob, Fb, Gb, Kb);
    r.add(re4d(ob, out), re4(Fb, dF) + re4(Gb, dG) + kdot(Kb, dK));
  }
}

static void test_cur_fin(double m, double w) {
  Report r{m > 0 ? "adj_ffv_cur_fin(massive)" : "adj_ffv_cur_fin(massless)"};
  for (int t = 0; t < NTRIAL; ++t) {
    C V[4], G_[4], dV[4], dG[4], ob[4];
    double K[4], dK[4];
    rvec(V); rvec(G_); rvec(dV); rvec(dG); rvec(ob); rmom(K);
    for (int k = 0; k < 4; ++k) dK[k] = U();
    CD Vd[4], Gd[4], out[4];
    D Kd[4];
    tie(V, dV, Vd); tie(G_, dG, Gd); tieK(K, dK, Kd);
    ffv_cur_fin<D, D>(Vd, Gd, CL, CR, Kd, m, w, out);
    C Vb[4], Gb[4];
    double Kb[4] = {0, 0, 0, 0};
    zero(Vb); zero(Gb);
    adj_ffv_cur_fin<double, double>(V, G_, CL, CR, K, m, w, ob, Vb, Gb, Kb);
    r.add(re4d(ob, out), re4(Vb, dV) + re4(Gb, dG) + kdot(Kb, dK));
  }
}

static void test_cur_fout(double m, double w) {
  Report r{m > 0 ? "adj_ffv_cur_fout(massive)" : "adj_ffv_cur_fout(massless)"};
  for (int t = 0; t < NTRIAL; ++t) {
    C F[4], V[4], dF[4], dV[4], ob[4];
    double K[4], dK[4];
    rvec(F); rvec(V); rvec(dF); rvec(dV); rvec(ob); rmom(K);
    for (int k = 0; k < 4; ++k) dK[k] = U();
    CD Fd[4], Vd[4], out[4];
    D Kd[4];
    tie(F, dF, Fd); tie(V, dV, Vd); tieK(K, dK, Kd);
    ffv_cur_fout<D, D>(Fd, Vd, CL, CR, Kd, m, w, out);
    C Fb[4], Vb[4];
    double Kb[4] = {0, 0, 0, 0};
    zero(Fb); zero(Vb);
    adj_ffv_cur_fout<double, double>(F, V, CL, CR, K, m, w, ob, Fb, Vb, Kb);
    r.add(re4d(ob, out), re4(Fb, dF) + re4(Vb, dV) + kdot(Kb, dK));
  }
}

static void test_vvv() {
  Report r{"adj_vvv_cur"};
  for (int t = 0; t < NTRIAL; ++t) {
    C A_[4], B[4], dA[4], dB[4], ob[4];
    double KA[4], KB[4], dKA[4], dKB[4];
    rvec(A_); rvec(B); rvec(dA); rvec(dB); rvec(ob);
    for (;;) {  // K = KA + KB away from zero
      for (int k = 0; k < 4; ++k) { KA[k] = U(-400, 400); KB[k] = U(-400, 400); }
      double K[4];
      for (int k = 0; k < 4; ++k) K[k] = KA[k] + KB[k];
      if (std::fabs(K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3]) > 2.0e4) break;
    }
    for (int k = 0; k < 4; ++k) { dKA[k] = U(); dKB[k] = U(); }
    CD Ad[4], Bd[4], out[4];
    D KAd[4], KBd[4];
    tie(A_, dA, Ad); tie(B, dB, Bd); tieK(KA, dKA, KAd); tieK(KB, dKB, KBd);
    vvv_cur<D, D>(Ad, KAd, Bd, KBd, G, out);
    C Ab[4], Bb[4];
    double KAb[4] = {0, 0, 0, 0}, KBb[4] = {0, 0, 0, 0};
    zero(Ab); zero(Bb);
    adj_vvv_cur<double, double>(A_, KA, B, KB, G, ob, Ab, KAb, Bb, KBb);
    r.add(re4d(ob, out), re4(Ab, dA) + re4(Bb, dB) + kdot(KAb, dKA) + kdot(KBb, dKB));
  }
}

template <int S>
static void test_vvvv(const char* name) {
  Report r{name};
  for (int t = 0; t < NTRIAL; ++t) {
    C X[4], Y[4], Z[4], dX[4], dY[4], dZ[4], ob[4];
    double K[4], dK[4];
    rvec(X); rvec(Y); rvec(Z); rvec(dX); rvec(dY); rvec(dZ); rvec(ob); rmom(K);
    for (int k = 0; k < 4; ++k) dK[k] = U();
    CD Xd[4], Yd[4], Zd[4], out[4];
    D Kd[4];
    tie(X, dX, Xd); tie(Y, dY, Yd); tie(Z, dZ, Zd); tieK(K, dK, Kd);
    vvvv_cur<S, D, D>(Xd, Yd, Zd, Kd, G * G, out);
    C Xb[4], Yb[4], Zb[4];
    double Kb[4] = {0, 0, 0, 0};
    zero(Xb); zero(Yb); zero(Zb);
    adj_vvvv_cur<S, double, double>(X, Y, Z, K, G * G, ob, Xb, Yb, Zb, Kb);
    r.add(re4d(ob, out), re4(Xb, dX) + re4(Yb, dY) + re4(Zb, dZ) + kdot(Kb, dK));
  }
}

// external wavefunctions: adjoint against central differences of the
// plain forward routine (fourth-order stencil in a relative step)
template <class Fwd, class Adj>
static void test_ext(const char* name, double m, Fwd fwd, Adj adj) {
  Report r{name};
  for (int t = 0; t < NTRIAL; ++t) {
    double p[4];
    const double P = U(20.0, 700.0);
    const double c = U(-0.999, 0.999), ph = U(0.0, 6.283185307179586);
    const double s = std::sqrt(1 - c * c);
    p[1] = P * s * std::cos(ph);
    p[2] = P * s * std::sin(ph);
    p[3] = P * c;
    p[0] = std::sqrt(P * P + m * m);
    double dp[4];
    for (int k = 0; k < 4; ++k) dp[k] = U();
    const int lam = (t & 1) ? 1 : -1;
    const bool flag = (t & 2) != 0;
    C wb[4];
    rvec(wb);
    double pb[4] = {0, 0, 0, 0};
    adj(p, m, lam, flag, wb, pb);
    const double h = 3e-2;  // rounding ~ eps |w| / h dominates below this step
    double lhs = 0;
    const double cs[4] = {1.0 / 12, -8.0 / 12, 8.0 / 12, -1.0 / 12};
    const double st[4] = {-2, -1, 1, 2};
    for (int j = 0; j < 4; ++j) {
      double q[4];
      for (int k = 0; k < 4; ++k) q[k] = p[k] + st[j] * h * dp[k];
      C w[4];
      fwd(q, m, lam, flag, w);
      lhs += cs[j] * re4(wb, w) / h;
    }
    r.add(lhs, kdot(pb, dp));
  }
}

int main() {
  test_bilinear();
  test_mdot_i();
  test_ffv_amp();
  test_cur_v0();
  test_cur_vm();
  test_cur_fin(173.0, 1.49);
  test_cur_fin(0.0, 0.0);
  test_cur_fout(173.0, 1.49);
  test_cur_fout(0.0, 0.0);
  test_vvv();
  test_vvvv<1>("adj_vvvv_cur<1>");
  test_vvvv<2>("adj_vvvv_cur<2>");
  test_vvvv<3>("adj_vvvv_cur<3>");
  test_ext(
      "adj_ext_vector", 0.0,
      [](const double* q, double, int lam, bool cj, C* w) { ext_vector<double>(q, lam, cj, w); },
      [](const double* p, double, int lam, bool cj, const C* wb, double* pb) {
        adj_ext_vector<double>(p, lam, cj, wb, pb);
      });
  test_ext(
      "adj_ext_u", 173.0,
      [](const double* q, double m, int lam, bool b, C* w) { ext_u<double>(q, m, lam, b, w); },
      [](const double* p, double m, int lam, bool b, const C* wb, double* pb) {
        adj_ext_u<double>(p, m, lam, b, wb, pb);
      });
  test_ext(
      "adj_ext_v", 173.0,
      [](const double* q, double m, int lam, bool b, C* w) { ext_v<double>(q, m, lam, b, w); },
      [](const double* p, double m, int lam, bool b, const C* wb, double* pb) {
        adj_ext_v<double>(p, m, lam, b, wb, pb);
      });
  test_ext(
      "adj_ext_u(massless)", 0.0,
      [](const double* q, double m, int lam, bool b, C* w) { ext_u<double>(q, m, lam, b, w); },
      [](const double* p, double m, int lam, bool b, const C* wb, double* pb) {
        adj_ext_u<double>(p, m, lam, b, wb, pb);
      });
  return 0;
}
