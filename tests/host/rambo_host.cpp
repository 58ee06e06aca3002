// Host build of the device RAMBO (rambo.h), for the CPU test
// test_rambo_host.py: reads event-major uniforms, writes momenta and
// weights, so the phase-space formulas of the HIP path can be compared with
// the oracle before any GPU run.
//
// usage: rambo_host NF SQRTS MASS IN OUT
//   IN:  nevt x 4 NF float64 uniforms (raw, event-major)
//   OUT: nevt x ((NF + 2) x 4 + 1) float64: momenta (E, px, py, pz) of all
//        particles, then the weight
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rambo.h"

using namespace mg;

template <int NF>
static void run(const std::vector<double>& in, std::vector<double>& out, const RamboArgs& a) {
  const size_t n = in.size() / (4 * NF);
  const int per = (NF + 2) * 4 + 1;
  out.assign(n * per, 0.0);
  for (size_t e = 0; e < n; ++e) {
    double r[4 * NF];
    for (int k = 0; k < 4 * NF; ++k) r[k] = in[e * 4 * NF + k];
    double p[NF + 2][4], w;
    rambo<NF>(r, a, p, w);
    for (int i = 0; i < NF + 2; ++i)
      for (int m = 0; m < 4; ++m) out[e * per + 4 * i + m] = p[i][m];
    out[e * per + per - 1] = w;
  }
}

int main(int argc, char** argv) {
  if (argc != 6) return 2;
  const int nf = atoi(argv[1]);
  const double sqrts = atof(argv[2]), mass = atof(argv[3]);
  FILE* f = fopen(argv[4], "rb");
  if (!f) return 3;
  std::vector<double> in;
  double buf[4096];
  size_t got;
  while ((got = fread(buf, sizeof(double), 4096, f)) > 0) in.insert(in.end(), buf, buf + got);
  fclose(f);
  // the same arguments mg_create derives (massless weight, Newton start)
  RamboArgs a{};
  a.sqrts = sqrts;
  const double pi = 3.14159265358979323846, s = sqrts * sqrts;
  double f1 = 1.0, f2 = 1.0;
  for (int k = 2; k <= nf - 1; ++k) f1 *= k;
  for (int k = 2; k <= nf - 2; ++k) f2 *= k;
  a.w0 = pow(pi / 2.0, nf - 1) * pow(s, nf - 2) / (f1 * f2);
  for (int i = 0; i < 4; ++i) a.m2[i] = 0.0;
  a.m2[0] = a.m2[1] = mass * mass;
  a.massive = mass > 0.0;
  a.xi0 = sqrt(1.0 - (2.0 * mass / sqrts) * (2.0 * mass / sqrts));
  std::vector<double> out;
  switch (nf) {
    case 2: run<2>(in, out, a); break;
    case 3: run<3>(in, out, a); break;
    case 4: run<4>(in, out, a); break;
    default: return 4;
  }
  f = fopen(argv[5], "wb");
  if (!f) return 5;
  fwrite(out.data(), sizeof(double), out.size(), f);
  fclose(f);
  return 0;
}
