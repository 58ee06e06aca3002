// Shared device/host definitions of the gfx950 |M|^2 library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "helas.h"
#include "helas_adj.h"

namespace mg {

// AoSoA page sizes (Sec. IV.b "AOSOA"): 64 events per page, so one wave64
// reads one (particle, component) row of a momentum page as 512 contiguous
// bytes -- a fully coalesced load.  -DMG_NEPPM=n builds another momentum
// page size (1: plain AoS) for the paper's page-size comparison.
#ifndef MG_NEPPM
#define MG_NEPPM 64
#endif
constexpr int NEPPM = MG_NEPPM;
constexpr int NEPPR = 64;

// Couplings and masses handed to the kernels by value (Sec. IV.c keeps
// physics parameters in constant memory; a kernel-argument struct lets two
// handles with different parameters coexist).
template <typename T>
struct Couplings {
  T gs, gs2;        // strong coupling and its square
  T cqed;           // photon-lepton coupling -e Q
  T czl, czr;       // Z-lepton chiral couplings
  double mt, wt;    // top mass and width
  double wtt;       // width of t- and u-channel top propagators (wt, or 0)
  double mz, wz;    // Z mass and width
};

struct HelList {
  int n;
  uint8_t code[64];
};

__host__ __device__ inline int64_t aosoa_mom(int64_t ievt, int ipar, int mu, int npar) {
  return ((ievt / NEPPM) * npar + ipar) * 4 * NEPPM + (int64_t)mu * NEPPM + (ievt % NEPPM);
}
__host__ __device__ inline int64_t aosoa_rnd(int64_t ievt, int irnd, int nrnd) {
  return ((ievt / NEPPR) * nrnd + irnd) * NEPPR + (ievt % NEPPR);
}

// Incoming momenta along +z and -z with equal energies, (E,0,0,E) and
// (E,0,0,-E), as RAMBO writes them in the partonic rest frame.  The SIGMAKIN
// kernels hold the amplitude body twice: for such events with the zero components
// written as constants (set_beams; jamps<..., BEAM = true>), so that the
// products with them fold away, and the general body for any other momenta.
// The test is exact, so both bodies see the same values.  The gradient
// kernel runs RAMBO itself and takes the beam body only.
template <int N>
__device__ __forceinline__ bool beams_on_axis(const double (&p)[N][4]) {
  const double E = p[0][0];
  return p[0][1] == 0.0 && p[0][2] == 0.0 && p[0][3] == E && p[1][0] == E &&
         p[1][1] == 0.0 && p[1][2] == 0.0 && p[1][3] == -E;
}
template <int N>
__device__ __forceinline__ void set_beams(double (&p)[N][4]) {
  const double E = p[0][0];
  p[0][1] = 0.0;
  p[0][2] = 0.0;
  p[0][3] = E;
  p[1][0] = E;
  p[1][1] = 0.0;
  p[1][2] = 0.0;
  p[1][3] = -E;
}
template <bool B>
struct Beam {
  static constexpr bool value = B;
};

}  // namespace mg
