// Host-side launchers shared by the kernels' translation units and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mg {

struct RamboArgs {
  double sqrts;
  double w0;      // massless phase-space volume (pi/2)^(n-1) s^(n-2) / ((n-1)!(n-2)!)
  double xi0;     // Newton start sqrt(1 - (sum m / sqrt s)^2)
  double m2[4];   // final-state masses squared
  int massive;
};

// all return 0, or -1 for an unsupported size
int launch_rng(int nrnd, uint64_t seed, int64_t off, int64_t nevt, double* rnd, hipStream_t s);
int launch_rambo(int nf, const double* rnd, int64_t nevt, const RamboArgs& a, double* mom,
                 double* wgt, hipStream_t s);
int launch_sample(int nf, uint64_t seed, int64_t off, int64_t nevt, const RamboArgs& a,
                  double* rnd, double* mom, double* wgt, hipStream_t s);

struct MeArgs {
  Couplings<double> c64;
  Couplings<float> c32;
  HelList hel;
  double inv_iden;
  double guard_kappa;  // reduced precision: FP64 recomputation above this kappa (0: off)
};

int launch_sigmakin(int proc, int prec, const MeArgs& a, const double* mom, int64_t nevt,
                    double* me, const double* wgt, double* evtw, hipStream_t s);
int launch_sigmakin_hel(int proc, int prec, const MeArgs& a, const double* mom, int64_t nevt,
                        double* mehel, hipStream_t s);
int launch_count_nonfinite(const double* x, int64_t n, int64_t* d_count, hipStream_t s);
int64_t xsec_blocks(int64_t n);
int launch_xsec_stats(const double* f, int64_t n, double* out, double* ws, hipStream_t s);
int64_t unweight_blocks(int64_t n);
int launch_unweight(const double* f, int64_t n, double fmax, uint64_t seed, int64_t off,
                    int64_t* idx, int64_t* count, int64_t* ws, hipStream_t s);
int64_t* unweight_scratch();

}  // namespace mg
