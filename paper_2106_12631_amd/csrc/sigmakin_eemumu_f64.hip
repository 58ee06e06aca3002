// SIGMAKIN for eemumu with double amplitudes: the generated colour-flow amplitudes
// and colour sum wrapped for the kernel of sigmakin_impl.h.
#include "sigmakin_impl.h"

namespace mg {
#include "generated/eemumu.inc"

struct P_eemumu {
  static constexpr int NPAR = gen_eemumu::NPAR;
  static constexpr int NCOL = gen_eemumu::NCOL;
  static constexpr int CDEN = gen_eemumu::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_eemumu::CNUM[0][0]; }
  template <typename T, bool UNI = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<T>& c, cx<T> (&J)[NCOL]) {
    gen_eemumu::jamps<T, UNI>(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_eemumu::colour_sum<T>(J);
  }
};

int launch_sigmakin_eemumu_f64(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, double* mehel, hipStream_t s) {
  return sigmakin_launch<P_eemumu, double, MG_EPL_BLOCK>(a, a.c64, mom, nevt, me, wgt, evtw, mehel, s);
}

// FP64 recomputation of the ill-conditioned events of a reduced-precision
// launch (precision guard of sigmakin_impl.h)
int launch_sigmakin_eemumu_guard(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_guard_launch<P_eemumu>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
