// SIGMAKIN for ggttg with double amplitudes: the generated colour-flow amplitudes
// and colour sum wrapped for the kernel of sigmakin_impl.h.
#include "sigmakin_impl.h"

namespace mg {
#include "generated/ggttg.inc"

struct P_ggttg {
  static constexpr int NPAR = gen_ggttg::NPAR;
  static constexpr int NCOL = gen_ggttg::NCOL;
  static constexpr int CDEN = gen_ggttg::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_ggttg::CNUM[0][0]; }
  template <typename T, bool UNI = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<T>& c, cx<T> (&J)[NCOL]) {
    gen_ggttg::jamps<T, UNI>(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_ggttg::colour_sum<T>(J);
  }
};

int launch_sigmakin_ggttg_f64(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, double* mehel, hipStream_t s) {
  return sigmakin_launch<P_ggttg, double, MG_EPL_BLOCK>(a, a.c64, mom, nevt, me, wgt, evtw, mehel, s);
}

// FP64 recomputation of the ill-conditioned events of a reduced-precision
// launch (precision guard of sigmakin_impl.h)
int launch_sigmakin_ggttg_guard(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_guard_launch<P_ggttg>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
