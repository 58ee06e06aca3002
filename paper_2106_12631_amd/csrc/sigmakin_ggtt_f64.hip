// SIGMAKIN for ggtt with double amplitudes: the generated colour-flow amplitudes
// and colour sum wrapped for the kernel of sigmakin_impl.h.
#include "sigmakin_impl.h"

namespace mg {
#include "generated/ggtt.inc"

struct P_ggtt {
  static constexpr int NPAR = gen_ggtt::NPAR;
  static constexpr int NCOL = gen_ggtt::NCOL;
  static constexpr int CDEN = gen_ggtt::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_ggtt::CNUM[0][0]; }
  template <typename T, bool UNI = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<T>& c, cx<T> (&J)[NCOL]) {
    gen_ggtt::jamps<T, UNI>(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_ggtt::colour_sum<T>(J);
  }
};

int launch_sigmakin_ggtt_f64(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, double* mehel, hipStream_t s) {
  return sigmakin_launch<P_ggtt, double, MG_EPL_BLOCK>(a, a.c64, mom, nevt, me, wgt, evtw, mehel, s);
}

// FP64 recomputation of the ill-conditioned events of a reduced-precision
// launch (precision guard of sigmakin_impl.h)
int launch_sigmakin_ggtt_guard(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_guard_launch<P_ggtt>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
