// SIGMAKIN for ggttgg with double amplitudes: the generated colour-flow amplitudes
// and colour sum wrapped for the kernel of sigmakin_impl.h.
#include "sigmakin_impl.h"

namespace mg {
#include "generated/ggttgg.inc"

struct P_ggttgg {
  static constexpr int NPAR = gen_ggttgg::NPAR;
  static constexpr int NCOL = gen_ggttgg::NCOL;
  static constexpr int CDEN = gen_ggttgg::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_ggttgg::CNUM[0][0]; }
  template <typename T, bool UNI = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<T>& c, cx<T> (&J)[NCOL]) {
    gen_ggttgg::jamps<T, UNI>(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_ggttgg::colour_sum<T>(J);
  }
};

int launch_sigmakin_ggttgg_f64(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, double* mehel, hipStream_t s) {
#ifdef MG_EVENT_PER_LANE_F64
  return sigmakin_launch<P_ggttgg, double, 64>(a, a.c64, mom, nevt, me, wgt, evtw, mehel, s);
#else
  return sigmakin_hpl_launch<P_ggttgg, double, 64>(a, a.c64, mom, nevt, me, wgt, evtw, mehel, s);
#endif
}

// FP64 recomputation of the ill-conditioned events of a reduced-precision
// launch (precision guard of sigmakin_impl.h)
int launch_sigmakin_ggttgg_guard(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_guard_launch<P_ggttgg>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
