// SIGMAKIN for eemumu with float amplitudes: the generated colour-flow amplitudes
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

int launch_sigmakin_eemumu_f32(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                              const double* wgt, double* evtw, double* mehel, hipStream_t s) {
  return sigmakin_launch<P_eemumu, float, MG_EPL_BLOCK>(a, a.c32, mom, nevt, me, wgt, evtw, mehel, s);
}

}  // namespace mg
