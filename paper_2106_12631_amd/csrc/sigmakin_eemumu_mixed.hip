// SIGMAKIN for eemumu, mixed precision: FP32 colour-flow amplitudes and the
// colour sum on the matrix cores (kernels of sigmakin_impl.h).
#include "sigmakin_impl.h"

namespace mg {
#include "generated/eemumu.inc"

struct P_eemumu {
  static constexpr int NPAR = gen_eemumu::NPAR;
  static constexpr int NCOL = gen_eemumu::NCOL;
  static constexpr int CDEN = gen_eemumu::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_eemumu::CNUM[0][0]; }
  template <typename T>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<float>& c, cx<float> (&J)[NCOL]) {
    gen_eemumu::jamps_f32m(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_eemumu::colour_sum<T>(J);
  }
};

int launch_sigmakin_eemumu_mfma_f32(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_launch<P_eemumu, ColourMfmaF32>(a, mom, nevt, me, wgt, evtw, s);
}

int launch_sigmakin_eemumu_mfma_bf16(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                 const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_launch<P_eemumu, ColourMfmaBf16>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
