// SIGMAKIN for ggtt, mixed precision: FP32 colour-flow amplitudes and the
// colour sum on the matrix cores (kernels of sigmakin_impl.h).
#include "sigmakin_impl.h"

namespace mg {
#include "generated/ggtt.inc"

struct P_ggtt {
  static constexpr int NPAR = gen_ggtt::NPAR;
  static constexpr int NCOL = gen_ggtt::NCOL;
  static constexpr int CDEN = gen_ggtt::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_ggtt::CNUM[0][0]; }
  template <typename T>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<float>& c, cx<float> (&J)[NCOL]) {
    gen_ggtt::jamps_f32m(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_ggtt::colour_sum<T>(J);
  }
};

int launch_sigmakin_ggtt_mfma_f32(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_launch<P_ggtt, ColourMfmaF32>(a, mom, nevt, me, wgt, evtw, s);
}

int launch_sigmakin_ggtt_mfma_bf16(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                 const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_launch<P_ggtt, ColourMfmaBf16>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
