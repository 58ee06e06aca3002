// SIGMAKIN for ggttg, mixed precision: FP32 colour-flow amplitudes and the
// colour sum on the matrix cores (kernels of sigmakin_impl.h).
#include "sigmakin_impl.h"

namespace mg {
#include "generated/ggttg.inc"

struct P_ggttg {
  static constexpr int NPAR = gen_ggttg::NPAR;
  static constexpr int NCOL = gen_ggttg::NCOL;
  static constexpr int CDEN = gen_ggttg::CDEN;
  __device__ static __forceinline__ const int* cnum() { return &gen_ggttg::CNUM[0][0]; }
  template <typename T>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<float>& c, cx<float> (&J)[NCOL]) {
    gen_ggttg::jamps_f32m(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_ggttg::colour_sum<T>(J);
  }
};

int launch_sigmakin_ggttg_mfma_f32(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_launch<P_ggttg, ColourMfmaF32>(a, mom, nevt, me, wgt, evtw, s);
}

int launch_sigmakin_ggttg_mfma_bf16(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                 const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_launch<P_ggttg, ColourMfmaBf16>(a, mom, nevt, me, wgt, evtw, s);
}

}  // namespace mg
