// SIGMAKIN for ggttgg, mixed precision: FP32 colour-flow amplitudes and the
// colour sum on the matrix cores (kernels of sigmakin_impl.h): one helicity
// per lane with the FP32 body of the helicity-per-lane FP32 kernel when all
// 64 helicities are kept, else event per lane with its own body.
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
                                               const Couplings<float>& c, cx<float> (&J)[NCOL]) {
    gen_ggttgg::jamps_f32m<UNI>(p, h, c, J);
  }
  template <typename T>
  __device__ static __forceinline__ T colour_sum(const cx<T> (&J)[NCOL]) {
    return gen_ggttgg::colour_sum<T>(J);
  }
};

struct P_ggttgg_hpl : P_ggttgg {
  template <typename T, bool UNI = false>
  __device__ static __forceinline__ void jamps(double (&p)[NPAR][4], unsigned h,
                                               const Couplings<float>& c, cx<float> (&J)[NCOL]) {
    gen_ggttgg::jamps<float, UNI>(p, h, c, J);
  }
};

int launch_sigmakin_ggttgg_mfma_f32(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_hpl_launch<P_ggttgg, P_ggttgg_hpl, ColourMfmaF32>(a, mom, nevt, me, wgt,
                                                                          evtw, s);
}

int launch_sigmakin_ggttgg_mfma_bf16(const MeArgs& a, const double* mom, int64_t nevt, double* me,
                                 const double* wgt, double* evtw, hipStream_t s) {
  return sigmakin_mixed_hpl_launch<P_ggttgg, P_ggttgg_hpl, ColourMfmaBf16>(a, mom, nevt, me, wgt,
                                                                           evtw, s);
}

}  // namespace mg
