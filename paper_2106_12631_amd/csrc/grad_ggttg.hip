// Gradient kernels for ggttg: the generated amplitudes on dual numbers
// (jamps_d64: FP64, jamps_d32: FP32 amplitudes) wrapped for adjoint_impl.h.
#include "adjoint_impl.h"

namespace mg {
#include "generated/ggttg.inc"

struct G64_ggttg {
  static constexpr int NCOL = gen_ggttg::NCOL;
  __device__ static __forceinline__ void jamps(dual<double> (&p)[gen_ggttg::NPAR][4], unsigned h,
                                               const Couplings<double>& c,
                                               cx<dual<double>> (&J)[NCOL]) {
    gen_ggttg::jamps_d64(p, h, c, J);
  }
  __device__ static __forceinline__ dual<double> colour_sum(const cx<dual<double>> (&J)[NCOL]) {
    return gen_ggttg::colour_sum<dual<double>>(J);
  }
};

struct G32_ggttg {
  static constexpr int NCOL = gen_ggttg::NCOL;
  __device__ static __forceinline__ void jamps(dual<double> (&p)[gen_ggttg::NPAR][4], unsigned h,
                                               const Couplings<float>& c,
                                               cx<dual<float>> (&J)[NCOL]) {
    gen_ggttg::jamps_d32(p, h, c, J);
  }
  __device__ static __forceinline__ dual<float> colour_sum(const cx<dual<float>> (&J)[NCOL]) {
    return gen_ggttg::colour_sum<dual<float>>(J);
  }
};

int launch_grad_ggttg(int prec, const MeArgs& a, const RamboArgs& ra, const double* rnd, int64_t nevt,
                   const double* gbar, double* grad_rnd, double* grad_logw, double* mew,
                   hipStream_t s) {
  if (prec == 0)
    return grad_launch<G64_ggttg, 3, dual<double>>(a, ra, a.c64, rnd, nevt, gbar, grad_rnd,
                                                  grad_logw, mew, s);
  return grad_launch<G32_ggttg, 3, dual<float>>(a, ra, a.c32, rnd, nevt, gbar, grad_rnd, grad_logw,
                                               mew, s);
}

}  // namespace mg
