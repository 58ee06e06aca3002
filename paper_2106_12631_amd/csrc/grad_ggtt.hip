// Gradient kernels for ggtt (adjoint_impl.h): the generated reverse-mode
// code (adjoint_a64: FP64, adjoint_a32: FP32 amplitudes).
#include "adjoint_impl.h"

namespace mg {
#include "generated/ggtt.inc"

struct A64_ggtt {
  __device__ static __forceinline__ double adjoint(double (&p)[gen_ggtt::NPAR][4], unsigned h,
                                                   const Couplings<double>& c,
                                                   double (&pb)[gen_ggtt::NPAR][4]) {
    return gen_ggtt::adjoint_a64(p, h, c, pb);
  }
};

struct A32_ggtt {
  __device__ static __forceinline__ double adjoint(double (&p)[gen_ggtt::NPAR][4], unsigned h,
                                                   const Couplings<float>& c,
                                                   double (&pb)[gen_ggtt::NPAR][4]) {
    return gen_ggtt::adjoint_a32(p, h, c, pb);
  }
};

int launch_grad_ggtt(int prec, const MeArgs& a, const RamboArgs& ra, const double* rnd, int64_t nevt,
                   const double* gbar, double* grad_rnd, double* grad_logw, double* mew,
                   hipStream_t s) {
  if (prec == 0)
    return adjoint_launch<A64_ggtt, 2, double>(a, ra, a.c64, rnd, nevt, gbar, grad_rnd, grad_logw,
                                                mew, s);
  return adjoint_launch<A32_ggtt, 2, float>(a, ra, a.c32, rnd, nevt, gbar, grad_rnd, grad_logw,
                                             mew, s);
}

}  // namespace mg
