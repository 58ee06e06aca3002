// Calibration kernels: the throughput each arithmetic unit of the GPU
// reaches on an instruction stream of one kind, to price the roofline of
// the matrix-element kernels.  Not part of the matrix-element path.
//
//   kind 0  FP64 vector FMA      (v_fma_f64)
//   kind 1  FP32 vector FMA      (v_fma_f32; packed FP32 is disabled in
//                                 every build of this project)
//   kind 2  BF16 MFMA            (v_mfma_f32_32x32x16_bf16)
//   kind 3  FP32 MFMA            (v_mfma_f32_32x32x2f32)
//   kind 4  FP64 MFMA            (v_mfma_f64_16x16x4f64)
//
// Every thread (or wave, for the matrix cores) runs independent dependency
// chains so that issue rate, not latency, limits it; the grid holds 16
// waves per CU.  mgcal_run returns the FLOP/s of one timed launch (after an
// untimed one) measured with HIP events, and the launch's duration.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BLOCK = 256;
constexpr int CHAINS = 8;   // independent FMA chains per thread
constexpr int UNROLL = 16;

template <typename T>
__global__ void __launch_bounds__(BLOCK) fma_kernel(T* out, int iters, T a, T b) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  T x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = (T)(gid % 97) * (T)1e-3 + (T)c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
#pragma unroll
      for (int c = 0; c < CHAINS; ++c) x[c] = fma(x[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[gid] = s;
}

constexpr int MCHAINS = 4;  // independent accumulators per wave

__global__ void __launch_bounds__(BLOCK) mfma_bf16_kernel(float* out, int iters) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  bf16x8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(float)((gid + j) % 7 - 3);
    b[j] = (__bf16)(float)((gid * 3 + j) % 5 - 2);
  }
  floatx16 acc[MCHAINS];
#pragma unroll
  for (int c = 0; c < MCHAINS; ++c) acc[c] = floatx16{0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < MCHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < MCHAINS; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[c][r];
  out[gid] = s;
}

__global__ void __launch_bounds__(BLOCK) mfma_f32_kernel(float* out, int iters) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  const float a = (float)(gid % 7 - 3), b = (float)(gid % 5 - 2);
  floatx16 acc[MCHAINS];
#pragma unroll
  for (int c = 0; c < MCHAINS; ++c) acc[c] = floatx16{0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < MCHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < MCHAINS; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[c][r];
  out[gid] = s;
}

__global__ void __launch_bounds__(BLOCK) mfma_f64_kernel(double* out, int iters) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  const double a = (double)(gid % 7 - 3), b = (double)(gid % 5 - 2);
  doublex4 acc[MCHAINS];
#pragma unroll
  for (int c = 0; c < MCHAINS; ++c) acc[c] = doublex4{0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < MCHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < MCHAINS; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += acc[c][r];
  out[gid] = s;
}

}  // namespace

extern "C" {

// Runs calibration kernel `kind` (0..4, see above) with `blocks` blocks of
// 256 threads and `iters` loop iterations on the null stream, synchronising
// the device.  out: device buffer of at least blocks * 256 * 8 bytes.
// Returns 0, -1 for a bad argument, -4 for a HIP error.
int mgcal_run(int kind, int blocks, int iters, void* out, double* flops_per_s, double* seconds) {
  if (kind < 0 || kind > 4 || blocks < 1 || iters < 1 || !out || !flops_per_s || !seconds)
    return -1;
  const double threads = (double)blocks * BLOCK;
  double flops = 0;
  switch (kind) {
    case 0:
    case 1: flops = threads * iters * UNROLL * CHAINS * 2.0; break;
    case 2: flops = threads / 64 * iters * MCHAINS * (2.0 * 32 * 32 * 16); break;
    case 3: flops = threads / 64 * iters * MCHAINS * (2.0 * 32 * 32 * 2); break;
    case 4: flops = threads / 64 * iters * MCHAINS * (2.0 * 16 * 16 * 4); break;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -4;
  for (int rep = 0; rep < 2; ++rep) {
    if (rep == 1) (void)hipEventRecord(e0, 0);
    switch (kind) {
      case 0: fma_kernel<double><<<blocks, BLOCK>>>((double*)out, iters, 0.999999, 1e-3); break;
      case 1: fma_kernel<float><<<blocks, BLOCK>>>((float*)out, iters, 0.999f, 1e-3f); break;
      case 2: mfma_bf16_kernel<<<blocks, BLOCK>>>((float*)out, iters); break;
      case 3: mfma_f32_kernel<<<blocks, BLOCK>>>((float*)out, iters); break;
      case 4: mfma_f64_kernel<<<blocks, BLOCK>>>((double*)out, iters); break;
    }
    if (rep == 1) (void)hipEventRecord(e1, 0);
  }
  const hipError_t err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess || hipGetLastError() != hipSuccess || !(ms > 0.f)) return -4;
  *seconds = ms * 1e-3;
  *flops_per_s = flops / *seconds;
  return 0;
}

}  // extern "C"
