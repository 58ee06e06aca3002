// Cross section and unweighted events from weighted events f_i = w_i |M|^2_i
// (the two outputs of a matrix-element generator, Sec. II: a fiducial cross
// section and a sample of unweighted events obtained from a larger set of
// weighted ones by Monte Carlo).
//
// xsec_stats_kernel: one block of 1024 threads; thread t sums a contiguous
// chunk of events in FP64 (sum f, sum f^2, max f, number of finite f), then a
// fixed-order tree over the block: the result does not depend on timing.
// Non-finite f are left out and counted.
//
// Hit-or-miss unweighting: event i is kept iff u_i fmax < f_i with u_i the
// Philox uniform of (seed, event evt_offset + i) at block UNW_BLOCK (a
// counter block no sampler uses, so the same seed may serve both).  The
// kept indices are written in increasing order (stream compaction):
//   unw_count_kernel   per 256-event block: number kept -> ws[b]
//   unw_scan_kernel    one block: exclusive prefix sum of ws in place, total
//   unw_write_kernel   per block: wave ballots + LDS offsets -> idx_out
#include <mutex>

#include "../../include/mg5mi.h"
#include "common.h"
#include "internal.h"
#include "philox.h"

namespace mg {

constexpr uint32_t UNW_BLOCK = 0x80000000u;

__device__ __forceinline__ double unweight_uniform(uint64_t seed, uint64_t ievt) {
  uint32_t c0 = (uint32_t)ievt, c1 = (uint32_t)(ievt >> 32), c2 = UNW_BLOCK, c3 = 0u;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  return bits_to_u(c0, c1);
}

__global__ void __launch_bounds__(1024) xsec_stats_kernel(const double* __restrict__ f, int64_t n,
                                                          double* __restrict__ out) {
  __shared__ double s0[1024], s1[1024], s2[1024], s3[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t b = (int64_t)t * chunk, e = b + chunk < n ? b + chunk : n;
  double sum = 0.0, sq = 0.0, mx = 0.0, cnt = 0.0;
  for (int64_t i = b; i < e; ++i) {
    const double v = f[i];
    if (isfinite(v)) {
      sum += v;
      sq += v * v;
      mx = v > mx ? v : mx;
      cnt += 1.0;
    }
  }
  s0[t] = sum;
  s1[t] = sq;
  s2[t] = mx;
  s3[t] = cnt;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (t < st) {
      s0[t] += s0[t + st];
      s1[t] += s1[t + st];
      s2[t] = s2[t + st] > s2[t] ? s2[t + st] : s2[t];
      s3[t] += s3[t + st];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
    out[2] = s2[0];
    out[3] = s3[0];
  }
}

__device__ __forceinline__ bool keep(const double* f, int64_t i, int64_t n, double fmax,
                                     uint64_t seed, int64_t off) {
  if (i >= n) return false;
  const double v = f[i];
  return unweight_uniform(seed, (uint64_t)(off + i)) * fmax < v;  // false for NaN
}

__global__ void __launch_bounds__(256) unw_count_kernel(const double* __restrict__ f, int64_t n,
                                                        double fmax, uint64_t seed, int64_t off,
                                                        int64_t* __restrict__ ws) {
  __shared__ int cnt[4];
  const int t = threadIdx.x, w = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  const uint64_t m = __ballot(keep(f, i, n, fmax, seed, off));
  if ((t & 63) == 0) cnt[w] = __popcll(m);
  __syncthreads();
  if (t == 0) ws[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// exclusive scan of ws[0..nb) in place; total -> *count
__global__ void __launch_bounds__(1024) unw_scan_kernel(int64_t* __restrict__ ws, int64_t nb,
                                                        int64_t* __restrict__ count) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (nb + 1023) / 1024;
  const int64_t b = (int64_t)t * chunk, e = b + chunk < nb ? b + chunk : nb;
  int64_t s = 0;
  for (int64_t k = b; k < e; ++k) s += ws[k];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t add = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = t ? part[t - 1] : 0;
  for (int64_t k = b; k < e; ++k) {
    const int64_t c = ws[k];
    ws[k] = run;
    run += c;
  }
  if (t == 1023) *count = part[1023];
}

__global__ void __launch_bounds__(256) unw_write_kernel(const double* __restrict__ f, int64_t n,
                                                        double fmax, uint64_t seed, int64_t off,
                                                        const int64_t* __restrict__ ws,
                                                        int64_t* __restrict__ idx) {
  __shared__ int cnt[4];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  const bool k = keep(f, i, n, fmax, seed, off);
  const uint64_t m = __ballot(k);
  if (l == 0) cnt[w] = __popcll(m);
  __syncthreads();
  int64_t base = ws[blockIdx.x];
  for (int v = 0; v < w; ++v) base += cnt[v];
  if (k) idx[base + __popcll(m & ((1ull << l) - 1ull))] = i;
}

// Fixed device scratch of the allocation-free unweighting entry point: one
// int64 per 256-event block, for at most MG_UNWEIGHT_NOALLOC_MAX_EVENTS
// events.  Every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t SCRATCH_BLOCKS = (MG_UNWEIGHT_NOALLOC_MAX_EVENTS + 255) / 256;
static __device__ __align__(256) int64_t scratch[SCRATCH_BLOCKS];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mutex;
static int64_t* scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device (nullptr on error).
int64_t* unweight_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = (int64_t*)ptr;
  }
  return scratch_ptr[dev];
}

int launch_xsec_stats(const double* f, int64_t n, double* out, hipStream_t s) {
  xsec_stats_kernel<<<1, 1024, 0, s>>>(f, n, out);
  return 0;
}

int64_t unweight_blocks(int64_t n) { return (n + 255) / 256; }

int launch_unweight(const double* f, int64_t n, double fmax, uint64_t seed, int64_t off,
                    int64_t* idx, int64_t* count, int64_t* ws, hipStream_t s) {
  const int64_t nb = unweight_blocks(n);
  if (nb > 0x7FFFFFFF) return -1;
  if (nb > 0) unw_count_kernel<<<(unsigned)nb, 256, 0, s>>>(f, n, fmax, seed, off, ws);
  unw_scan_kernel<<<1, 1024, 0, s>>>(ws, nb, count);  // nb = 0: writes count = 0
  if (nb > 0) unw_write_kernel<<<(unsigned)nb, 256, 0, s>>>(f, n, fmax, seed, off, ws, idx);
  return 0;
}

}  // namespace mg
