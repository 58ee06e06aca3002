// Cross section and unweighted events from weighted events f_i = w_i |M|^2_i
// (the two outputs of a matrix-element generator, Sec. II: a fiducial cross
// section and a sample of unweighted events obtained from a larger set of
// weighted ones by Monte Carlo).
//
// xsec_partial_kernel + xsec_final_kernel: FP64 sums of f and f^2, the
// maximum and the number of finite f in two passes of fixed shape (blocks
// over contiguous event ranges, then one block over their partials), so the
// result does not depend on timing.  Non-finite f are left out.
//
// Hit-or-miss unweighting: event i is kept iff u_i fmax < f_i with u_i the
// Philox uniform of (seed, event evt_offset + i) at block UNW_BLOCK (a
// counter block no sampler uses, so the same seed may serve both).  The
// kept indices are written in increasing order (stream compaction):
//   unw_count_kernel   per 256-event block: number kept -> ws[b]
//   unw_scan_kernel    one block: exclusive prefix sum of ws in place, total
//   unw_write_kernel   per block: wave ballots + LDS offsets -> idx_out
#include <mutex>

#include "mg5mi.h"
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

// Deterministic two-pass reduction of (sum f, sum f^2, max f, finite count).
// Pass 1: block b reduces the contiguous event range [b*chunk, (b+1)*chunk)
// (coalesced: thread t reads events b*chunk + t + 256 k), then a fixed tree
// over its 256 threads -> ws[4b .. 4b+3].  Pass 2: one block of 1024 threads
// reduces the nb partials (thread t: partials t, t + 1024, ...) by a fixed
// tree.  The block count and ranges depend on n only, so the result does not
// depend on timing.
constexpr int XS_THREADS = 256;
constexpr int64_t XS_MAX_BLOCKS = 2048;
constexpr int64_t XS_MIN_CHUNK = 4096;

int64_t xsec_blocks(int64_t n) {
  int64_t nb = (n + XS_MIN_CHUNK - 1) / XS_MIN_CHUNK;
  return nb < 1 ? 1 : (nb > XS_MAX_BLOCKS ? XS_MAX_BLOCKS : nb);
}

template <int NT>
__device__ __forceinline__ void reduce4(double (&s)[4][NT], int t) {
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (t < st) {
      s[0][t] += s[0][t + st];
      s[1][t] += s[1][t + st];
      s[2][t] = s[2][t + st] > s[2][t] ? s[2][t + st] : s[2][t];
      s[3][t] += s[3][t + st];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(XS_THREADS) xsec_partial_kernel(const double* __restrict__ f,
                                                                  int64_t n, int64_t chunk,
                                                                  double* __restrict__ ws) {
  __shared__ double s[4][XS_THREADS];
  const int t = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  double sum = 0.0, sq = 0.0, mx = 0.0, cnt = 0.0;
  for (int64_t i = b + t; i < e; i += XS_THREADS) {
    const double v = f[i];
    if (isfinite(v)) {
      sum += v;
      sq += v * v;
      mx = v > mx ? v : mx;
      cnt += 1.0;
    }
  }
  s[0][t] = sum;
  s[1][t] = sq;
  s[2][t] = mx;
  s[3][t] = cnt;
  __syncthreads();
  reduce4<XS_THREADS>(s, t);
  if (t < 4) ws[4 * blockIdx.x + t] = s[t][0];
}

__global__ void __launch_bounds__(1024) xsec_final_kernel(const double* __restrict__ ws,
                                                          int64_t nb, double* __restrict__ out) {
  __shared__ double s[4][1024];
  const int t = threadIdx.x;
  double sum = 0.0, sq = 0.0, mx = 0.0, cnt = 0.0;
  for (int64_t k = t; k < nb; k += 1024) {
    sum += ws[4 * k];
    sq += ws[4 * k + 1];
    mx = ws[4 * k + 2] > mx ? ws[4 * k + 2] : mx;
    cnt += ws[4 * k + 3];
  }
  s[0][t] = sum;
  s[1][t] = sq;
  s[2][t] = mx;
  s[3][t] = cnt;
  __syncthreads();
  reduce4<1024>(s, t);
  if (t < 4) out[t] = s[t][0];
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

int launch_xsec_stats(const double* f, int64_t n, double* out, double* ws, hipStream_t s) {
  const int64_t nb = xsec_blocks(n);
  const int64_t chunk = n > 0 ? (n + nb - 1) / nb : 0;
  xsec_partial_kernel<<<(unsigned)nb, XS_THREADS, 0, s>>>(f, n, chunk, ws);
  xsec_final_kernel<<<1, 1024, 0, s>>>(ws, nb, out);
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
