// Colour sum on the matrix cores (gfx950 MFMA), one wave of 64 events.
//
// Per helicity the squared amplitude is the quadratic form
//   |M|^2 = sum_ij C_ij Re(conj(J_i) J_j) = Re^T C Re + Im^T C Im
// with the event-independent colour matrix C (Sec. II).  For a wave of 64
// events this is a dense product Z = C [Re | Im] of an ncol x ncol matrix
// with an ncol x 128 matrix (64 events x real/imaginary part), followed by
// the per-event dot products sum_i J_i Z_i.  The jamps come out of the
// amplitude code one event per lane; they are staged through LDS into the
// operand layout of the MFMA instructions:
//
//   32x32 output, register r of lane l holds D[m][n] with n = l % 32,
//   m = 8 (r / 4) + 4 (l / 32) + r % 4;
//   v_mfma_f32_32x32x2_f32:  A[m = l%32][k = l/32],         B[k = l/32][n = l%32]
//   v_mfma_f32_32x32x16_bf16: A[m = l%32][k = 8(l/32) + j],  B[k = 8(l/32) + j][n = l%32]
//
// Two forms:
//   ColourMfmaF32   FP32 operands (C integer numerators exact in FP32),
//                   FP32 accumulation;
//   ColourMfmaBf16  the jamps split into three BF16 terms hi + mid + lo
//                   (together the 24 significand bits of FP32) against the
//                   integer numerators of C, exact in BF16 (|C| <= 512 with
//                   at most 8 significant bits), FP32 accumulation.  The
//                   three splits are laid side by side along K, so one
//                   product [C C C] [hi; mid; lo] gives C J.
// Every lane of the wave must call sum() together (it uses LDS exchange and
// block barriers); the kernels using it run one wave per block.
#pragma once
#include <hip/hip_runtime.h>

#include "helas.h"

namespace mg {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

// round-to-nearest-even FP32 -> BF16 bits (inputs are finite)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short b) {
  return __uint_as_float((unsigned)b << 16);
}

// dot of the 32x32 block D with the staged jamps in D's layout, reduced over
// the two half-waves: every lane ends with the value of its column
template <int NCOL>
__device__ __forceinline__ float block_dot(const floatx16& d, const float* f, int lane) {
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (m < NCOL) s += d[r] * f[m * 64];
  }
  return s + __shfl_xor(s, 32);
}

template <int NCOL>
struct ColourMfmaF32 {
  static constexpr int KB = (NCOL + 1) / 2;   // K blocks of 2
  static constexpr int LDS_BYTES = 2 * NCOL * 64 * 4;
  float a[KB];

  // cnum: the NCOL x NCOL integer numerators of C, row-major
  __device__ __forceinline__ void init(const int* cnum, int lane) {
    const int m = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = 2 * kb + kh;
      a[kb] = (m < NCOL && k < NCOL) ? (float)cnum[m * NCOL + k] : 0.f;
    }
  }

  // returns sum_ij C_ij Re(conj(J_i) J_j) (numerators of C) for this lane's event
  __device__ __forceinline__ float sum(void* lds_raw, const cx<float> (&J)[NCOL], int lane) {
    float* f = (float*)lds_raw;  // [part][k][64]
#pragma unroll
    for (int k = 0; k < NCOL; ++k) {
      f[k * 64 + lane] = J[k].r;
      f[(NCOL + k) * 64 + lane] = J[k].i;
    }
    __syncthreads();
    float tot = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int part = b >> 1, half = b & 1;
      const float* col = f + part * NCOL * 64 + half * 32 + (lane & 31);
      floatx16 d = {0};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int k = 2 * kb + (lane >> 5);
        const float bv = (k < NCOL) ? col[k * 64] : 0.f;
        d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kb], bv, d, 0, 0, 0);
      }
      const float s = block_dot<NCOL>(d, col, lane);
      if (half == (lane >> 5)) tot += s;
    }
    __syncthreads();
    return tot;
  }
};

template <int NCOL>
struct ColourMfmaBf16 {
  static constexpr int KP = 3 * NCOL;           // hi, mid, lo side by side along K
  static constexpr int KB = (KP + 15) / 16;     // K blocks of 16
  static constexpr int KPAD = KB * 16;
  static constexpr int LDS_F32 = 2 * NCOL * 64 * 4;
  static constexpr int LDS_BYTES = LDS_F32 + 128 * KPAD * 2;
  bf16x8 a[KB];

  __device__ __forceinline__ void init(const int* cnum, int lane) {
    const int m = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      ushort8 u;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int kk = 16 * kb + 8 * kh + j;
        u[j] = (m < NCOL && kk < KP) ? bf16_bits((float)cnum[m * NCOL + kk % NCOL])
                                     : (unsigned short)0;
      }
      a[kb] = __builtin_bit_cast(bf16x8, u);
    }
  }

  __device__ __forceinline__ float sum(void* lds_raw, const cx<float> (&J)[NCOL], int lane) {
    float* f = (float*)lds_raw;                                       // [part][k][64]
    unsigned short* h = (unsigned short*)((char*)lds_raw + LDS_F32);  // [column][KPAD]
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      unsigned short* row = h + (part * 64 + lane) * KPAD;
#pragma unroll
      for (int k = 0; k < NCOL; ++k) {
        const float x = part ? J[k].i : J[k].r;
        f[(part * NCOL + k) * 64 + lane] = x;
        const unsigned short b0 = bf16_bits(x);
        const float r1 = x - bf16_value(b0);
        const unsigned short b1 = bf16_bits(r1);
        const float r2 = r1 - bf16_value(b1);
        row[k] = b0;
        row[NCOL + k] = b1;
        row[2 * NCOL + k] = bf16_bits(r2);
      }
#pragma unroll
      for (int k = KP; k < KPAD; ++k) row[k] = 0;
    }
    __syncthreads();
    float tot = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int part = b >> 1, half = b & 1;
      const int column = part * 64 + half * 32 + (lane & 31);
      const ushort8* src = (const ushort8*)(h + column * KPAD + 8 * (lane >> 5));
      floatx16 d = {0};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const bf16x8 bv = __builtin_bit_cast(bf16x8, src[2 * kb]);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], bv, d, 0, 0, 0);
      }
      const float s = block_dot<NCOL>(d, f + part * NCOL * 64 + half * 32 + (lane & 31), lane);
      if (half == (lane >> 5)) tot += s;
    }
    __syncthreads();
    return tot;
  }
};

}  // namespace mg
