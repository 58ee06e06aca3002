// Colour sum on the matrix cores (gfx950 MFMA), one wave of 64 events.
//
// Per helicity the squared amplitude is the quadratic form
//   |M|^2 = sum_ij C_ij Re(conj(J_i) J_j) = Re^T C Re + Im^T C Im
// with the event-independent colour matrix C (Sec. II).  For a wave of 64
// events this is a dense product Z = C [Re | Im] of an ncol x ncol matrix
// with an ncol x 128 matrix, followed by the per-event dot products
// sum_i J_i Z_i.  The product runs as two 32-event tiles per part (events
// 0-31: "lo", 32-63: "hi"), in the operand layouts
//
//   32x32 output, register r of lane l holds D[m][n] with n = l % 32,
//   m = 8 (r / 4) + 4 (l / 32) + r % 4;
//   v_mfma_f32_32x32x2_f32:  A[m = l%32][k = l/32],         B[k = l/32][n = l%32]
//   v_mfma_f32_32x32x16_bf16: A[m = l%32][k = 8(l/32) + j],  B[k = 8(l/32) + j][n = l%32]
//
// The amplitudes come out of the generated code one event per lane.  Lane l
// and lane l + 32 hold the two halves of every B column and D row group the
// tiles need, so one v_permlane32_swap per register builds both tiles'
// operands from the lane's own values: with a from every lane and b from
// every lane, swap(a, b) returns r0 = (a of lanes 0-31, b of lanes 0-31
// moved up) -- the lo tile -- and r1 = (a of lanes 32-63 moved down, b of
// lanes 32-63) -- the hi tile.  The operands need no LDS staging and no
// barrier (the kernels may park the constant A operands in LDS).
//
// Two forms:
//   ColourMfmaF32   FP32 operands (C integer numerators exact in FP32),
//                   FP32 accumulation;
//   ColourMfmaBf16  each FP32 jamp split exactly into three BF16 terms by
//                   truncation (hi = top 8 significand bits, mid = next 8,
//                   lo = the rest, exact because it has at most 8 bits)
//                   against the integer numerators of C, exact in BF16
//                   (|C| <= 512 with at most 8 significant bits), FP32
//                   accumulation.  K runs over (split, colour group of 8):
//                   chunk c = s G + g holds split s of colours 8g .. 8g+7,
//                   and C is repeated for the three splits, so one product
//                   gives C (hi + mid + lo) = C J.
// The A operands (the colour matrix, the same for every event) are not
// built on the device: the generator writes them per K block and lane in
// the layout above (CS_A_F32, CS_A_BF16 of the generated code), and init()
// loads this lane's.
// Every lane of the wave must call sum() together (cross-lane operations);
// the kernels using it run one wave per block.
#pragma once
#include <hip/hip_runtime.h>

#include "helas.h"

namespace mg {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

// the upper halves of two words in one: (a >> 16 << 16) | (b >> 16), one
// v_perm_b32 (byte select 2, 3 of b, then 2, 3 of a)
__device__ __forceinline__ unsigned pack_upper(unsigned a, unsigned b) {
  return __builtin_amdgcn_perm(a, b, 0x07060302u);
}

// (lo tile, hi tile) operands from this lane's a and b (see above)
__device__ __forceinline__ void swap_halves(unsigned a, unsigned b, unsigned& lo, unsigned& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  lo = r[0];
  hi = r[1];
}
__device__ __forceinline__ void swap_halves(float a, float b, float& lo, float& hi) {
  unsigned ul, uh;
  swap_halves(__float_as_uint(a), __float_as_uint(b), ul, uh);
  lo = __uint_as_float(ul);
  hi = __uint_as_float(uh);
}

// Dot of the two tiles' 32x32 outputs with the amplitudes x (this lane's
// event, one part) in D's row layout, summed into this lane's event.
// part_lo / part_hi accumulate over the real and imaginary parts.
template <int NCOL>
__device__ __forceinline__ void tile_dots(const floatx16& dlo, const floatx16& dhi,
                                          const float (&x)[NCOL], float& part_lo,
                                          float& part_hi) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int mlo = 8 * (r / 4) + r % 4, mhi = mlo + 4;
    if (mlo < NCOL) {
      float jlo, jhi;
      swap_halves(x[mlo], mhi < NCOL ? x[mhi] : 0.f, jlo, jhi);
      part_lo += dlo[r] * jlo;
      part_hi += dhi[r] * jhi;
    }
  }
}

// lane l < 32: its event's total is part_lo(l) + part_lo(l + 32);
// lane l >= 32: part_hi(l - 32) + part_hi(l)
__device__ __forceinline__ float combine_halves(float part_lo, float part_hi, int lane) {
  float from_hi, from_lo;  // r0 of lanes >= 32 = part_hi of lane - 32; r1 of lanes < 32 = part_lo of lane + 32
  swap_halves(part_lo, part_hi, from_hi, from_lo);
  return lane < 32 ? part_lo + from_lo : part_hi + from_hi;
}

template <int NCOL>
struct ColourMfmaF32 {
  static constexpr int KB = (NCOL + 1) / 2;  // K blocks of 2
  using Word = float;                        // one A-operand register per K block
  float a[KB];

  // the A operands can be parked in LDS (tab[kb][lane]) between colour sums
  // so that they take no registers across the amplitude code
  __device__ __forceinline__ void save(Word* tab, int lane) const {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) tab[kb * 64 + lane] = a[kb];
  }
  __device__ __forceinline__ void restore(const Word* tab, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) a[kb] = tab[kb * 64 + lane];
  }

  // the generated table: tab[kb][lane] = C[lane % 32][2 kb + lane / 32]
  // (numerators, 0 past the matrix)
  template <class P>
  __device__ static __forceinline__ const Word* table() {
    return P::cs_a_f32();
  }
  __device__ __forceinline__ void init(const Word* tab, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) a[kb] = tab[kb * 64 + lane];
  }

  // returns sum_ij C_ij Re(conj(J_i) J_j) (numerators of C) for this lane's event
  __device__ __forceinline__ float sum(const cx<float> (&J)[NCOL], int lane) {
    return sum_parts([&](int part, int k) { return part ? J[k].i : J[k].r; },
                     [&](int kb) { return a[kb]; }, lane);
  }

  // the same with the amplitudes read through get(part, k) (part 0: real,
  // 1: imaginary), one part at a time, and the A operand of K block kb
  // through aop(kb) (e.g. from a table written by save())
  template <class Get, class AOp>
  __device__ __forceinline__ float sum_parts(Get get, AOp aop, int lane) {
    float part_lo = 0.f, part_hi = 0.f;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      float x[NCOL];
#pragma unroll
      for (int k = 0; k < NCOL; ++k) x[k] = get(part, k);
      floatx16 dlo = {0}, dhi = {0};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        float blo, bhi;
        swap_halves(x[2 * kb], 2 * kb + 1 < NCOL ? x[2 * kb + 1] : 0.f, blo, bhi);
        const float ak = aop(kb);
        dlo = __builtin_amdgcn_mfma_f32_32x32x2f32(ak, blo, dlo, 0, 0, 0);
        dhi = __builtin_amdgcn_mfma_f32_32x32x2f32(ak, bhi, dhi, 0, 0, 0);
      }
      tile_dots<NCOL>(dlo, dhi, x, part_lo, part_hi);
    }
    return combine_halves(part_lo, part_hi, lane);
  }
};

template <int NCOL>
struct ColourMfmaBf16 {
  static constexpr int G = (NCOL + 7) / 8;  // colour groups of 8
  static constexpr int NCH = 3 * G;         // chunks (split, group) of 8 K entries
  static constexpr int KB = (NCH + 1) / 2;  // K blocks of 16 (two chunks)
  using Word = uintx4;
  bf16x8 a[KB];

  __device__ __forceinline__ void save(Word* tab, int lane) const {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) tab[kb * 64 + lane] = __builtin_bit_cast(uintx4, a[kb]);
  }
  __device__ __forceinline__ void restore(const Word* tab, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) a[kb] = __builtin_bit_cast(bf16x8, tab[kb * 64 + lane]);
  }

  // the generated table: tab[kb][lane] = C[lane % 32][8 g + j], j = 0..7,
  // g = (2 kb + lane / 32) % G, as eight BF16 numerators (exact: at most 8
  // significant bits), 0 past the matrix and the last chunk
  template <class P>
  __device__ static __forceinline__ const Word* table() {
    return (const Word*)P::cs_a_bf16();
  }
  __device__ __forceinline__ void init(const Word* tab, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) a[kb] = __builtin_bit_cast(bf16x8, tab[kb * 64 + lane]);
  }

  __device__ __forceinline__ float sum(const cx<float> (&J)[NCOL], int lane) {
    return sum_parts([&](int part, int k) { return part ? J[k].i : J[k].r; },
                     [&](int kb) { return a[kb]; }, lane);
  }

  template <class Get, class AOp>
  __device__ __forceinline__ float sum_parts(Get get, AOp aop, int lane) {
    float part_lo = 0.f, part_hi = 0.f;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      float x[NCOL];
#pragma unroll
      for (int k = 0; k < NCOL; ++k) x[k] = get(part, k);
      // the exact three-term split of every amplitude by truncation, each
      // term in the upper half of a word: hi = x, mid = x - hi, lo =
      // mid's residual (at most 8 significant bits remain: exact in BF16)
      unsigned t[3][NCOL];
#pragma unroll
      for (int k = 0; k < NCOL; ++k) {
        const unsigned u = __float_as_uint(x[k]);
        const float r1 = x[k] - __uint_as_float(u & 0xFFFF0000u);
        const unsigned u1 = __float_as_uint(r1);
        t[0][k] = u;
        t[1][k] = u1;
        t[2][k] = __float_as_uint(r1 - __uint_as_float(u1 & 0xFFFF0000u));
      }
      floatx16 dlo = {0}, dhi = {0};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        unsigned ulo[4], uhi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          unsigned w[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            // chunk c: term s of colours 8 g + 2 q (low half) and + 1 (high)
            const int c = 2 * kb + h, s = c / G, g = c % G;
            const int k0 = 8 * g + 2 * q, k1 = k0 + 1;
            w[h] = c < NCH ? pack_upper(k1 < NCOL ? t[s < 3 ? s : 0][k1] : 0u,
                                        k0 < NCOL ? t[s < 3 ? s : 0][k0] : 0u)
                           : 0u;
          }
          swap_halves(w[0], w[1], ulo[q], uhi[q]);
        }
        const uintx4 vlo = {ulo[0], ulo[1], ulo[2], ulo[3]};
        const uintx4 vhi = {uhi[0], uhi[1], uhi[2], uhi[3]};
        const bf16x8 ak = aop(kb);
        dlo = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ak, __builtin_bit_cast(bf16x8, vlo), dlo, 0,
                                                      0, 0);
        dhi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ak, __builtin_bit_cast(bf16x8, vhi), dhi, 0,
                                                      0, 0);
      }
      tile_dots<NCOL>(dlo, dhi, x, part_lo, part_hi);
    }
    return combine_halves(part_lo, part_hi, lane);
  }
};

}  // namespace mg
