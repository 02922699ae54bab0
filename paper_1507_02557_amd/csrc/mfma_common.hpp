// Wave-level building blocks of the matrix-core kernels: MFMA wrappers and
// their lane layouts, operand precisions, wavefront synchronisation.
#pragma once

#include "stage_common.hpp"

namespace hdg {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// D = A B + C for 16x16 tiles, K = 4: lane l passes A[l%16][l/16] and
// B[l/16][l%16] and holds D[4(l/16)+i][l%16] in component i.
__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP16 operands, FP32 accumulation: 16x16x16 (lane l passes A[l%16][4(l/16)+i]
// and B[4(l/16)+i][l%16], i < 4) and 16x16x32 (A[l%16][8(l/16)+i],
// B[8(l/16)+i][l%16], i < 8); the result layout is that of mma_f32.
__device__ __forceinline__ f32x4 mma_f16(f16x4 a, f16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_f16(f16x8 a, f16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// BF16 operands, FP32 accumulation, 16x16x16 (lane layout of the FP16
// 16x16x16 one; the instruction takes the BF16 bit patterns as 16-bit
// integers).
__device__ __forceinline__ f32x4 mma_f16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c, 0,
                                                   0, 0);
}

// Operand precision of the element-batched operator products.
//   0: FP32 operands (16x16x4).
//   1: split FP16, 16x16x32: x = hi + lo with hi = fp16(s x), lo = fp16(s x - hi)
//      for a power-of-two scale s per operator and per element column, so
//      each operand carries about 22 significant bits; A B is formed as
//      hi hi + hi lo + lo hi with FP32 accumulation.
//   2: the same split with 16x16x16 instructions (less padding of K).
//   3: split BF16, 16x16x16: x = hi + lo, hi = bf16(x), lo = bf16(x - hi)
//      (about 16 significant bits; BF16 keeps FP32's exponent range), A B as
//      hi hi + hi lo + lo hi.
//   4: three-piece BF16, 16x16x16: x = hi + mid + lo, each the BF16 rounding
//      of what the previous pieces leave (about 24 significant bits), A B as
//      the six products whose piece orders add up to at most 2:
//      hi hi + hi mid + mid hi + hi lo + lo hi + mid mid.
template <int P>
struct Prec;
template <>
struct Prec<0> {
  static constexpr int KI = 1, KK = 4, NPC = 1;
  typedef float V;
};
template <>
struct Prec<1> {
  static constexpr int KI = 8, KK = 32, NPC = 2;
  typedef f16x8 V;
  typedef _Float16 E;
};
template <>
struct Prec<2> {
  static constexpr int KI = 4, KK = 16, NPC = 2;
  typedef f16x4 V;
  typedef _Float16 E;
};
template <>
struct Prec<3> {
  static constexpr int KI = 4, KK = 16, NPC = 2;
  typedef bf16x4 V;
  typedef __bf16 E;
};
template <>
struct Prec<4> {
  static constexpr int KI = 4, KK = 16, NPC = 3;
  typedef bf16x4 V;
  typedef __bf16 E;
};

// Power of two that brings a column maximum m into [2^14, 2^15) (1 for m = 0).
__device__ __forceinline__ float col_scale(float m) {
  if (!(m > 0.f)) return 1.f;
  int e;
  frexpf(m, &e);
  e = 15 - e;
  e = e < -120 ? -120 : (e > 120 ? 120 : e);
  return ldexpf(1.f, e);
}
// Maximum over the four lanes of a column (lanes n, n+16, n+32, n+48).
__device__ __forceinline__ float col_max(float m) {
  m = fmaxf(m, __shfl_xor(m, 16));
  return fmaxf(m, __shfl_xor(m, 32));
}
// Split of KI scaled values into NPC pieces of the precision's element type:
// each piece is the rounding of what the previous pieces leave.
template <class PR>
__device__ __forceinline__ void split_pieces(const float (&v)[PR::KI], float sc, typename PR::V (&pc)[PR::NPC]) {
  typedef typename PR::E E;
#pragma unroll
  for (int i = 0; i < PR::KI; ++i) {
    float x = v[i] * sc;
#pragma unroll
    for (int q = 0; q < PR::NPC; ++q) {
      const E h = (E)x;
      pc[q][i] = h;
      x -= (float)h;
    }
  }
}

// acc += A B over the split pieces: the products of pieces (qa, qb) with
// qa + qb < NPC (two pieces: hi hi, hi lo, lo hi; three pieces: hi hi,
// hi mid, mid hi, hi lo, lo hi, mid mid), smallest terms first.
template <class PR>
__device__ __forceinline__ f32x4 mma_split(const typename PR::V (&a)[PR::NPC], const typename PR::V (&b)[PR::NPC],
                                           f32x4 acc) {
#pragma unroll
  for (int o = PR::NPC - 1; o >= 0; --o)
#pragma unroll
    for (int qa = 0; qa <= o; ++qa) acc = mma_f16(a[qa], b[o - qa], acc);
  return acc;
}

}  // namespace hdg
