// Wave-level helpers of the backward kernels: a sum over the 64 lanes
// without LDS, and the bfloat16 pair split that lets float32 operands run
// on the bf16 matrix cores.
#pragma once

#include "common.h"

namespace qr {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int kCtrl>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl,
                                                               0xF, 0xF, false));
}

__device__ __forceinline__ uint32_t fbits(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float bitsf(uint32_t x) { return __builtin_bit_cast(float, x); }

// Sum over the 64 lanes (every lane returns the total): v_permlane32_swap
// exchanges lanes 32..63 of its first operand with lanes 0..31 of its
// second and v_permlane16_swap odd with even 16-lane rows, so adding the two
// results of a self-swap folds the halves, then the rows; DPP moves finish
// inside the 16-lane rows. All lanes must be active.
__device__ __forceinline__ float wave_sum(float x) {
  const auto a = __builtin_amdgcn_permlane32_swap(fbits(x), fbits(x), false, false);
  float k = bitsf(a[0]) + bitsf(a[1]);
  const auto b = __builtin_amdgcn_permlane16_swap(fbits(k), fbits(k), false, false);
  k = bitsf(b[0]) + bitsf(b[1]);
  k += dpp<0xB1>(k);   // quad_perm [1,0,3,2]
  k += dpp<0x4E>(k);   // quad_perm [2,3,0,1]
  k += dpp<0x124>(k);  // row_ror:4
  k += dpp<0x128>(k);  // row_ror:8
  return k;
}

// Transposed wave sums: many per-lane values are summed over the 64 lanes so
// that lane l ends with the total of value l. Each stage pairs lanes that
// differ in one bit of the lane index and halves the live registers: of two
// registers (a, b) a lane keeps a if its bit is 0, b if it is 1, and adds the
// partner's copy of the same register. Bits 5 and 4 pair lane halves and
// 16-lane rows (v_permlane32_swap: upper 32 lanes of the first operand with
// the lower 32 of the second; v_permlane16_swap: odd rows of the first with
// even rows of the second); bits 3..0 pair lane i with i ^ 15, i ^ 7, i ^ 2
// and i ^ 1 inside each row (DPP row_mirror, row_half_mirror and two quad
// permutations). All lanes must be active.
__device__ __forceinline__ float tsum_bit5(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(fbits(a), fbits(b), false, false);
  return bitsf(r[0]) + bitsf(r[1]);
}
__device__ __forceinline__ float tsum_bit4(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(fbits(a), fbits(b), false, false);
  return bitsf(r[0]) + bitsf(r[1]);
}
template <int kCtrl>
__device__ __forceinline__ float tsum_dpp(float a, float b, bool bit) {
  const float send = bit ? a : b;
  return (bit ? b : a) + dpp<kCtrl>(send);
}
// The last four stages: register k of r4 holds, in a lane with bits 5 and 4
// equal to (b5, b4), the sum of value k + 16 b4 + 32 b5 over the four lanes
// that share the lane's bits 3..0. Returns lane l's total of value l.
__device__ __forceinline__ float tsum_rows(const float (&r4)[16], int lane) {
  float r3[8], r2[4], r1[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) r3[k] = tsum_dpp<0x140>(r4[k], r4[k + 8], lane & 8);  // row_mirror
#pragma unroll
  for (int k = 0; k < 4; ++k) r2[k] = tsum_dpp<0x141>(r3[k], r3[k + 4], lane & 4);  // row_half_mirror
#pragma unroll
  for (int k = 0; k < 2; ++k) r1[k] = tsum_dpp<0x4E>(r2[k], r2[k + 2], lane & 2);   // quad_perm [2,3,0,1]
  return tsum_dpp<0xB1>(r1[0], r1[1], lane & 1);                                    // quad_perm [1,0,3,2]
}

// x = hi + lo with hi the bf16 rounding of x and lo that of the remainder.
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const __bf16 h = static_cast<__bf16>(x[i]);
    hi[i] = h;
    lo[i] = static_cast<__bf16>(x[i] - static_cast<float>(h));
  }
}

// acc += A B for split operands: hi.hi + lo.hi + hi.lo (the lo.lo term is
// below 2^-16 of the product).
__device__ __forceinline__ void mfma3(floatx4& acc, const bf16x8& ahi, const bf16x8& alo,
                                      const bf16x8& bhi, const bf16x8& blo) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
}

}  // namespace qr
