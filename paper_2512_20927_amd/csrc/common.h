// Internal helpers shared by the HIP sources of the library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "qrender.h"

namespace qr {

constexpr int kTile = QR_TILE;
constexpr int kTilePix = QR_TILE * QR_TILE;  // 256 pixels, one per thread
constexpr int kWave = 64;

// ---- error reporting (thread-local, host) ---------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
int check_launch(const char* what);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---- feature decoding -----------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// Four OCP e4m3 codes (bytes 0..3 of r, byte 0 first) to float32, times s.
// gfx950's v_cvt_pk_f32_fp8 decodes two OCP e4m3 values (subnormals
// included) per instruction.
__device__ __forceinline__ float4 e4m3x4_to_f32(uint32_t r, float s) {
  typedef float f32x2_ __attribute__((ext_vector_type(2)));
  const f32x2_ lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(r), false);
  const f32x2_ hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(r), true);
  return make_float4(lo.x * s, lo.y * s, hi.x * s, hi.y * s);
}

// Loads 4 consecutive features (d .. d+3, d % 4 == 0) of row g as float32.
template <int DT>
__device__ __forceinline__ float4 load_feat4(const void* __restrict__ feats,
                                             const float* __restrict__ scale,
                                             int64_t g, int dim, int d) {
  if constexpr (DT == QR_F32) {
    return *reinterpret_cast<const float4*>(static_cast<const float*>(feats) + g * dim + d);
  } else if constexpr (DT == QR_BF16) {
    const uint2 r = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(feats) + g * dim + d);
    return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xFFFF0000u),
                       __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xFFFF0000u));
  } else {
    const uint32_t r = *reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(feats) + g * dim + d);
    const float s = scale[g];
    return e4m3x4_to_f32(r, s);
  }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Exclusive scan of one value per thread across a 256-thread workgroup (four
// wave64s): shuffle scan inside each wave, wave totals through `lds4` (four
// words of LDS). Optionally returns the workgroup total. Contains barriers:
// every thread of the workgroup must call it.
__device__ __forceinline__ uint32_t block_scan_exclusive(uint32_t v, uint32_t* lds4,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) lds4[wave] = inc;
  __syncthreads();
  uint32_t wave_base = 0;
  for (int w = 0; w < wave; ++w) wave_base += lds4[w];
  if (total) *total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return wave_base + inc - v;
}

}  // namespace qr
