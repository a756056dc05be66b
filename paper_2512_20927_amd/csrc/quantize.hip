// Storage encoders for the feature table: bfloat16 and OCP FP8 e4m3 with a
// per-Gaussian float32 scale. Both renderers decode these in their load path
// and accumulate in float32.
#include "common.h"

namespace qr {

// float32 -> bfloat16 bits, round to nearest, ties to even.
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  return static_cast<uint16_t>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// |x| <= 448 (finite) -> e4m3 code, nearest with ties to even.
// Normal range: round the float32 pattern to 3 mantissa bits (the carry may
// bump the exponent) and rebias the exponent from 127 to 7. Below 2^-6 the
// e4m3 grid is uniform with step 2^-9, so the code is rint(|x| * 2^9).
__device__ __forceinline__ uint32_t f32_to_e4m3(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float mag = fminf(fabsf(x), 448.f);
  uint32_t code;
  if (mag < 0.015625f) {
    code = static_cast<uint32_t>(rintf(mag * 512.f));
  } else {
    const uint32_t b = __float_as_uint(mag);
    const uint32_t r = (b + 0x7FFFFu + ((b >> 20) & 1u)) >> 20;
    code = r - (120u << 3);
  }
  return sign | code;
}

__global__ void __launch_bounds__(256)
quantize_bf16_kernel(int64_t count, const float* __restrict__ f, uint16_t* __restrict__ out) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i < count) out[i] = f32_to_bf16(f[i]);
}

// one wave64 per row: max |f| -> scale, then the codes of f / scale
__global__ void __launch_bounds__(256)
quantize_e4m3_kernel(int64_t n, int dim, const float* __restrict__ f, uint8_t* __restrict__ out,
                     float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t row = blockIdx.x * 4LL + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* fr = f + row * dim;
  float m = 0.f;
  for (int d = lane; d < dim; d += 64) m = fmaxf(m, fabsf(fr[d]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  const float s = m > 0.f ? m / 448.f : 1.f;
  if (lane == 0) scale[row] = s;
  uint8_t* orow = out + row * dim;
  for (int d = lane; d < dim; d += 64) orow[d] = static_cast<uint8_t>(f32_to_e4m3(fr[d] / s));
}

}  // namespace qr

using namespace qr;

extern "C" int qr_quantize_features(void* stream, int64_t n, int32_t dim, const float* features,
                                    int32_t dtype, void* out, float* scale) {
  if (n < 0 || dim <= 0) return fail(QR_ERR_INVALID_ARG, "qr_quantize_features: bad sizes");
  if (dtype != QR_BF16 && dtype != QR_FP8_E4M3)
    return fail(QR_ERR_UNSUPPORTED, "qr_quantize_features: dtype must be QR_BF16 or QR_FP8_E4M3");
  if (n == 0) return QR_OK;
  if (!features || !out) return fail(QR_ERR_INVALID_ARG, "qr_quantize_features: null pointer");
  if (dtype == QR_FP8_E4M3 && !scale)
    return fail(QR_ERR_INVALID_ARG, "qr_quantize_features: FP8 needs a scale array");
  hipStream_t s = as_stream(stream);
  if (dtype == QR_BF16) {
    const int64_t count = n * dim;
    hipLaunchKernelGGL(quantize_bf16_kernel, dim3(static_cast<unsigned>(ceil_div(count, 256))),
                       dim3(256), 0, s, count, features, static_cast<uint16_t*>(out));
  } else {
    hipLaunchKernelGGL(quantize_e4m3_kernel, dim3(static_cast<unsigned>(ceil_div(n, 4))), dim3(256),
                       0, s, n, dim, features, static_cast<uint8_t*>(out), scale);
  }
  return check_launch("qr_quantize_features");
}
