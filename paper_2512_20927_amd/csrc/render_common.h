// Helpers shared by the forward and backward renderers.
#pragma once

#include "common.h"

namespace qr {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2. Remap so that XCD x receives a contiguous run of tiles:
// neighbouring tiles share most of their Gaussians (records and feature
// rows), which then hit the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int xcd = bid % kXcd;
  const int slot = bid / kXcd;
  const int per = nblocks / kXcd;
  const int rem = nblocks % kXcd;
  return xcd * per + min(xcd, rem) + slot;
}

// t_m = 1 - m/(K+1) evaluated in double and rounded once to float;
// m = K+1 gives 0, a threshold no transmittance falls below.
__device__ __forceinline__ float quantile_threshold(int m, int K) {
  return static_cast<float>(1.0 - static_cast<double>(m) / static_cast<double>(K + 1));
}

// Stratified-K threshold t_m = clip(mu + sigma z_m, 0, 1) with
// z_m = Phi^-1(1 - m/(K+1)), in double, rounded once to float. z_m depends on
// m and K only, so the walk computes it once per tile (stratified_z) and
// forms t_m per ray from it.
__device__ __forceinline__ double stratified_z(int m, int K) {
  return normcdfinv(1.0 - static_cast<double>(m) / static_cast<double>(K + 1));
}
__device__ __forceinline__ float stratified_threshold_z(double z, double mu, double sigma) {
  const double t = mu + sigma * z;
  return static_cast<float>(fmin(fmax(t, 0.0), 1.0));
}

// alpha' = min(alpha_max, o exp(power)), power = -(a dx^2 + 2 b dx dy + c dy^2)/2,
// with every multiply-add written out so that forward and backward kernels
// evaluate bit-identical values.
struct AlphaEval {
  float alpha, G, dx, dy;
  bool clamped;
};

__device__ __forceinline__ AlphaEval eval_alpha(float2 mean, float4 co, float pxc, float pyc,
                                                float alpha_max) {
  AlphaEval r;
  r.dx = pxc - mean.x;
  r.dy = pyc - mean.y;
  const float cross2 = ((2.f * co.y) * r.dx) * r.dy;  // products only: nothing to contract
  const float q = fmaf(co.x * r.dx, r.dx, fmaf(co.z * r.dy, r.dy, cross2));
  // G = exp(-q/2) = 2^(-q log2(e) / 2): one hardware v_exp_f32 (about one ulp;
  // the rounding of the scaled exponent adds |q| 2^-25 relative)
  constexpr float kNegHalfLog2e = -0.72134752044448170368f;
  r.G = __builtin_amdgcn_exp2f(q * kNegHalfLog2e);
  const float raw = co.w * r.G;
  r.clamped = raw >= alpha_max;
  r.alpha = r.clamped ? alpha_max : raw;
  return r;
}

__device__ __forceinline__ float gauss_alpha(float2 mean, float4 co, float pxc, float pyc,
                                             float alpha_max) {
  return eval_alpha(mean, co, pxc, pyc, alpha_max).alpha;
}

__device__ __forceinline__ void store_stream(float4* p, float4 v) {
  f32x4 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<f32x4*>(p));
}

// Global-memory (address space 1) pointers. Accesses through a pointer that
// was itself read from memory (a per-view record) compile to flat_*
// instructions, which also count against the LDS counter and so add waits to
// every LDS access; through these they compile to global_* instructions.
#define QR_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ void store_stream(QR_GLOBAL float4* p, float4 v) {
  f32x4 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<QR_GLOBAL f32x4*>(p));
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// load_feat4 through global pointers (native vector types: HIP's vector
// classes cannot be copied out of another address space).
template <int DT>
__device__ __forceinline__ float4 load_feat4_global(const QR_GLOBAL void* __restrict__ feats,
                                                    const QR_GLOBAL float* __restrict__ scale,
                                                    int64_t g, int dim, int d) {
  if constexpr (DT == QR_F32) {
    const f32x4 x = *reinterpret_cast<const QR_GLOBAL f32x4*>(
        static_cast<const QR_GLOBAL float*>(feats) + g * dim + d);
    return make_float4(x.x, x.y, x.z, x.w);
  } else if constexpr (DT == QR_BF16) {
    const u32x2 r = *reinterpret_cast<const QR_GLOBAL u32x2*>(
        static_cast<const QR_GLOBAL uint16_t*>(feats) + g * dim + d);
    return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xFFFF0000u),
                       __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xFFFF0000u));
  } else {
    const uint32_t r = *reinterpret_cast<const QR_GLOBAL uint32_t*>(
        static_cast<const QR_GLOBAL uint8_t*>(feats) + g * dim + d);
    const float s = scale[g];
    return e4m3x4_to_f32(r, s);
  }
}

// Host-side validation shared by the render entry points (callers that write
// float32 only also check prm->out_dtype == QR_F32 themselves).
inline int validate_render(const char* name, int32_t width, int32_t height, const qr_params* prm,
                           const uint32_t* tile_offsets, const uint32_t* sorted_gid,
                           const float* means2d, const float* conic_opacity, const void* features,
                           int32_t dtype, const float* feature_scale, int32_t dim,
                           const void* out) {
  if (width <= 0 || height <= 0) return fail(QR_ERR_INVALID_ARG, "%s: image size must be positive", name);
  if (static_cast<int64_t>(ceil_div(width, kTile)) * ceil_div(height, kTile) >= (1ll << 31))
    return fail(QR_ERR_UNSUPPORTED, "%s: image too large", name);
  if (!prm) return fail(QR_ERR_INVALID_ARG, "%s: null params", name);
  if (!(prm->alpha_min > 0.f) || !(prm->alpha_max >= prm->alpha_min) || !(prm->alpha_max < 1.f))
    return fail(QR_ERR_INVALID_ARG, "%s: need 0 < alpha_min <= alpha_max < 1", name);
  if (!(prm->T_eps >= 0.f)) return fail(QR_ERR_INVALID_ARG, "%s: T_eps must be >= 0", name);
  if (prm->out_dtype != QR_F32 && prm->out_dtype != QR_BF16)
    return fail(QR_ERR_UNSUPPORTED, "%s: unknown output dtype %d", name, prm->out_dtype);
  if (prm->selection != QR_SELECT_QUANTILE && prm->selection != QR_SELECT_STRATIFIED &&
      prm->selection != QR_SELECT_TOPK)
    return fail(QR_ERR_UNSUPPORTED, "%s: unknown selection rule %d", name, prm->selection);
  if (!tile_offsets || !sorted_gid || !means2d || !conic_opacity || !features || !out)
    return fail(QR_ERR_INVALID_ARG, "%s: null array pointer", name);
  if (dtype != QR_F32 && dtype != QR_BF16 && dtype != QR_FP8_E4M3)
    return fail(QR_ERR_UNSUPPORTED, "%s: unknown feature dtype %d", name, dtype);
  if (dtype == QR_FP8_E4M3 && !feature_scale)
    return fail(QR_ERR_INVALID_ARG, "%s: FP8 features need a per-Gaussian scale", name);
  if (dim <= 0 || dim % 16 != 0 || dim > QR_MAX_DIM)
    return fail(QR_ERR_UNSUPPORTED, "%s: dim = %d must be a positive multiple of 16 <= %d", name,
                dim, QR_MAX_DIM);
  return QR_OK;
}

}  // namespace qr
