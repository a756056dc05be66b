// De-voxelisation: per-Gaussian features as the elementwise max (or mean) of
// the predictions of the voxels a Gaussian covers (the step that produces the
// feature table the renderer reads; Appendix, de-voxelisation), and its
// backward. Gaussian g owns voxel slots [offsets[g], offsets[g+1]); slot m
// reads row voxel_unique[m] of the unique-voxel prediction table.
//
// One wave per Gaussian, lanes across the feature columns (four per lane per
// pass); the slot -> row indices are wave-uniform (scalar loads), the rows
// are gathered four slots at a time so their loads overlap. Slots whose index
// is outside [0, n_unique), and offsets outside [0, n_slots], are ignored
// (bounds-checked in the kernel).
#include "common.h"

namespace qr {

constexpr int kDvWaves = 4;  // Gaussians per workgroup

__device__ __forceinline__ void devox_range(const int64_t* __restrict__ offsets, int64_t g,
                                            int64_t n_slots, int64_t& lo, int64_t& hi) {
  lo = min(max(offsets[g], static_cast<int64_t>(0)), n_slots);
  hi = min(max(offsets[g + 1], lo), n_slots);
}

template <int REDUCE>
__global__ void __launch_bounds__(64 * kDvWaves)
devoxelize_kernel(int64_t n_gauss, int dim, const int64_t* __restrict__ offsets,
                  const int32_t* __restrict__ voxel_unique, int64_t n_slots, int64_t n_unique,
                  const float* __restrict__ pred, float* __restrict__ out,
                  int32_t* __restrict__ argmax) {
  const int lane = threadIdx.x & 63;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kDvWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (g >= n_gauss) return;
  int64_t lo, hi;
  devox_range(offsets, g, n_slots, lo, hi);
  const int dim4 = dim >> 2;
  for (int c4 = lane; c4 < dim4; c4 += 64) {
    float4 best = make_float4(0.f, 0.f, 0.f, 0.f);
    int4 bi = make_int4(-1, -1, -1, -1);
    int cnt = 0;
    for (int64_t m0 = lo; m0 < hi; m0 += 4) {
      float4 r[4];
      bool ok[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // loads of four slots issued together
        const int64_t m = m0 + u;
        const int vi = m < hi ? __builtin_amdgcn_readfirstlane(voxel_unique[m]) : -1;
        ok[u] = m < hi && vi >= 0 && vi < n_unique;
        r[u] = ok[u] ? reinterpret_cast<const float4*>(pred + static_cast<int64_t>(vi) * dim)[c4]
                     : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!ok[u]) continue;
        const int m = static_cast<int>(m0 + u);
        if (REDUCE == QR_REDUCE_MAX) {
          if (cnt == 0 || r[u].x > best.x) { best.x = r[u].x; bi.x = m; }
          if (cnt == 0 || r[u].y > best.y) { best.y = r[u].y; bi.y = m; }
          if (cnt == 0 || r[u].z > best.z) { best.z = r[u].z; bi.z = m; }
          if (cnt == 0 || r[u].w > best.w) { best.w = r[u].w; bi.w = m; }
        } else {
          best.x += r[u].x;
          best.y += r[u].y;
          best.z += r[u].z;
          best.w += r[u].w;
        }
        ++cnt;
      }
    }
    if (REDUCE == QR_REDUCE_MEAN && cnt > 0) {
      const float inv = 1.f / static_cast<float>(cnt);
      best = make_float4(best.x * inv, best.y * inv, best.z * inv, best.w * inv);
    }
    reinterpret_cast<float4*>(out + g * dim)[c4] = best;
    if (REDUCE == QR_REDUCE_MAX && argmax) reinterpret_cast<int4*>(argmax + g * dim)[c4] = bi;
  }
}

template <int REDUCE>
__global__ void __launch_bounds__(64 * kDvWaves)
devoxelize_backward_kernel(int64_t n_gauss, int dim, const int64_t* __restrict__ offsets,
                           const int32_t* __restrict__ voxel_unique, int64_t n_slots,
                           int64_t n_unique, const float* __restrict__ grad_out,
                           const int32_t* __restrict__ argmax, float* __restrict__ grad_pred) {
  const int lane = threadIdx.x & 63;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kDvWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (g >= n_gauss) return;
  int64_t lo, hi;
  devox_range(offsets, g, n_slots, lo, hi);
  if (hi == lo) return;
  if (REDUCE == QR_REDUCE_MAX) {
    for (int c = lane; c < dim; c += 64) {
      const int m = argmax[g * dim + c];
      if (m < lo || m >= hi) continue;
      const int vi = voxel_unique[m];
      if (vi < 0 || vi >= n_unique) continue;
      atomicAdd(&grad_pred[static_cast<int64_t>(vi) * dim + c], grad_out[g * dim + c]);
    }
  } else {
    int cnt = 0;
    for (int64_t m = lo; m < hi; ++m) {
      const int vi = __builtin_amdgcn_readfirstlane(voxel_unique[m]);
      cnt += (vi >= 0 && vi < n_unique) ? 1 : 0;
    }
    if (cnt == 0) return;
    const float inv = 1.f / static_cast<float>(cnt);
    for (int64_t m = lo; m < hi; ++m) {
      const int vi = __builtin_amdgcn_readfirstlane(voxel_unique[m]);
      if (vi < 0 || vi >= n_unique) continue;
      for (int c = lane; c < dim; c += 64)
        atomicAdd(&grad_pred[static_cast<int64_t>(vi) * dim + c], grad_out[g * dim + c] * inv);
    }
  }
}

inline int validate_devox(const char* name, int64_t n_gauss, int32_t dim, const int64_t* offsets,
                          const int32_t* voxel_unique, int64_t n_slots, int64_t n_unique,
                          int32_t reduce) {
  if (n_gauss < 0 || n_slots < 0 || n_unique < 0) return fail(QR_ERR_INVALID_ARG, "%s: negative count", name);
  if (n_gauss > (1ll << 31) * kDvWaves || n_slots >= (1ll << 31))
    return fail(QR_ERR_UNSUPPORTED, "%s: too many Gaussians or slots", name);
  if (dim <= 0 || dim % 4 != 0 || dim > QR_MAX_DIM)
    return fail(QR_ERR_UNSUPPORTED, "%s: dim = %d must be a positive multiple of 4 <= %d", name, dim, QR_MAX_DIM);
  if (reduce != QR_REDUCE_MAX && reduce != QR_REDUCE_MEAN)
    return fail(QR_ERR_UNSUPPORTED, "%s: unknown reduction %d", name, reduce);
  if (n_gauss > 0 && !offsets) return fail(QR_ERR_INVALID_ARG, "%s: null offsets", name);
  if (n_slots > 0 && !voxel_unique) return fail(QR_ERR_INVALID_ARG, "%s: null voxel_unique", name);
  return QR_OK;
}

}  // namespace qr

using namespace qr;

extern "C" int qr_devoxelize(void* stream, int64_t n_gauss, int32_t dim, const int64_t* offsets,
                             const int32_t* voxel_unique, int64_t n_slots, int64_t n_unique,
                             const float* unique_pred, int32_t reduce, float* out,
                             int32_t* argmax) {
  int rc = validate_devox("qr_devoxelize", n_gauss, dim, offsets, voxel_unique, n_slots, n_unique, reduce);
  if (rc != QR_OK) return rc;
  if (n_gauss == 0) return QR_OK;
  if (!out || (n_unique > 0 && !unique_pred))
    return fail(QR_ERR_INVALID_ARG, "qr_devoxelize: null array pointer");
  hipStream_t s = as_stream(stream);
  const dim3 grid(static_cast<unsigned>((n_gauss + kDvWaves - 1) / kDvWaves));
  if (reduce == QR_REDUCE_MAX)
    hipLaunchKernelGGL(devoxelize_kernel<QR_REDUCE_MAX>, grid, dim3(64 * kDvWaves), 0, s, n_gauss, dim,
                       offsets, voxel_unique, n_slots, n_unique, unique_pred, out, argmax);
  else
    hipLaunchKernelGGL(devoxelize_kernel<QR_REDUCE_MEAN>, grid, dim3(64 * kDvWaves), 0, s, n_gauss, dim,
                       offsets, voxel_unique, n_slots, n_unique, unique_pred, out, nullptr);
  return check_launch("qr_devoxelize");
}

extern "C" int qr_devoxelize_backward(void* stream, int64_t n_gauss, int32_t dim,
                                      const int64_t* offsets, const int32_t* voxel_unique,
                                      int64_t n_slots, int64_t n_unique, int32_t reduce,
                                      const float* grad_out, const int32_t* argmax,
                                      float* grad_unique) {
  int rc = validate_devox("qr_devoxelize_backward", n_gauss, dim, offsets, voxel_unique, n_slots,
                          n_unique, reduce);
  if (rc != QR_OK) return rc;
  if (n_gauss == 0) return QR_OK;
  if (!grad_out || !grad_unique || (reduce == QR_REDUCE_MAX && !argmax))
    return fail(QR_ERR_INVALID_ARG, "qr_devoxelize_backward: null array pointer");
  hipStream_t s = as_stream(stream);
  const dim3 grid(static_cast<unsigned>((n_gauss + kDvWaves - 1) / kDvWaves));
  if (reduce == QR_REDUCE_MAX)
    hipLaunchKernelGGL(devoxelize_backward_kernel<QR_REDUCE_MAX>, grid, dim3(64 * kDvWaves), 0, s,
                       n_gauss, dim, offsets, voxel_unique, n_slots, n_unique, grad_out, argmax,
                       grad_unique);
  else
    hipLaunchKernelGGL(devoxelize_backward_kernel<QR_REDUCE_MEAN>, grid, dim3(64 * kDvWaves), 0, s,
                       n_gauss, dim, offsets, voxel_unique, n_slots, n_unique, grad_out, nullptr,
                       grad_unique);
  return check_launch("qr_devoxelize_backward");
}
