// Quantile Rendering forward (Algorithm 1, Sec. 4.2).
//
// One workgroup per 16x16 tile, one thread per pixel (4 wave64s).
// Phase 1 (selection): the tile's depth-sorted list is staged into LDS in
// batches of 256 projected records; every pixel walks it front to back with
// the transmittance chain T_test = T (1 - alpha') and the threshold test
// T_test < t_{k+1}, recording the <= K selected (Gaussian id, w^Q) pairs in
// LDS. A pixel is done once all K thresholds are consumed (the paper's stop
// test T_test < 1/(K+1) is the same event), and the whole workgroup leaves the
// list as soon as every pixel is done.
// Phase 2 (gather-blend): each wave takes four pixels at a time, its lanes
// spanning the feature dimension; the <= K selected feature rows of all four
// are requested together (mostly L2 hits: neighbouring pixels select the same
// Gaussians), accumulated in float32, scaled by 1 / (1 - T^Q), and streamed
// to the [H, W, D] map with non-temporal stores. The map write is the dominant HBM
// traffic of the whole pipeline.
#include "common.h"
#include "render_common.h"

namespace qr {

template <int DT>
__global__ void __launch_bounds__(kTilePix)
render_quantile_kernel(int W, int H, int tiles_x, int n_tiles, qr_params prm, int K,
                       const uint32_t* __restrict__ tile_offsets,
                       const uint32_t* __restrict__ sorted_gid,
                       const float2* __restrict__ means2d, const float4* __restrict__ conic_opacity,
                       const void* __restrict__ feats, const float* __restrict__ scale, int dim,
                       float* __restrict__ out, float* __restrict__ T_q_out,
                       int32_t* __restrict__ n_sel_out, int32_t* __restrict__ sel_gid_out,
                       float* __restrict__ sel_w_out) {
  extern __shared__ unsigned char dyn_lds[];
  int* s_sel_gid = reinterpret_cast<int*>(dyn_lds);                 // [256][K]
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + kTilePix * K;  // [256][K]
  __shared__ float2 s_mean[kTilePix];
  __shared__ float4 s_co[kTilePix];
  __shared__ int s_gid[kTilePix];
  __shared__ float s_thr[QR_MAX_K + 1];
  __shared__ float s_inv[kTilePix];
  __shared__ int s_ns[kTilePix];

  const int tid = threadIdx.x;
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid % kTile);
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;

  if (tid <= K) s_thr[tid] = quantile_threshold(tid + 1, K);  // s_thr[k] = t_{k+1}; s_thr[K] = 0

  const int lo = static_cast<int>(tile_offsets[tile]);
  const int hi = static_cast<int>(tile_offsets[tile + 1]);

  float T = 1.f, TQ = 1.f;
  int k = 0, ns = 0;
  bool done = !inside;
  int* my_gid = s_sel_gid + tid * K;
  float* my_w = s_sel_w + tid * K;

  for (int batch = lo; batch < hi; batch += kTilePix) {
    if (__syncthreads_count(!done) == 0) break;
    const int idx = batch + tid;
    if (idx < hi) {
      const int g = static_cast<int>(sorted_gid[idx]);
      s_gid[tid] = g;
      s_mean[tid] = means2d[g];
      s_co[tid] = conic_opacity[g];
    }
    __syncthreads();
    const int cnt = min(kTilePix, hi - batch);
    for (int j = 0; j < cnt && !done; ++j) {
      const float alpha = gauss_alpha(s_mean[j], s_co[j], pxc, pyc, prm.alpha_max);
      if (alpha < prm.alpha_min) continue;  // not on this pixel's ray
      const float T_test = T * (1.f - alpha);
      if (T_test < s_thr[k]) {  // crossing: a quantile Gaussian
        my_gid[ns] = s_gid[j];
        my_w[ns] = TQ * alpha;
        ++ns;
        TQ = TQ * (1.f - alpha);
        ++k;
        while (k < K && T_test < s_thr[k]) ++k;  // thresholds crossed by the same step
        if (k == K) done = true;
      }
      T = T_test;
    }
  }
  if (inside) {
    const int pix = py * W + px;
    if (T_q_out) T_q_out[pix] = TQ;
    if (n_sel_out) n_sel_out[pix] = ns;
    if (sel_gid_out) {
      for (int j = 0; j < K; ++j) {
        sel_gid_out[static_cast<int64_t>(pix) * K + j] = j < ns ? my_gid[j] : -1;
        sel_w_out[static_cast<int64_t>(pix) * K + j] = j < ns ? my_w[j] : 0.f;
      }
    }
  }
  s_ns[tid] = inside ? ns : -1;
  s_inv[tid] = ns > 0 ? 1.f / (1.f - TQ) : 0.f;
  __syncthreads();

  // Phase 2: gather-blend. Wave w owns pixels [64 w, 64 w + 64) and takes
  // them kPG at a time; lanes span the feature dimension. Every selected row
  // of the kPG pixels is requested before any is accumulated (rows of pixels
  // with fewer selections are padded with weight 0 and a valid row of the
  // group), so each lane keeps 2 kPG independent loads in flight.
  constexpr int kPG = 4;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int dim4 = dim >> 2;
  for (int p0 = wave * 64; p0 < wave * 64 + 64; p0 += kPG) {
    int n[kPG];
    int nmax = 0, safe = 0;
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      n[q] = s_ns[p0 + q];
      if (n[q] > nmax) {
        nmax = n[q];
        safe = s_sel_gid[(p0 + q) * K];
      }
    }
    for (int c = lane; c < dim4; c += 64) {
      float4 acc[kPG];
#pragma unroll
      for (int q = 0; q < kPG; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int j = 0; j < nmax; ++j) {
        float4 f[kPG];
        float w[kPG];
#pragma unroll
        for (int q = 0; q < kPG; ++q) {
          const bool ok = j < n[q];
          const int g = ok ? s_sel_gid[(p0 + q) * K + j] : safe;
          w[q] = ok ? s_sel_w[(p0 + q) * K + j] : 0.f;
          f[q] = load_feat4<DT>(feats, scale, g, dim, 4 * c);
        }
#pragma unroll
        for (int q = 0; q < kPG; ++q) {
          acc[q].x += w[q] * f[q].x;
          acc[q].y += w[q] * f[q].y;
          acc[q].z += w[q] * f[q].z;
          acc[q].w += w[q] * f[q].w;
        }
      }
#pragma unroll
      for (int q = 0; q < kPG; ++q) {
        if (n[q] < 0) continue;  // outside the image
        const int p = p0 + q;
        const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
        float4* dst = reinterpret_cast<float4*>(out + (static_cast<int64_t>(gy) * W + gx) * dim);
        const float inv = s_inv[p];
        store_stream(dst + c, make_float4(acc[q].x * inv, acc[q].y * inv, acc[q].z * inv, acc[q].w * inv));
      }
    }
  }
}

}  // namespace qr

using namespace qr;

extern "C" int qr_render_quantile(void* stream, int32_t width, int32_t height,
                                  const qr_params* prm, int32_t K, const uint32_t* tile_offsets,
                                  const uint32_t* sorted_gid, const float* means2d,
                                  const float* conic_opacity, const void* features, int32_t dtype,
                                  const float* feature_scale, int32_t dim, float* out, float* T_q,
                                  int32_t* n_sel, int32_t* sel_gid, float* sel_w) {
  int rc = validate_render("qr_render_quantile", width, height, prm, tile_offsets, sorted_gid,
                           means2d, conic_opacity, features, dtype, feature_scale, dim, out);
  if (rc != QR_OK) return rc;
  if (K < 1 || K > QR_MAX_K)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile: K = %d outside [1, %d]", K, QR_MAX_K);
  if ((sel_gid == nullptr) != (sel_w == nullptr))
    return fail(QR_ERR_INVALID_ARG, "qr_render_quantile: sel_gid and sel_w must both be given or both NULL");
  const int tiles_x = static_cast<int>(ceil_div(width, kTile));
  const int tiles_y = static_cast<int>(ceil_div(height, kTile));
  const int n_tiles = tiles_x * tiles_y;
  const size_t lds = static_cast<size_t>(kTilePix) * K * (sizeof(int) + sizeof(float));
  hipStream_t s = as_stream(stream);
#define QR_LAUNCH(DT)                                                                             \
  hipLaunchKernelGGL(render_quantile_kernel<DT>, dim3(n_tiles), dim3(kTilePix), lds, s, width,    \
                     height, tiles_x, n_tiles, *prm, K, tile_offsets, sorted_gid,                 \
                     reinterpret_cast<const float2*>(means2d),                                    \
                     reinterpret_cast<const float4*>(conic_opacity), features, feature_scale, dim, \
                     out, T_q, n_sel, sel_gid, sel_w)
  switch (dtype) {
    case QR_F32: QR_LAUNCH(QR_F32); break;
    case QR_BF16: QR_LAUNCH(QR_BF16); break;
    default: QR_LAUNCH(QR_FP8_E4M3); break;
  }
#undef QR_LAUNCH
  return check_launch("qr_render_quantile");
}
