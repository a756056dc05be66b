// Backward pass of the dense blend (Eq. 1): gradients with respect to the
// decoded float32 features, the 2D means, the conics (a, b, c) and the
// opacities. (The Quantile Rendering backward is in
// render_quantile_backward.hip.)
//
// The kernel re-runs the forward walk of its tile with the identical float32
// arithmetic (same helpers, same operation order), so exactly the entries
// the forward blended are differentiated, and takes transmittances from that
// recomputation instead of stored per-pixel lists.
//
// With g = dL/d(out_p), d_i = <g, f_i>, w_i = T_i alpha'_i, out = sum w f:
//    dL/df_i      = w_i g
//    dL/dalpha'_i = T_i d_i - (<g, out> - sum_{l <= i} w_l d_l) / (1 - alpha'_i)
// and alpha' = o G, G = exp(-(a dx^2 + 2 b dx dy + c dy^2)/2) gives
//    dalpha'/do = G, dalpha'/dpower = alpha' (0 for both if clamped),
//    dpower/da = -dx^2/2, /db = -dx dy, /dc = -dy^2/2,
//    dpower/du = a dx + b dy, /dv = b dx + c dy.
// Per-tile partial sums are accumulated into the caller's gradient arrays
// with float32 atomics.
#include "common.h"
#include "render_common.h"
#include "wave_ops.h"

namespace qr {

constexpr int kCW = 32;          // feature columns staged per chunk
constexpr int kGStride = kCW + 1;  // LDS row stride of the grad_out chunk

// Loads the [256 px x kCW] slice [c0, c0 + kCW) of the tile's grad_out into
// LDS (rows of pixels outside the image, and columns past dim, are zero).
__device__ __forceinline__ void load_grad_chunk(float* s_g, const QR_GLOBAL float* __restrict__ grad_out,
                                                int W, int H, int tx, int ty, int dim, int c0) {
  constexpr int per_row = kCW / 4;
  for (int e = threadIdx.x; e < kTilePix * per_row; e += kTilePix) {
    const int p = e / per_row, c4 = e - p * per_row;
    const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (gx < W && gy < H && c0 + 4 * c4 < dim)  // dim is a multiple of 16, not of kCW
      v = *reinterpret_cast<const QR_GLOBAL f32x4*>(grad_out + (static_cast<int64_t>(gy) * W + gx) * dim + c0 + 4 * c4);
    float* r = s_g + p * kGStride + 4 * c4;
    r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
  }
}

// ============================================================================
// Dense backward. One workgroup per tile, one thread per pixel; the list is
// walked front to back in batches of 32 entries exactly as in the forward.
// For each batch, over 32-column chunks of grad_out staged in LDS, two
// contractions on v_mfma_f32_16x16x32_bf16 (float32 operands split into
// bfloat16 pairs, hi.hi + hi.lo + lo.hi, float32 accumulation):
//   D  = G F^T  [256 px x 32 entries], the dots d_pj = <g_p, f_j> (each wave
//        its 64 pixels, accumulated over the chunks);
//   dF = W^T G  [32 entries x 32 columns] per chunk, W[p][j] = T_pj alpha'_pj
//        (each wave one 16 x 16 block over all 256 pixels), added to
//        grad_features with one atomic per (entry, column);
// then dL/dalpha'_pj uses the prefix sum_{l<=j} w_l d_l against the whole-ray
// total <g_p, out_p>, and each entry's geometric gradient is summed over the
// tile's pixels (wave sums, then the four waves) before one atomic per value.
constexpr int kDB = 32;            // list entries per batch (= MFMA K / N)
constexpr int kWS = kTilePix + 1;  // LDS stride of an entry's weights

template <int DT>
__global__ void __launch_bounds__(kTilePix, 2)
dense_backward_kernel(int W, int H, int tiles_x, int n_tiles, qr_params prm,
                      const uint32_t* __restrict__ tile_offsets,
                      const uint32_t* __restrict__ sorted_gid, const float2* __restrict__ means2d,
                      const float4* __restrict__ conic_opacity, const void* __restrict__ feats,
                      const float* __restrict__ scale, int dim, const float* __restrict__ out,
                      const float* __restrict__ grad_out, float* __restrict__ grad_features,
                      float* __restrict__ grad_means2d, float* __restrict__ grad_co) {
  const QR_GLOBAL void* gfeats = (const QR_GLOBAL void*)feats;
  const QR_GLOBAL float* gscale = (const QR_GLOBAL float*)scale;
  const QR_GLOBAL float* ggrad = (const QR_GLOBAL float*)grad_out;
  QR_GLOBAL float* ggf = (QR_GLOBAL float*)grad_features;
  __shared__ float s_g[kTilePix * kGStride];  // grad_out chunk; later the batch's dots [kDB][kWS]
  __shared__ float s_f[kDB * kGStride];       // feature chunk [entry][column]
  __shared__ float s_w[kDB * kWS];            // weights [entry][pixel]
  __shared__ float2 s_mean[kDB];
  __shared__ float4 s_co[kDB];
  __shared__ int s_gid[kDB];
  __shared__ float s_red[4][kDB][6];  // per wave, entry and value
  __shared__ float s_tot[kTilePix];
  static_assert(kDB * kWS <= kTilePix * kGStride, "dots must fit in the grad_out chunk space");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row = lane & 15, kq = (lane >> 4) * 8;
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid % kTile);
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;
  const int lo = static_cast<int>(tile_offsets[tile]);
  const int hi = static_cast<int>(tile_offsets[tile + 1]);
  if (lo == hi) return;

  // <g_p, out_p> for each pixel: wave per pixel, lanes across D
  for (int p = wave; p < kTilePix; p += 4) {
    const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
    float acc = 0.f;
    if (gx < W && gy < H) {
      const int64_t base = (static_cast<int64_t>(gy) * W + gx) * dim;
      for (int c = lane * 4; c < dim; c += 256) {
        const f32x4 a = *reinterpret_cast<const QR_GLOBAL f32x4*>(ggrad + base + c);
        const f32x4 b = *reinterpret_cast<const QR_GLOBAL f32x4*>((const QR_GLOBAL float*)out + base + c);
        acc += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) s_tot[p] = acc;
  }
  __syncthreads();
  const float total = s_tot[tid];

  float T = 1.f, prefix = 0.f;
  bool done = !inside;
  for (int batch = lo; batch < hi; batch += kDB) {
    if (__syncthreads_count(!done) == 0) break;
    const int cnt = min(kDB, hi - batch);
    if (tid < cnt) {
      const int g = static_cast<int>(sorted_gid[batch + tid]);
      s_gid[tid] = g;
      s_mean[tid] = means2d[g];
      s_co[tid] = conic_opacity[g];
    }
    __syncthreads();
    // forward walk of the batch: this pixel's weights (0 off the ray, after
    // the stop and past the list end)
    for (int j = 0; j < kDB; ++j) {
      float w = 0.f;
      if (j < cnt && !done) {
        const float alpha = gauss_alpha(s_mean[j], s_co[j], pxc, pyc, prm.alpha_max);
        if (alpha >= prm.alpha_min) {
          const float T_test = T * (1.f - alpha);
          if (T_test < prm.T_eps) {
            done = true;
          } else {
            w = alpha * T;
            T = T_test;
          }
        }
      }
      s_w[j * kWS + tid] = w;
    }
    floatx4 dacc[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) dacc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < dim; c0 += kCW) {
      __syncthreads();  // previous chunk consumed (and the weights written)
      load_grad_chunk(s_g, ggrad, W, H, tx, ty, dim, c0);
      {  // feature chunk: entry tid / 8, four columns each
        const int j = tid >> 3, c4 = tid & 7;
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < cnt && c0 + 4 * c4 < dim) f = load_feat4_global<DT>(gfeats, gscale, s_gid[j], dim, c0 + 4 * c4);
        float* r = s_f + j * kGStride + 4 * c4;
        r[0] = f.x; r[1] = f.y; r[2] = f.z; r[3] = f.w;
      }
      __syncthreads();
      // dots: A = G (pixel wave*64 + mb*16 + row, columns kq..kq+7),
      //       B = F^T (columns kq..kq+7, entry nb*16 + row)
      {
        bf16x8 bhi[2], blo[2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          float x[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) x[i] = s_f[(nb * 16 + row) * kGStride + kq + i];
          split8(x, bhi[nb], blo[nb]);
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          float x[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) x[i] = s_g[(wave * 64 + mb * 16 + row) * kGStride + kq + i];
          bf16x8 ahi, alo;
          split8(x, ahi, alo);
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) mfma3(dacc[mb][nb], ahi, alo, bhi[nb], blo[nb]);
        }
      }
      // feature gradients of this chunk: wave w computes the 16 x 16 block
      // (entries 16 (w / 2) .., columns 16 (w % 2) ..) over all pixels
      if (grad_features) {
        const int e0 = (wave >> 1) * 16, n0 = (wave & 1) * 16;
        floatx4 facc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int k0 = 0; k0 < kTilePix; k0 += 32) {
          float a[8], b[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            a[i] = s_w[(e0 + row) * kWS + k0 + kq + i];
            b[i] = s_g[(k0 + kq + i) * kGStride + n0 + row];
          }
          bf16x8 ahi, alo, bhi, blo;
          split8(a, ahi, alo);
          split8(b, bhi, blo);
          mfma3(facc, ahi, alo, bhi, blo);
        }
        // lane holds dF[e0 + 4 (lane / 16) + i][n0 + lane % 16]
        const int col = c0 + n0 + row;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = e0 + 4 * (lane >> 4) + i;
          if (j < cnt && col < dim && facc[i] != 0.f)
            __hip_atomic_fetch_add(ggf + static_cast<int64_t>(s_gid[j]) * dim + col, facc[i],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    // park the dots in the (now free) grad_out chunk space: s_d[entry][pixel]
    __syncthreads();
    float* s_d = s_g;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          s_d[(nb * 16 + row) * kWS + wave * 64 + mb * 16 + 4 * (lane >> 4) + i] = dacc[mb][nb][i];
    __syncthreads();
    // dL/dalpha' and the geometric chain rule per (pixel, entry); each
    // entry's six sums over a wave's pixels go to s_red, and after one
    // barrier per batch, one atomic per (entry, value)
    for (int j = 0; j < cnt; ++j) {  // cnt is uniform across the workgroup
      const float w = s_w[j * kWS + tid];
      float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (w != 0.f) {
        const float dj = s_d[j * kWS + tid];
        prefix += w * dj;
        const AlphaEval e = eval_alpha(s_mean[j], s_co[j], pxc, pyc, prm.alpha_max);
        if (!e.clamped) {
          const float4 co = s_co[j];
          const float T_before = w / e.alpha;  // w = alpha' T
          const float dL_da = T_before * dj - (total - prefix) / (1.f - e.alpha);
          const float dpow = dL_da * e.alpha;
          v[0] = dpow * (-0.5f * e.dx * e.dx);
          v[1] = dpow * (-e.dx * e.dy);
          v[2] = dpow * (-0.5f * e.dy * e.dy);
          v[3] = dL_da * e.G;
          v[4] = dpow * (co.x * e.dx + co.y * e.dy);
          v[5] = dpow * (co.y * e.dx + co.z * e.dy);
        }
      }
      const bool any = __ballot(w != 0.f) != 0ull;  // uniform over the wave
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const float sv = any ? wave_sum(v[q]) : 0.f;
        if (lane == 0) s_red[wave][j][q] = sv;
      }
    }
    __syncthreads();
    for (int i = tid; i < cnt * 6; i += kTilePix) {
      const int j = i / 6, q = i - j * 6;
      const float sv = s_red[0][j][q] + s_red[1][j][q] + s_red[2][j][q] + s_red[3][j][q];
      if (sv == 0.f) continue;
      const int g = s_gid[j];
      if (q < 4) {
        if (grad_co) atomicAdd(&grad_co[4 * g + q], sv);
      } else if (grad_means2d) {
        atomicAdd(&grad_means2d[2 * g + q - 4], sv);
      }
    }
  }
}

inline int validate_backward(const char* name, const float* grad_out) {
  if (!grad_out) return fail(QR_ERR_INVALID_ARG, "%s: null grad_out", name);
  return QR_OK;
}

}  // namespace qr

using namespace qr;

extern "C" int qr_render_dense_backward(void* stream, int32_t width, int32_t height,
                                        const qr_params* prm, const uint32_t* tile_offsets,
                                        const uint32_t* sorted_gid, const float* means2d,
                                        const float* conic_opacity, const void* features,
                                        int32_t dtype, const float* feature_scale, int32_t dim,
                                        const float* out, const float* grad_out,
                                        float* grad_features, float* grad_means2d,
                                        float* grad_conic_opacity) {
  int rc = validate_render("qr_render_dense_backward", width, height, prm, tile_offsets,
                           sorted_gid, means2d, conic_opacity, features, dtype, feature_scale, dim,
                           grad_out);
  if (rc != QR_OK) return rc;
  if (!out) return fail(QR_ERR_INVALID_ARG, "qr_render_dense_backward: null forward output");
  const int tiles_x = static_cast<int>(ceil_div(width, kTile));
  const int tiles_y = static_cast<int>(ceil_div(height, kTile));
  const int n_tiles = tiles_x * tiles_y;
  hipStream_t s = as_stream(stream);
#define QR_LAUNCH(DT)                                                                              \
  hipLaunchKernelGGL(dense_backward_kernel<DT>, dim3(n_tiles), dim3(kTilePix), 0, s, width, height, \
                     tiles_x, n_tiles, *prm, tile_offsets, sorted_gid,                             \
                     reinterpret_cast<const float2*>(means2d),                                     \
                     reinterpret_cast<const float4*>(conic_opacity), features, feature_scale, dim,  \
                     out, grad_out, grad_features, grad_means2d, grad_conic_opacity)
  switch (dtype) {
    case QR_F32: QR_LAUNCH(QR_F32); break;
    case QR_BF16: QR_LAUNCH(QR_BF16); break;
    default: QR_LAUNCH(QR_FP8_E4M3); break;
  }
#undef QR_LAUNCH
  return check_launch("qr_render_dense_backward");
}
