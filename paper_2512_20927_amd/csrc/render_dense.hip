// Dense alpha-blend forward (Eq. 1: out = sum_i T_i alpha'_i f_i over every
// Gaussian on the ray, stopping before T drops below T_eps).
//
// Per tile the output is a contraction W [256 px x G] . F [G x D] where
// W[p, g] = T_{p,g} alpha'_{p,g} (zero off the ray or after the stop) and F
// holds the feature rows of the tile's depth-sorted list. One workgroup
// computes one tile x one 128-column slice of D:
//   - 32 list entries at a time, each pixel thread walks its transmittance
//     chain and writes its 32 weights into LDS; the 32 feature rows (slice)
//     are decoded to float32 alongside;
//   - both operands are split into bfloat16 pairs x = x_hi + x_lo (x_hi the
//     rounded value, x_lo the rounded remainder) and the product is formed as
//     W_hi F_hi + W_hi F_lo + W_lo F_hi on v_mfma_f32_16x16x32_bf16 with
//     float32 accumulation (bf16 features are exact in x_hi, so their F_lo
//     term is dropped). The omitted W_lo F_lo term and the second roundings
//     are below 2^-16 of each product, i.e. float32-class accuracy at the
//     bf16 matrix rate;
//   - each wave64 owns 64 pixels (4 pixel rows) x 128 columns: 32
//     accumulator tiles of 16x16;
//   - the workgroup leaves the list once every pixel has stopped.
// The weight walk is recomputed by each of the D/128 slices of a tile.
#include "common.h"
#include "render_common.h"

namespace qr {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kDC = 128;            // feature columns per workgroup
constexpr int kGB = 32;             // list entries per batch (= MFMA K)
constexpr int kKS = kGB + 8;        // LDS stride (bf16) of a 32-entry row: 80 B

__device__ __forceinline__ void split_bf16(float x, __bf16* hi, __bf16* lo) {
  const __bf16 h = static_cast<__bf16>(x);
  *hi = h;
  *lo = static_cast<__bf16>(x - static_cast<float>(h));
}

template <int DT>
__global__ void __launch_bounds__(kTilePix, 2)
render_dense_kernel(int W, int H, int tiles_x, int n_tiles, qr_params prm,
                    const uint32_t* __restrict__ tile_offsets, const uint32_t* __restrict__ sorted_gid,
                    const float2* __restrict__ means2d, const float4* __restrict__ conic_opacity,
                    const void* __restrict__ feats, const float* __restrict__ scale, int dim,
                    float* __restrict__ out, float* __restrict__ T_final,
                    int32_t* __restrict__ n_contrib) {
  constexpr bool kSplitF = DT != QR_BF16;
  // A operand rows: one per pixel, 32 entries; B operand rows: one per column
  __shared__ __attribute__((aligned(16))) __bf16 s_Ahi[kTilePix * kKS];
  __shared__ __attribute__((aligned(16))) __bf16 s_Alo[kTilePix * kKS];
  __shared__ __attribute__((aligned(16))) __bf16 s_Bhi[kDC * kKS];
  __shared__ __attribute__((aligned(16))) __bf16 s_Blo[kSplitF ? kDC * kKS : 8];
  __shared__ float2 s_mean[kGB];
  __shared__ float4 s_co[kGB];
  __shared__ int s_gid[kGB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const int d0 = blockIdx.y * kDC;
  const int dc = min(kDC, dim - d0);  // multiple of 16
  const int n_nt = dc >> 4;
  const int dc4 = dc >> 2;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid % kTile);
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;
  const int lo = static_cast<int>(tile_offsets[tile]);
  const int hi = static_cast<int>(tile_offsets[tile + 1]);

  float T = 1.f;
  int ncon = 0;
  bool done = !inside;
  floatx4 acc[4][8];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int batch = lo; batch < hi; batch += kGB) {
    if (__syncthreads_count(!done) == 0) break;
    const int cnt = min(kGB, hi - batch);
    if (tid < cnt) {
      const int g = static_cast<int>(sorted_gid[batch + tid]);
      s_gid[tid] = g;
      s_mean[tid] = means2d[g];
      s_co[tid] = conic_opacity[g];
    }
    __syncthreads();
    // feature slice of the batch, split to bf16, stored column-major (B
    // operand: 8 consecutive entries of one column per lane); missing rows
    // are zero
    for (int e = tid; e < kGB * dc4; e += kTilePix) {
      const int r = e / dc4, c4 = e - r * dc4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < cnt) v = load_feat4<DT>(feats, scale, s_gid[r], dim, d0 + 4 * c4);
      const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = 4 * c4 + i;
        if constexpr (kSplitF) {
          split_bf16(vv[i], &s_Bhi[col * kKS + r], &s_Blo[col * kKS + r]);
        } else {
          s_Bhi[col * kKS + r] = static_cast<__bf16>(vv[i]);  // exact: the value is bf16
        }
      }
    }
    // per-pixel weights of the batch (Eq. 1), in list order
    __bf16* arow_hi = s_Ahi + tid * kKS;
    __bf16* arow_lo = s_Alo + tid * kKS;
    bool any_w = false;
    for (int j = 0; j < kGB; ++j) {
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
            ncon = batch - lo + j + 1;
          }
        }
      }
      any_w |= w != 0.f;
      split_bf16(w, &arow_hi[j], &arow_lo[j]);
    }
    // a wave whose 64 pixels take nothing from this batch skips its MFMAs
    // (thread tid is pixel tid, so wave w's pixels are exactly its A rows)
    const bool wave_busy = __ballot(any_w) != 0ull;
    __syncthreads();
    if (!wave_busy) continue;
    // W[64 px x 32] . F[32 x dc] for this wave's 64 pixels
    const int kq = (lane >> 4) * 8;  // this lane's 8 consecutive entries
    const int row = lane & 15;
    bf16x8 ahi[4], alo[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int p = wave * 64 + mt * 16 + row;
      ahi[mt] = *reinterpret_cast<const bf16x8*>(&s_Ahi[p * kKS + kq]);
      alo[mt] = *reinterpret_cast<const bf16x8*>(&s_Alo[p * kKS + kq]);
    }
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
      if (nt < n_nt) {
        const int col = nt * 16 + row;
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(&s_Bhi[col * kKS + kq]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mt], bhi, acc[mt][nt], 0, 0, 0);
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[mt], bhi, acc[mt][nt], 0, 0, 0);
        }
        if constexpr (kSplitF) {
          const bf16x8 blo = *reinterpret_cast<const bf16x8*>(&s_Blo[col * kKS + kq]);
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mt], blo, acc[mt][nt], 0, 0, 0);
        }
      }
    }
  }

  if (blockIdx.y == 0 && inside) {
    const int pix = py * W + px;
    if (T_final) T_final[pix] = T;
    if (n_contrib) n_contrib[pix] = ncon;
  }
  // accumulator layout: lane holds D[4*(lane/16) + v][lane % 16]
  const int prow_base = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int gy = ty * kTile + wave * 4 + mt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gx = tx * kTile + 4 * prow_base + v;
      if (gx < W && gy < H) {
        float* dst = out + (static_cast<int64_t>(gy) * W + gx) * dim + d0 + (lane & 15);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
          if (nt < n_nt) __builtin_nontemporal_store(acc[mt][nt][v], dst + nt * 16);
      }
    }
  }
}

}  // namespace qr

using namespace qr;

extern "C" int qr_render_dense(void* stream, int32_t width, int32_t height, const qr_params* prm,
                               const uint32_t* tile_offsets, const uint32_t* sorted_gid,
                               const float* means2d, const float* conic_opacity,
                               const void* features, int32_t dtype, const float* feature_scale,
                               int32_t dim, float* out, float* T_final, int32_t* n_contrib) {
  int rc = validate_render("qr_render_dense", width, height, prm, tile_offsets, sorted_gid,
                           means2d, conic_opacity, features, dtype, feature_scale, dim, out);
  if (rc != QR_OK) return rc;
  if (prm->out_dtype != QR_F32)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_dense: float32 output only");
  const int tiles_x = static_cast<int>(ceil_div(width, kTile));
  const int tiles_y = static_cast<int>(ceil_div(height, kTile));
  const int n_tiles = tiles_x * tiles_y;
  const dim3 grid(n_tiles, static_cast<unsigned>(ceil_div(dim, kDC)));
  hipStream_t s = as_stream(stream);
#define QR_LAUNCH(DT)                                                                              \
  hipLaunchKernelGGL(render_dense_kernel<DT>, grid, dim3(kTilePix), 0, s, width, height, tiles_x,  \
                     n_tiles, *prm, tile_offsets, sorted_gid,                                      \
                     reinterpret_cast<const float2*>(means2d),                                     \
                     reinterpret_cast<const float4*>(conic_opacity), features, feature_scale, dim,  \
                     out, T_final, n_contrib)
  switch (dtype) {
    case QR_F32: QR_LAUNCH(QR_F32); break;
    case QR_BF16: QR_LAUNCH(QR_BF16); break;
    default: QR_LAUNCH(QR_FP8_E4M3); break;
  }
#undef QR_LAUNCH
  return check_launch("qr_render_dense");
}
