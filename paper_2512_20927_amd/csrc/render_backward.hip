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
#include "dense_walk.h"
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

// ============================================================================
// Dense backward for widths up to 512 columns, as two kernels that each read
// dL/d(out) once (the kernel above re-reads it once per 32-entry batch):
//  - dense_backward_geo_kernel, one workgroup per 64-pixel strip of a tile:
//    the forward strip kernel's split walk (dense_walk.h, so the same weights
//    are formed). Wave w holds dL/d(out) of the strip's pixels for columns
//    128 w .. 128 w + 127 in registers as MFMA operands (bfloat16 pairs) and
//    forms, per batch, its partial dots D = G F^T [64 px x 32 entries] over
//    those columns; the four partials are summed through LDS and each wave
//    turns the dots of its eight entries into the geometric gradients (the
//    prefix sums of w d are exchanged between the waves like the walk's
//    products). <g, out> is formed once from the same registers.
//  - dense_backward_feat_kernel, one workgroup of eight waves per (tile,
//    128-column slice): two threads walk each pixel's chain in list order
//    (one per half of a batch), the weights go to LDS as bfloat16 pairs
//    W^T [entries x 256 px], and wave w contracts them with the dL/d(out)
//    of the slice's 16-column block w, held in registers: dF [32 entries x
//    16 columns] per batch, one atomic per (entry, column). (The walk is
//    the kernel's VALU cost and is repeated per slice, hence wide slices.)
constexpr int kGeoCols = 128;          // columns per wave (dense_backward_geo_kernel)
constexpr int kGeoMaxDim = 4 * kGeoCols;
constexpr int kDS = kWalkBatch + 1;    // LDS stride of a pixel's partial dots
constexpr int kStripPx = 64;
constexpr int kFeatWaves = 8;          // waves of dense_backward_feat_kernel (one 16-column block each)
constexpr int kFeatCols = 16 * kFeatWaves;  // columns per workgroup
constexpr int kWT = kTilePix + 8;      // LDS stride (bf16) of an entry's weights

struct GeoLds {
  float2 mean[2][kWalkBatch];
  float4 co[2][kWalkBatch];
  uint32_t gid[2][kWalkBatch];
  float dpart[4][kStripPx * kDS];  // partial dots per wave: [pixel][entry]
  float part[4][kStripPx];
  float tend[4][kStripPx];
  uint32_t info[4][kStripPx];
  float spart[4][kStripPx];        // sum of w d over a wave's eight entries
  float tot[4][kStripPx];          // partial <g, out> per wave
};

// Eight consecutive features (columns c .. c+7) of row g as raw loads
// (float32 values; bfloat16 or e4m3 codes as bits, with the row's scale),
// and their split into bfloat16 pairs (bfloat16 rows are exact in the high
// part), so that loads can be requested well before they are used.
struct Feat8Raw {
  f32x4 a, b;
};

template <int DT>
__device__ __forceinline__ Feat8Raw feat8_load(const QR_GLOBAL void* feats, const QR_GLOBAL float* scale,
                                               uint32_t g, int dim, int c) {
  const uint64_t off = static_cast<uint64_t>(g) * static_cast<uint32_t>(dim) + static_cast<uint32_t>(c);
  Feat8Raw r;
  if constexpr (DT == QR_F32) {
    r.a = *reinterpret_cast<const QR_GLOBAL f32x4*>(static_cast<const QR_GLOBAL float*>(feats) + off);
    r.b = *reinterpret_cast<const QR_GLOBAL f32x4*>(static_cast<const QR_GLOBAL float*>(feats) + off + 4);
  } else if constexpr (DT == QR_BF16) {
    r.a = *reinterpret_cast<const QR_GLOBAL f32x4*>(static_cast<const QR_GLOBAL uint16_t*>(feats) + off);
  } else {
    const f32x2 w = *reinterpret_cast<const QR_GLOBAL f32x2*>(static_cast<const QR_GLOBAL uint8_t*>(feats) + off);
    r.a = f32x4{w.x, w.y, scale[g], 0.f};
  }
  return r;
}

template <int DT>
__device__ __forceinline__ void feat8_split(const Feat8Raw& r, bf16x8& hi, bf16x8& lo) {
  float x[8];
  if constexpr (DT == QR_F32) {
    x[0] = r.a.x; x[1] = r.a.y; x[2] = r.a.z; x[3] = r.a.w;
    x[4] = r.b.x; x[5] = r.b.y; x[6] = r.b.z; x[7] = r.b.w;
  } else if constexpr (DT == QR_BF16) {
    hi = __builtin_bit_cast(bf16x8, r.a);
    lo = bf16x8{};
    return;
  } else {
    const float4 p = e4m3x4_to_f32(__float_as_uint(r.a.x), r.a.z);
    const float4 q = e4m3x4_to_f32(__float_as_uint(r.a.y), r.a.z);
    x[0] = p.x; x[1] = p.y; x[2] = p.z; x[3] = p.w;
    x[4] = q.x; x[5] = q.y; x[6] = q.z; x[7] = q.w;
  }
  split8(x, hi, lo);
}

template <int DT>
__global__ void __launch_bounds__(kTilePix, 2)
dense_backward_geo_kernel(int W, int H, int tiles_x, int n_units, qr_params prm,
                          const uint32_t* __restrict__ tile_offsets_,
                          const uint32_t* __restrict__ sorted_gid_, const float2* __restrict__ means2d_,
                          const float4* __restrict__ conic_opacity_, const void* __restrict__ feats_,
                          const float* __restrict__ scale_, int dim, const float* __restrict__ out_,
                          const float* __restrict__ grad_out_, float* __restrict__ grad_means2d_,
                          float* __restrict__ grad_co_) {
  const QR_GLOBAL uint32_t* tile_offsets = (const QR_GLOBAL uint32_t*)tile_offsets_;
  const QR_GLOBAL uint32_t* sorted_gid = (const QR_GLOBAL uint32_t*)sorted_gid_;
  const QR_GLOBAL f32x2* means2d = (const QR_GLOBAL f32x2*)means2d_;
  const QR_GLOBAL f32x4* conic_opacity = (const QR_GLOBAL f32x4*)conic_opacity_;
  const QR_GLOBAL void* feats = (const QR_GLOBAL void*)feats_;
  const QR_GLOBAL float* scale = (const QR_GLOBAL float*)scale_;
  const QR_GLOBAL float* out = (const QR_GLOBAL float*)out_;
  const QR_GLOBAL float* grad_out = (const QR_GLOBAL float*)grad_out_;
  QR_GLOBAL float* grad_means2d = (QR_GLOBAL float*)grad_means2d_;
  QR_GLOBAL float* grad_co = (QR_GLOBAL float*)grad_co_;
  __shared__ GeoLds L;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kb = lane >> 4, ci = lane & 15;
  const int u = xcd_remap(blockIdx.x, n_units);
  const int tile = u >> 2, strip = u & 3;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int lo = static_cast<int>(tile_offsets[tile]);
  const int hi = static_cast<int>(tile_offsets[tile + 1]);
  if (lo == hi) return;  // uniform
  // the lane's pixel in the walk (the same in every wave)
  const int px = tx * kTile + ci;
  const int py = ty * kTile + strip * 4 + kb;
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;

  // dL/d(out) of the strip for this wave's columns, as A operands: pixel
  // (ci, strip row p), columns 128 w + 32 s + 8 kb .. + 7; and <g, out>
  const bool wcols = kGeoCols * wave < dim;  // uniform
  bf16x8 ghi[4][4], glo[4][4];
  {
    float tp[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      tp[p] = 0.f;
      const int gx = tx * kTile + ci, gy = ty * kTile + strip * 4 + p;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int c = kGeoCols * wave + 32 * s + 8 * kb;
        float g8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (gx < W && gy < H && c < dim) {
          const int64_t base = (static_cast<int64_t>(gy) * W + gx) * dim + c;
          const f32x4 a = *reinterpret_cast<const QR_GLOBAL f32x4*>(grad_out + base);
          const f32x4 b = *reinterpret_cast<const QR_GLOBAL f32x4*>(grad_out + base + 4);
          const f32x4 oa = *reinterpret_cast<const QR_GLOBAL f32x4*>(out + base);
          const f32x4 ob = *reinterpret_cast<const QR_GLOBAL f32x4*>(out + base + 4);
          g8[0] = a.x; g8[1] = a.y; g8[2] = a.z; g8[3] = a.w;
          g8[4] = b.x; g8[5] = b.y; g8[6] = b.z; g8[7] = b.w;
          tp[p] += a.x * oa.x + a.y * oa.y + a.z * oa.z + a.w * oa.w + b.x * ob.x + b.y * ob.y +
                   b.z * ob.z + b.w * ob.w;
        }
        split8(g8, ghi[p][s], glo[p][s]);
      }
    }
    // sum over the four lanes of a pixel (kb = 0..3), then over the waves
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      tp[p] += __shfl_xor(tp[p], 16);
      tp[p] += __shfl_xor(tp[p], 32);
      if (kb == 0) L.tot[wave][16 * p + ci] = tp[p];
    }
  }
  // records of the first batch, requested by threads 0..31 one batch ahead
  int rgid = -1;
  f32x2 rmean = f32x2{0.f, 0.f};
  f32x4 rco = f32x4{0.f, 0.f, 0.f, 0.f};
  if (tid < kWalkBatch && lo + tid < hi) {
    rgid = static_cast<int>(sorted_gid[lo + tid]);
    rmean = means2d[rgid];
    rco = conic_opacity[rgid];
  }
  __syncthreads();
  const float total = L.tot[0][lane] + L.tot[1][lane] + L.tot[2][lane] + L.tot[3][lane];

  float T = 1.f, P = 0.f;
  bool done = !inside;
  int ncon = 0;
  int par = 0;
  for (int batch = lo; batch < hi; batch += kWalkBatch, par ^= 1) {
    const int cnt = min(kWalkBatch, hi - batch);
    const int nb = batch + kWalkBatch;
    // stage the batch into buffer `par` (last read two batches back, before
    // the previous iteration's first barrier); id slots past the list
    // repeat the batch's first id
    const int g0 = __shfl(rgid, 0);
    if (tid < kWalkBatch) {
      L.gid[par][tid] = static_cast<uint32_t>(tid < cnt ? rgid : g0);
      L.mean[par][tid] = make_float2(rmean.x, rmean.y);
      L.co[par][tid] = make_float4(rco.x, rco.y, rco.z, rco.w);
    }
    if (__syncthreads_count(!done) == 0) break;  // publishes the records; uniform
    const bool prefetch = tid < kWalkBatch && nb + tid < hi;
    if (prefetch) rgid = static_cast<int>(sorted_gid[nb + tid]);

    // partial dots over this wave's columns: D[pixel][entry], A = G, B = F^T
    // (entry 16 e + ci, columns 128 w + 32 s + 8 kb .. + 7; columns past dim
    // load column 0 and are zeroed)
    floatx4 acc[4][2];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int e = 0; e < 2; ++e) acc[p][e] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (wcols) {
      const uint32_t ge[2] = {L.gid[par][ci], L.gid[par][16 + ci]};
      // the rows of step s + 1 are requested before step s is multiplied
      // (float32 rows at their step: registers)
      constexpr bool kAhead = DT != QR_F32;
      Feat8Raw fr[2][2];
      const auto load_step = [&](int s, Feat8Raw (&r)[2]) {
        const int c = kGeoCols * wave + 32 * s + 8 * kb;
#pragma unroll
        for (int e = 0; e < 2; ++e) r[e] = feat8_load<DT>(feats, scale, ge[e], dim, c < dim ? c : 0);
      };
      if (kAhead) load_step(0, fr[0]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (kGeoCols * wave + 32 * s >= dim) break;  // uniform
        if (!kAhead) load_step(s, fr[s & 1]);
        else if (s + 1 < 4 && kGeoCols * wave + 32 * (s + 1) < dim) load_step(s + 1, fr[(s + 1) & 1]);
        const bool live = kGeoCols * wave + 32 * s + 8 * kb < dim;
        bf16x8 fhi[2], flo[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          feat8_split<DT>(fr[s & 1][e], fhi[e], flo[e]);
          if (!live) {
            fhi[e] = bf16x8{};
            flo[e] = bf16x8{};
          }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            acc[p][e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ghi[p][s], fhi[e], acc[p][e], 0, 0, 0);
            acc[p][e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(glo[p][s], fhi[e], acc[p][e], 0, 0, 0);
            if constexpr (DT != QR_BF16)
              acc[p][e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ghi[p][s], flo[e], acc[p][e], 0, 0, 0);
          }
      }
    }
    // lane (kb, ci) holds D[pixel 16 p + 4 kb + i][entry 16 e + ci]
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          L.dpart[wave][(16 * p + 4 * kb + i) * kDS + 16 * e + ci] = acc[p][e][i];

    // the walk, first half
    float al[kWalkQ];
    L.part[wave][lane] =
        walk_alpha8(L.mean[par], L.co[par], kWalkQ * wave, cnt, done, pxc, pyc, prm, al);
    if (prefetch) {
      rmean = means2d[rgid];
      rco = conic_opacity[rgid];
    }


    __syncthreads();

    // second half: this wave's weights; the dots of its eight entries
    float Tl = T;
    for (int q = 0; q < wave; ++q) Tl *= L.part[q][lane];
    float w[kWalkQ];
    const uint32_t inf = walk_weights8(Tl, al, prm.T_eps, w);
    L.tend[wave][lane] = Tl;
    L.info[wave][lane] = inf;
    float d[kWalkQ];
    float S = 0.f;
#pragma unroll
    for (int j = 0; j < kWalkQ; ++j) {
      const int k = lane * kDS + kWalkQ * wave + j;
      d[j] = L.dpart[0][k] + L.dpart[1][k] + L.dpart[2][k] + L.dpart[3][k];
      S += w[j] * d[j];
    }
    L.spart[wave][lane] = S;
    __syncthreads();

    // prefix of w d before this wave's entries; the pixel's state after the
    // batch (the same in every wave)
    float Pq = P;
    for (int q = 0; q < wave; ++q) Pq += L.spart[q][lane];
#pragma unroll
    for (int q = 0; q < 4; ++q) P += L.spart[q][lane];
    walk_fold(&L.tend[0][0], &L.info[0][0], kStripPx, lane, batch - lo, T, done, ncon);

    // dL/dalpha' and the chain rule per (pixel, entry), summed over the
    // strip's pixels with transposed wave sums (value q of entry j is value
    // j + 8 q, so lane j + 8 q ends with its total), one atomic per (entry,
    // value)
    float r5[32];
    bool any = false;
#pragma unroll
    for (int j = 0; j < kWalkQ; ++j) {
      const int e = kWalkQ * wave + j;
      float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (w[j] != 0.f) {
        any = true;
        Pq += w[j] * d[j];
        const AlphaEval ev = eval_alpha(L.mean[par][e], L.co[par][e], pxc, pyc, prm.alpha_max);
        if (!ev.clamped) {
          const float4 co = L.co[par][e];
          const float T_before = w[j] / ev.alpha;  // w = alpha' T
          const float dL_da = T_before * d[j] - (total - Pq) / (1.f - ev.alpha);
          const float dpow = dL_da * ev.alpha;
          v[0] = dpow * (-0.5f * ev.dx * ev.dx);
          v[1] = dpow * (-ev.dx * ev.dy);
          v[2] = dpow * (-0.5f * ev.dy * ev.dy);
          v[3] = dL_da * ev.G;
          v[4] = dpow * (co.x * ev.dx + co.y * ev.dy);
          v[5] = dpow * (co.y * ev.dx + co.z * ev.dy);
        }
      }
      // the first stage at once: values j + 8 q and j + 8 q + 32
      r5[j] = tsum_bit5(v[0], v[4]);
      r5[j + 8] = tsum_bit5(v[1], v[5]);
      r5[j + 16] = tsum_bit5(v[2], 0.f);
      r5[j + 24] = tsum_bit5(v[3], 0.f);
    }
    if (__ballot(any) == 0ull) continue;  // uniform: no weight in this wave's entries
    float r4[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) r4[k] = tsum_bit4(r5[k], r5[k + 16]);
    const float sv = tsum_rows(r4, lane);
    if (lane < 6 * kWalkQ && sv != 0.f) {
      const int j = lane & 7, q = lane >> 3;
      const uint32_t g = L.gid[par][kWalkQ * wave + j];
      if (q < 4) {
        if (grad_co) __hip_atomic_fetch_add(grad_co + 4 * g + q, sv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (grad_means2d) {
        __hip_atomic_fetch_add(grad_means2d + 2 * g + q - 4, sv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

struct FeatLds {
  __attribute__((aligned(16))) __bf16 whi[kWalkBatch * kWT];  // W^T [entry][pixel]
  __attribute__((aligned(16))) __bf16 wlo[kWalkBatch * kWT];
  float2 mean[2][kWalkBatch];
  float4 co[2][kWalkBatch];
  uint32_t gid[2][kWalkBatch];
  float Th[kTilePix];      // T and stop flag of each pixel after the first half of a batch
  uint32_t dh[kTilePix];
  float Tf[kTilePix];      // ... and after the whole batch
  uint32_t df[kTilePix];
};

__global__ void __launch_bounds__(kFeatWaves * 64, 4)
dense_backward_feat_kernel(int W, int H, int tiles_x, int n_units, int n_slices, qr_params prm,
                           const uint32_t* __restrict__ tile_offsets_,
                           const uint32_t* __restrict__ sorted_gid_,
                           const float2* __restrict__ means2d_,
                           const float4* __restrict__ conic_opacity_, int dim,
                           const float* __restrict__ grad_out_, float* __restrict__ grad_features_) {
  const QR_GLOBAL uint32_t* tile_offsets = (const QR_GLOBAL uint32_t*)tile_offsets_;
  const QR_GLOBAL uint32_t* sorted_gid = (const QR_GLOBAL uint32_t*)sorted_gid_;
  const QR_GLOBAL f32x2* means2d = (const QR_GLOBAL f32x2*)means2d_;
  const QR_GLOBAL f32x4* conic_opacity = (const QR_GLOBAL f32x4*)conic_opacity_;
  const QR_GLOBAL float* grad_out = (const QR_GLOBAL float*)grad_out_;
  QR_GLOBAL float* grad_features = (QR_GLOBAL float*)grad_features_;
  __shared__ FeatLds L;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kb = lane >> 4, ci = lane & 15;
  // the slices of a tile are consecutive units (same XCD: shared records)
  const int u = xcd_remap(blockIdx.x, n_units);
  const int tile = u / n_slices, slice = u % n_slices;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int lo = static_cast<int>(tile_offsets[tile]);
  const int hi = static_cast<int>(tile_offsets[tile + 1]);
  if (lo == hi) return;  // uniform
  // thread tid walks pixel pix = tid % 256 of the tile over half h of each
  // batch: entries 16 h .. 16 h + 15
  const int pix = tid & (kTilePix - 1), half = tid >> 8;
  const int px = tx * kTile + (pix % kTile);
  const int py = ty * kTile + (pix / kTile);
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;

  // B operands: dL/d(out) of pixels 32 k + 8 kb .. + 7, column `col`
  const int col = slice * kFeatCols + 16 * wave + ci;
  const bool wcols = slice * kFeatCols + 16 * wave < dim;  // uniform
  bf16x8 bhi[8], blo[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float x[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int p = 32 * k + 8 * kb + t;
      const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
      x[t] = (wcols && gx < W && gy < H) ? grad_out[(static_cast<int64_t>(gy) * W + gx) * dim + col] : 0.f;
    }
    split8(x, bhi[k], blo[k]);
  }

  int rgid = -1;
  f32x2 rmean = f32x2{0.f, 0.f};
  f32x4 rco = f32x4{0.f, 0.f, 0.f, 0.f};
  if (tid < kWalkBatch && lo + tid < hi) {
    rgid = static_cast<int>(sorted_gid[lo + tid]);
    rmean = means2d[rgid];
    rco = conic_opacity[rgid];
  }
  float T = 1.f;
  bool done = !inside;
  int par = 0;
  for (int batch = lo; batch < hi; batch += kWalkBatch, par ^= 1) {
    const int cnt = min(kWalkBatch, hi - batch);
    const int nb = batch + kWalkBatch;
    if (tid < kWalkBatch) {
      L.gid[par][tid] = static_cast<uint32_t>(rgid);
      L.mean[par][tid] = make_float2(rmean.x, rmean.y);
      L.co[par][tid] = make_float4(rco.x, rco.y, rco.z, rco.w);
    }
    // publishes the records (and orders this batch's weight stores after the
    // previous batch's MFMA reads); uniform exit once every pixel stopped
    if (__syncthreads_count(!done) == 0) break;
    const bool prefetch = tid < kWalkBatch && nb + tid < hi;
    if (prefetch) rgid = static_cast<int>(sorted_gid[nb + tid]);
    // Eq. 1 along this pixel's ray, in list order, as two halves of the
    // batch: both take alpha' of their entries at once; the first half then
    // runs the transmittance chain with the stop test, and the second
    // continues it from the first's T and stop flag (the same operations in
    // the same order as one sequential walk)
    constexpr int kHalf = kWalkBatch / 2;
    float al[kHalf];
#pragma unroll
    for (int j = 0; j < kHalf; ++j) {
      const int e = kHalf * half + j;
      al[j] = 0.f;
      if (e < cnt && !done) {
        const float a = gauss_alpha(L.mean[par][e], L.co[par][e], pxc, pyc, prm.alpha_max);
        if (a >= prm.alpha_min) al[j] = a;
      }
    }
    const auto chain = [&]() {
#pragma unroll
      for (int j = 0; j < kHalf; ++j) {
        float w = 0.f;
        if (al[j] > 0.f && !done) {
          const float T_test = T * (1.f - al[j]);
          if (T_test < prm.T_eps) {
            done = true;
          } else {
            w = al[j] * T;
            T = T_test;
          }
        }
        const int e = kHalf * half + j;
        const __bf16 h = static_cast<__bf16>(w);
        L.whi[e * kWT + pix] = h;
        L.wlo[e * kWT + pix] = static_cast<__bf16>(w - static_cast<float>(h));
      }
    };
    if (half == 0) {
      chain();
      L.Th[pix] = T;
      L.dh[pix] = done;
    }
    __syncthreads();
    if (half == 1) {
      T = L.Th[pix];
      done = L.dh[pix] != 0u;
      chain();
      L.Tf[pix] = T;
      L.df[pix] = done;
    }
    if (prefetch) {
      rmean = means2d[rgid];
      rco = conic_opacity[rgid];
    }
    __syncthreads();
    if (half == 0) {
      T = L.Tf[pix];
      done = L.df[pix] != 0u;
    }
    if (!wcols) continue;
    // dF [entry 16 e + ci][column] = sum over the tile's pixels of W^T G
    floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (16 * e >= cnt) break;  // uniform
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int a0 = (16 * e + ci) * kWT + 32 * k + 8 * kb;
        const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(&L.whi[a0]);
        const bf16x8 alo = *reinterpret_cast<const bf16x8*>(&L.wlo[a0]);
        mfma3(acc[e], ahi, alo, bhi[k], blo[k]);
      }
    }
    // lane (kb, ci) holds dF[entry 16 e + 4 kb + i][column 16 w + ci]
    if (col < dim) {
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = 16 * e + 4 * kb + i;
          if (j < cnt && acc[e][i] != 0.f)
            __hip_atomic_fetch_add(grad_features + static_cast<int64_t>(L.gid[par][j]) * dim + col,
                                   acc[e][i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  if (dim <= kGeoMaxDim) {
    // two kernels, each reading dL/d(out) once
    if (grad_features) {
      const int n_slices = static_cast<int>(ceil_div(dim, kFeatCols));
      const int n_units = n_tiles * n_slices;
      hipLaunchKernelGGL(dense_backward_feat_kernel, dim3(n_units), dim3(kFeatWaves * 64), 0, s, width,
                         height, tiles_x, n_units, n_slices, *prm, tile_offsets, sorted_gid,
                         reinterpret_cast<const float2*>(means2d),
                         reinterpret_cast<const float4*>(conic_opacity), dim, grad_out, grad_features);
    }
    if (grad_means2d || grad_conic_opacity) {
      const int n_units = n_tiles * 4;
#define QR_LAUNCH(DT)                                                                               \
  hipLaunchKernelGGL(dense_backward_geo_kernel<DT>, dim3(n_units), dim3(kTilePix), 0, s, width,      \
                     height, tiles_x, n_units, *prm, tile_offsets, sorted_gid,                      \
                     reinterpret_cast<const float2*>(means2d),                                      \
                     reinterpret_cast<const float4*>(conic_opacity), features, feature_scale, dim,   \
                     out, grad_out, grad_means2d, grad_conic_opacity)
      switch (dtype) {
        case QR_F32: QR_LAUNCH(QR_F32); break;
        case QR_BF16: QR_LAUNCH(QR_BF16); break;
        default: QR_LAUNCH(QR_FP8_E4M3); break;
      }
#undef QR_LAUNCH
    }
    return check_launch("qr_render_dense_backward");
  }
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
