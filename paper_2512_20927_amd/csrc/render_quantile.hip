// Quantile Rendering forward (Algorithm 1, Sec. 4.2).
//
// One workgroup per 16x16 tile, one thread per pixel (4 wave64s).
// Phase 1 (selection, quantile_select.h, shared with the backward): the tile's depth-sorted list is staged into LDS in
// batches of 256 projected records; every pixel walks it front to back with
// the transmittance chain T_test = T (1 - alpha') and the threshold test
// T_test < t_{k+1}, recording the <= K selected (Gaussian id, w^Q) pairs in
// LDS. A pixel is done once all K thresholds are consumed (the paper's stop
// test T_test < 1/(K+1) is the same event), and the whole workgroup leaves the
// list as soon as every pixel is done.
// Phase 2 (gather-blend): pixels are gathered four at a time (a row segment
// of the tile) with the lanes of a wave spanning the feature dimension. The
// four pixels' selection lists are first merged into their distinct
// selections, each carrying the four weights already divided by the pixel's
// 1 - T^Q, so every distinct feature row is loaded once per group (mostly
// from L2: neighbouring pixels select the same Gaussians); rows are
// accumulated in float32 and streamed to the [H, W, D] map with non-temporal
// stores. The map write is the dominant HBM traffic of the whole pipeline.
// Everything after the walk is wave-local: wave w's pixels (tile rows
// 4w .. 4w+3) are exactly the pixels of the groups it gathers.
#include "quantile_select.h"

namespace qr {

// R distinct rows of a merged group, both column slots of the lane: all 2R
// loads are requested before the first is used, then accumulated in row order.
template <int DT, int R>
__device__ __forceinline__ void accum_rows(const GView& v, const int* ug, const float4* uw,
                                           const uint8_t* um, int e0, int l0, int l1, int dim,
                                           float4 (&a0)[kPG], float4 (&a1)[kPG]) {
  float4 f0[R], f1[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int g = __builtin_amdgcn_readfirstlane(ug[e0 + e]);
    f0[e] = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * l0);
    f1[e] = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * l1);
  }
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const float4 w = uw[e0 + e];
    const float ws[kPG] = {w.x, w.y, w.z, w.w};
    // pixels that did not select the row have weight 0: skipped by uniform
    // (scalar) branches instead of multiplied
    const uint32_t mk = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(um[e0 + e]));
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      if (!(mk & (1u << q))) continue;
      a0[q].x += ws[q] * f0[e].x;
      a0[q].y += ws[q] * f0[e].y;
      a0[q].z += ws[q] * f0[e].z;
      a0[q].w += ws[q] * f0[e].w;
      a1[q].x += ws[q] * f1[e].x;
      a1[q].y += ws[q] * f1[e].y;
      a1[q].z += ws[q] * f1[e].z;
      a1[q].w += ws[q] * f1[e].w;
    }
  }
}

// Stores four features (columns 4 c4 .. 4 c4 + 3) of map pixel pix, as
// float32 or as bfloat16 codes rounded to nearest even (OT = QR_BF16).
template <int OT>
__device__ __forceinline__ void store_out4(QR_GLOBAL float* out, int64_t pix, int dim, int c4,
                                           float4 v) {
  if constexpr (OT == QR_F32) {
    store_stream(reinterpret_cast<QR_GLOBAL float4*>(out + pix * dim) + c4, v);
  } else {
    const u32x2 x = {static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v.x))) |
                         (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v.y))) << 16),
                     static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v.z))) |
                         (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v.w))) << 16)};
    __builtin_nontemporal_store(
        x, reinterpret_cast<QR_GLOBAL u32x2*>(reinterpret_cast<QR_GLOBAL uint16_t*>(out) + pix * dim + 4 * c4));
  }
}

// Gather-blend of one 4-pixel group whose distinct selections are merged:
// out[p] = sum_e (w_pe / (1 - T^Q_p)) f_e (the normalisation is folded into
// the merged weights). Each lane owns two float4 columns per pass (512
// features per pass for the wave); rows are taken four at a time, the last
// two or one on their own, so no multiply is spent on padding.
template <int DT, int OT, class Lds>
__device__ __forceinline__ void gather_group_merged(const GView& v, const Lds& L, int grp,
                                                    int nu, int tx, int ty, int lane, int dim) {
  const int dim4 = dim >> 2;
  const int p0 = grp * kPG;
  const int* ug = &L.ugid[grp * Lds::kCap];
  const float4* uw = &L.uw[grp * Lds::kCap];
  const uint8_t* um = &L.umask[grp * Lds::kCap];
  for (int cb = 0; cb < dim4; cb += 128) {
    const int c0 = cb + lane, c1 = cb + 64 + lane;
    const int l0 = min(c0, dim4 - 1), l1 = min(c1, dim4 - 1);  // in-bounds columns to load
    float4 a0[kPG], a1[kPG];
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      a0[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      a1[q] = a0[q];
    }
    int e0 = 0;
    for (; e0 + 4 <= nu; e0 += 4) accum_rows<DT, 4>(v, ug, uw, um, e0, l0, l1, dim, a0, a1);
    if (e0 + 2 <= nu) {
      accum_rows<DT, 2>(v, ug, uw, um, e0, l0, l1, dim, a0, a1);
      e0 += 2;
    }
    if (e0 < nu) accum_rows<DT, 1>(v, ug, uw, um, e0, l0, l1, dim, a0, a1);
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      const int p = p0 + q;
      if (L.ns[p] < 0) continue;  // outside the image
      const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
      const int64_t pix = static_cast<int64_t>(gy) * v.W + gx;
      if (c0 < dim4) store_out4<OT>(v.out, pix, dim, c0, a0[q]);
      if (c1 < dim4) store_out4<OT>(v.out, pix, dim, c1, a1[q]);
    }
  }
}

// Gather-blend of all sixteen merged groups of a wave at once, for narrow
// rows (dim <= 128): lpg lanes per group (the power of two >= dim / 4, one
// float4 column each), so 64 / lpg groups are blended side by side, and all
// kUCap (16) row loads of a lane are requested before the first is used
// (slots past a group's distinct count load a row of the group again and are
// not accumulated). One memory round trip per round instead of one per
// group. Groups with more than kUCap distinct selections (also under the
// larger merge capacity) are skipped here.
template <int DT, int OT, class Lds>
__device__ __forceinline__ void gather_groups_narrow(const GView& v, const Lds& L, int wave,
                                                     int tx, int ty, int lane, int dim) {
  constexpr int kCap = Lds::kCap;
  const int dim4 = dim >> 2;
  const int lpg_log = dim4 <= 4 ? 2 : dim4 <= 8 ? 3 : dim4 <= 16 ? 4 : 5;
  const int gpr = 64 >> lpg_log;  // groups per round
  const int c = lane & ((1 << lpg_log) - 1);
  const int cl = min(c, dim4 - 1);  // in-bounds column to load
  constexpr int kWaveGroups = kGroups / 4;
  for (int r0 = 0; r0 < kWaveGroups; r0 += gpr) {
    const int grp = wave * kWaveGroups + r0 + (lane >> lpg_log);
    const int nu_all = L.unum[grp];
    const int nu = nu_all > kUCap ? -1 : nu_all;  // more than kUCap: the overflow path
    float4 a[kPG];
#pragma unroll
    for (int q = 0; q < kPG; ++q) a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (nu > 0) {
      const int* ug = &L.ugid[grp * kCap];
      float4 f[kUCap];
#pragma unroll
      for (int e = 0; e < kUCap; ++e)
        f[e] = load_feat4_global<DT>(v.feats, v.scale, ug[min(e, nu - 1)], dim, 4 * cl);
#pragma unroll
      for (int e = 0; e < kUCap; ++e) {
        if (e < nu) {
          const float4 w = L.uw[grp * kCap + e];
          const float ws[kPG] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int q = 0; q < kPG; ++q) {
            a[q].x += ws[q] * f[e].x;
            a[q].y += ws[q] * f[e].y;
            a[q].z += ws[q] * f[e].z;
            a[q].w += ws[q] * f[e].w;
          }
        }
      }
    }
    if (nu >= 0 && c < dim4) {
      const int p0 = grp * kPG;
#pragma unroll
      for (int q = 0; q < kPG; ++q) {
        const int p = p0 + q;
        if (L.ns[p] < 0) continue;  // outside the image
        const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
        store_out4<OT>(v.out, static_cast<int64_t>(gy) * v.W + gx, dim, c, a[q]);
      }
    }
  }
}

// The groups that gather_groups_narrow skipped (more than kUCap distinct
// selections, or than the merge capacity), with the same lane layout: pixel by pixel, each pixel's
// selections taken eight at a time (their ids, then their rows, each batch
// requested together), all such groups of a round side by side.
template <int DT, int OT, class Lds>
__device__ __forceinline__ void gather_groups_narrow_overflow(const GView& v, const Lds& L,
                                                              const int* __restrict__ s_sel_pos,
                                                              const float* __restrict__ s_sel_w,
                                                              int KP, int K, int wave, int tx, int ty,
                                                              int lane, int dim) {
  constexpr int kChunk = 8;
  const int dim4 = dim >> 2;
  const int lpg_log = dim4 <= 4 ? 2 : dim4 <= 8 ? 3 : dim4 <= 16 ? 4 : 5;
  const int gpr = 64 >> lpg_log;
  const int c = lane & ((1 << lpg_log) - 1);
  const int cl = min(c, dim4 - 1);
  constexpr int kWaveGroups = kGroups / 4;
  for (int r0 = 0; r0 < kWaveGroups; r0 += gpr) {
    const int grp = wave * kWaveGroups + r0 + (lane >> lpg_log);
    const bool mine = L.unum[grp] < 0 || L.unum[grp] > kUCap;
    if (!__any(mine)) continue;
#pragma unroll 1
    for (int q = 0; q < kPG; ++q) {
      const int p = grp * kPG + q;
      const int n = mine ? L.ns[p] : -1;  // -1: not this path's pixel, or outside the image
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int j0 = 0; j0 < K; j0 += kChunk) {
        if (!__any(n > j0)) break;
        if (n > j0) {
          int g[kChunk];
          float w[kChunk];
#pragma unroll
          for (int jj = 0; jj < kChunk; ++jj) {
            const int j = min(j0 + jj, n - 1);
            g[jj] = static_cast<int>(v.sorted_gid[s_sel_pos[p * KP + j]]);
            w[jj] = s_sel_w[p * KP + j];
          }
          float4 f[kChunk];
#pragma unroll
          for (int jj = 0; jj < kChunk; ++jj) f[jj] = load_feat4_global<DT>(v.feats, v.scale, g[jj], dim, 4 * cl);
#pragma unroll
          for (int jj = 0; jj < kChunk; ++jj) {
            if (j0 + jj < n) {
              a.x += w[jj] * f[jj].x;
              a.y += w[jj] * f[jj].y;
              a.z += w[jj] * f[jj].z;
              a.w += w[jj] * f[jj].w;
            }
          }
        }
      }
      if (n >= 0 && c < dim4) {
        const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
        const float inv = L.inv[p];
        store_out4<OT>(v.out, static_cast<int64_t>(gy) * v.W + gx, dim, c,
                       make_float4(a.x * inv, a.y * inv, a.z * inv, a.w * inv));
      }
    }
  }
}

// Gather-blend of a group with more distinct selections than the merge
// capacity: pixel by pixel, each selection's row loaded for its own pixel.
template <int DT, int OT, class Lds>
__device__ __forceinline__ void gather_group_per_pixel(const GView& v, const Lds& L,
                                                       const int* __restrict__ s_sel_pos,
                                                       const float* __restrict__ s_sel_w, int KP,
                                                       int grp, int tx, int ty, int lane, int dim) {
  const int dim4 = dim >> 2;
  const int p0 = grp * kPG;
  int n[kPG];
  int nmax = 0, safe = 0;
#pragma unroll
  for (int q = 0; q < kPG; ++q) {
    n[q] = L.ns[p0 + q];
    if (n[q] > nmax) {
      nmax = n[q];
      safe = static_cast<int>(v.sorted_gid[s_sel_pos[(p0 + q) * KP]]);
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
        const int g = ok ? static_cast<int>(v.sorted_gid[s_sel_pos[(p0 + q) * KP + j]]) : safe;
        w[q] = ok ? s_sel_w[(p0 + q) * KP + j] : 0.f;
        f[q] = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * c);
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
      const float inv = L.inv[p];
      store_out4<OT>(v.out, static_cast<int64_t>(gy) * v.W + gx, dim, c,
                     make_float4(acc[q].x * inv, acc[q].y * inv, acc[q].z * inv, acc[q].w * inv));
    }
  }
}

// Algorithm 1 for every pixel of one tile, then the gather-blend of the
// selected rows. Called by all 256 threads of the workgroup. Workgroup
// barriers occur only around the staging of record batches; the pixels of
// wave w are tile rows 4w .. 4w+3, which are exactly the pixels of the
// gather groups it owns, so everything after the walk is wave-local.
// Shared LDS (the record batch) is only rewritten after a barrier that every
// wave reaches once it has finished the previous tile.
template <int DT, int OT, int MODE, class Lds>
__device__ __forceinline__ void quantile_tile(const GView& v, int tile, int K, int dim,
                                              const qr_params& prm, Lds& L,
                                              int* __restrict__ s_sel_gid,
                                              float* __restrict__ s_sel_w,
                                              int32_t* __restrict__ sel_gid_out,
                                              float* __restrict__ sel_w_out,
                                              float* __restrict__ T_final_out,
                                              int32_t* __restrict__ last_pos_out) {
  const int W = v.W, H = v.H;
  const int tiles_x = (W + kTile - 1) / kTile;
  const int tid = threadIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid % kTile);
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;

  const int lo = static_cast<int>(v.tile_offsets[tile]);
  const int hi = static_cast<int>(v.tile_offsets[tile + 1]);
  const int KP = (K + 3) & ~3;  // selection row stride: 16-byte aligned rows
  int* s_sel_pos = s_sel_gid;   // selections are kept as tile-list positions
  const PixelSel sel = quantile_select<MODE>(v, lo, hi, K, pxc, pyc, inside, prm, L, s_sel_pos, s_sel_w, KP);
  const int ns = sel.ns;
  const float TQ = sel.TQ;
  const int* my_pos = s_sel_pos + tid * KP;
  const float* my_w = s_sel_w + tid * KP;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int kWaveGroups = kGroups / 4;
  if (dim <= 128) {
    gather_groups_narrow<DT, OT>(v, L, wave, tx, ty, lane, dim);
    gather_groups_narrow_overflow<DT, OT>(v, L, s_sel_pos, s_sel_w, KP, K, wave, tx, ty, lane, dim);
  } else {
    for (int gl = 0; gl < kWaveGroups; ++gl) {
      const int grp = wave * kWaveGroups + gl;
      const int nu = __builtin_amdgcn_readfirstlane(L.unum[grp]);
      if (nu >= 0)
        gather_group_merged<DT, OT>(v, L, grp, nu, tx, ty, lane, dim);
      else  // more distinct selections than the merge capacity (rare)
        gather_group_per_pixel<DT, OT>(v, L, s_sel_pos, s_sel_w, KP, grp, tx, ty, lane, dim);
    }
  }
  // Per-pixel outputs last: a load issued after a store waits for it, so no
  // store precedes the loads of the merge and the gather.
  if (inside) {
    const int pix = py * W + px;
    if (v.T_q) v.T_q[pix] = TQ;
    if (v.n_sel) v.n_sel[pix] = ns;
    if (T_final_out) T_final_out[pix] = sel.T;
    if (last_pos_out) last_pos_out[pix] = sel.last;
    if (sel_gid_out) {
      for (int j = 0; j < K; ++j) {
        sel_gid_out[static_cast<int64_t>(pix) * K + j] =
            j < ns ? static_cast<int>(v.sorted_gid[my_pos[j]]) : -1;
        sel_w_out[static_cast<int64_t>(pix) * K + j] = j < ns ? my_w[j] : 0.f;
      }
    }
  }
}

template <int DT, int OT, int MODE, int UCAP>
__global__ void __launch_bounds__(kTilePix, kWavesPerSimd)
render_quantile_kernel(ViewArgs v, int n_tiles, qr_params prm, int K, int dim,
                       int32_t* __restrict__ sel_gid_out, float* __restrict__ sel_w_out,
                       float* __restrict__ T_final_out, int32_t* __restrict__ last_pos_out) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ QuantileLdsT<UCAP> L;
  int* s_sel_gid = reinterpret_cast<int*>(dyn_lds);                            // [256][KP]
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + kTilePix * ((K + 3) & ~3);  // [256][KP]
  quantile_tile<DT, OT, MODE>(to_global(v), xcd_remap(blockIdx.x, n_tiles), K, dim, prm, L, s_sel_gid,
                    s_sel_w, sel_gid_out, sel_w_out, T_final_out, last_pos_out);
}

// Many views in one persistent launch. The schedule is cut into one
// contiguous range per XCD (workgroup b runs on XCD b % 8), each with its own
// atomic counter: a workgroup takes items of its XCD's range in order, so the
// tiles in flight on an XCD are neighbours whose records and feature rows
// share that XCD's L2; once its range is used up it takes items from the
// other ranges, and it leaves when every range is used up.
constexpr int kXcdQueues = 8;

__device__ __forceinline__ uint32_t queue_begin(int64_t n_items, int q) {
  return static_cast<uint32_t>(n_items * q / kXcdQueues);
}

template <int DT, int OT, int MODE, int UCAP>
__global__ void __launch_bounds__(kTilePix, kWavesPerSimd)
render_quantile_batched_kernel(const qr_view* __restrict__ views, const uint32_t* __restrict__ schedule,
                               int64_t n_items, uint32_t* __restrict__ counter, qr_params prm,
                               int K, int dim) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ QuantileLdsT<UCAP> L;
  __shared__ uint32_t s_item[2];
  int* s_sel_gid = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + kTilePix * ((K + 3) & ~3);
  // The item slot alternates between two words: a wave that runs ahead into
  // the next iteration writes the other word, and cannot come back to this
  // one before every wave has passed the next barrier (and so has read it).
  const int home = static_cast<int>(blockIdx.x % kXcdQueues);
  for (int it = 0;; it ^= 1) {
    if (threadIdx.x == 0) {
      uint32_t item = 0xFFFFFFFFu;  // none left
      for (int d = 0; d < kXcdQueues; ++d) {
        const int q = (home + d) % kXcdQueues;
        const uint32_t b = queue_begin(n_items, q), e = queue_begin(n_items, q + 1);
        if (b == e) continue;
        const uint32_t i = atomicAdd(&counter[q], 1u);
        if (i < e - b) {
          item = b + i;
          break;
        }
      }
      s_item[it] = item;
    }
    __syncthreads();
    // uniform values: view records and tile indices stay in scalar registers
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item[it]);
    if (item >= n_items) break;
    const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[item]);
    const GView v = to_global(view_args(views[packed >> kViewShift]));
    quantile_tile<DT, OT, MODE>(v, static_cast<int>(packed & kTileMask), K, dim, prm, L, s_sel_gid, s_sel_w,
                      nullptr, nullptr, nullptr, nullptr);
  }
}

// Many views in one launch, one workgroup per (view, tile) item. Items are
// dealt to the XCDs in contiguous runs of the schedule (neighbouring tiles of
// a view share L2 contents); workgroups retire as they finish, so work on
// other streams can take their slots.
template <int DT, int OT, int MODE, int UCAP>
__global__ void __launch_bounds__(kTilePix, kWavesPerSimd)
render_quantile_batched_grid_kernel(const qr_view* __restrict__ views,
                                    const uint32_t* __restrict__ schedule, int n_items,
                                    qr_params prm, int K, int dim) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ QuantileLdsT<UCAP> L;
  int* s_sel_gid = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + kTilePix * ((K + 3) & ~3);
  const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[xcd_remap(blockIdx.x, n_items)]);
  const GView v = to_global(view_args(views[packed >> kViewShift]));
  quantile_tile<DT, OT, MODE>(v, static_cast<int>(packed & kTileMask), K, dim, prm, L, s_sel_gid, s_sel_w,
                    nullptr, nullptr, nullptr, nullptr);
}

__global__ void reset_counter_kernel(uint32_t* __restrict__ c) {
  if (threadIdx.x < kXcdQueues) c[threadIdx.x] = 0u;
}

}  // namespace qr

using namespace qr;

// Instantiates QR_LAUNCH(feature dtype, output dtype, selection rule, merge
// capacity) for the runtime values; the larger merge capacity is built for
// float32 maps (bfloat16 maps keep 16, which is correct at any K).
#define QR_DISPATCH_DT(dt, OT, SM, UC)                        \
  switch (dt) {                                               \
    case QR_F32: QR_LAUNCH(QR_F32, OT, SM, UC); break;        \
    case QR_BF16: QR_LAUNCH(QR_BF16, OT, SM, UC); break;      \
    default: QR_LAUNCH(QR_FP8_E4M3, OT, SM, UC); break;       \
  }
#define QR_DISPATCH_OT(dt, ot, SM, K)                                                   \
  do {                                                                                  \
    if ((ot) == QR_BF16) { QR_DISPATCH_DT(dt, QR_BF16, SM, kUCap) }                     \
    else if (ucap_for(K) == kUCapLarge) { QR_DISPATCH_DT(dt, QR_F32, SM, kUCapLarge) }  \
    else { QR_DISPATCH_DT(dt, QR_F32, SM, kUCap) }                                      \
  } while (0)
#define QR_DISPATCH(dt, ot, sm, K)                                                  \
  do {                                                                              \
    if ((sm) == QR_SELECT_TOPK) QR_DISPATCH_OT(dt, ot, QR_SELECT_TOPK, K);          \
    else if ((sm) == QR_SELECT_STRATIFIED) QR_DISPATCH_OT(dt, ot, QR_SELECT_STRATIFIED, K); \
    else QR_DISPATCH_OT(dt, ot, QR_SELECT_QUANTILE, K);                             \
  } while (0)

extern "C" int qr_render_quantile(void* stream, int32_t width, int32_t height,
                                  const qr_params* prm, int32_t K, const uint32_t* tile_offsets,
                                  const uint32_t* sorted_gid, const float* means2d,
                                  const float* conic_opacity, const void* features, int32_t dtype,
                                  const float* feature_scale, int32_t dim, float* out, float* T_q,
                                  int32_t* n_sel, float* T_final, int32_t* last_pos,
                                  int32_t* sel_gid, float* sel_w) {
  int rc = validate_render("qr_render_quantile", width, height, prm, tile_offsets, sorted_gid,
                           means2d, conic_opacity, features, dtype, feature_scale, dim, out);
  if (rc != QR_OK) return rc;
  if (K < 1 || K > QR_MAX_K)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile: K = %d outside [1, %d]", K, QR_MAX_K);
  if ((sel_gid == nullptr) != (sel_w == nullptr))
    return fail(QR_ERR_INVALID_ARG, "qr_render_quantile: sel_gid and sel_w must both be given or both NULL");
  if ((T_final || last_pos) && prm->selection != QR_SELECT_QUANTILE)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile: T_final and last_pos are Algorithm 1's; "
                "pass NULL with another selection rule");
  const int tiles_x = static_cast<int>(ceil_div(width, kTile));
  const int tiles_y = static_cast<int>(ceil_div(height, kTile));
  const int n_tiles = tiles_x * tiles_y;
  (void)tiles_x;
  const size_t lds = static_cast<size_t>(kTilePix) * ((K + 3) & ~3) * (sizeof(int) + sizeof(float));
  hipStream_t s = as_stream(stream);
  const ViewArgs v{width, height, tile_offsets, sorted_gid, reinterpret_cast<const float2*>(means2d),
                   reinterpret_cast<const float4*>(conic_opacity), features, feature_scale, out, T_q,
                   n_sel};
#define QR_LAUNCH(DT, OT, SM, UC)                                                                     \
  hipLaunchKernelGGL((render_quantile_kernel<DT, OT, SM, UC>), dim3(n_tiles), dim3(kTilePix), lds, s, v, \
                     n_tiles, *prm, K, dim, sel_gid, sel_w, T_final, last_pos)
  QR_DISPATCH(dtype, prm->out_dtype, prm->selection, K);
#undef QR_LAUNCH
  return check_launch("qr_render_quantile");
}

extern "C" int qr_render_quantile_batched(void* stream, int32_t n_views, const qr_view* views,
                                          const qr_params* prm, int32_t K, int32_t dtype,
                                          int32_t dim, const uint32_t* schedule, int64_t n_items,
                                          int32_t n_workgroups, void* workspace,
                                          size_t workspace_bytes) {
  if (n_views <= 0 || n_views > (1 << (32 - kViewShift)))
    return fail(QR_ERR_INVALID_ARG, "qr_render_quantile_batched: n_views = %d out of range", n_views);
  if (!views || !schedule || !prm)
    return fail(QR_ERR_INVALID_ARG, "qr_render_quantile_batched: null pointer");
  if (n_workgroups < 0) return fail(QR_ERR_INVALID_ARG, "qr_render_quantile_batched: n_workgroups < 0");
  if (n_workgroups > 0 && (!workspace || workspace_bytes < kXcdQueues * sizeof(uint32_t)))
    return fail(QR_ERR_CAPACITY, "qr_render_quantile_batched: persistent mode needs a %d-byte workspace",
                static_cast<int>(kXcdQueues * sizeof(uint32_t)));
  if (n_items < 0 || n_items >= (1ll << 31))
    return fail(QR_ERR_INVALID_ARG, "qr_render_quantile_batched: bad item count");
  if (K < 1 || K > QR_MAX_K)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_batched: K = %d outside [1, %d]", K, QR_MAX_K);
  if (dtype != QR_F32 && dtype != QR_BF16 && dtype != QR_FP8_E4M3)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_batched: unknown dtype %d", dtype);
  if (dim <= 0 || dim % 16 != 0 || dim > QR_MAX_DIM)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_batched: dim = %d", dim);
  if (!(prm->alpha_min > 0.f) || !(prm->alpha_max >= prm->alpha_min) || !(prm->alpha_max < 1.f))
    return fail(QR_ERR_INVALID_ARG, "qr_render_quantile_batched: need 0 < alpha_min <= alpha_max < 1");
  if (prm->out_dtype != QR_F32 && prm->out_dtype != QR_BF16)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_batched: unknown output dtype %d", prm->out_dtype);
  if (prm->selection != QR_SELECT_QUANTILE && prm->selection != QR_SELECT_STRATIFIED &&
      prm->selection != QR_SELECT_TOPK)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_batched: unknown selection rule %d", prm->selection);
  if (n_items == 0) return QR_OK;
  hipStream_t s = as_stream(stream);
  const size_t lds = static_cast<size_t>(kTilePix) * ((K + 3) & ~3) * (sizeof(int) + sizeof(float));
  if (n_workgroups == 0) {
    const int ni = static_cast<int>(n_items);
#define QR_LAUNCH(DT, OT, SM, UC)                                                                     \
  hipLaunchKernelGGL((render_quantile_batched_grid_kernel<DT, OT, SM, UC>), dim3(ni), dim3(kTilePix), lds, \
                     s, views, schedule, ni, *prm, K, dim)
    QR_DISPATCH(dtype, prm->out_dtype, prm->selection, K);
#undef QR_LAUNCH
    return check_launch("qr_render_quantile_batched");
  }
  auto* counter = static_cast<uint32_t*>(workspace);
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
#define QR_LAUNCH(DT, OT, SM, UC)                                                                     \
  hipLaunchKernelGGL((render_quantile_batched_kernel<DT, OT, SM, UC>), dim3(n_workgroups), dim3(kTilePix), \
                     lds, s, views, schedule, n_items, counter, *prm, K, dim)
  QR_DISPATCH(dtype, prm->out_dtype, prm->selection, K);
#undef QR_LAUNCH
  return check_launch("qr_render_quantile_batched");
}
