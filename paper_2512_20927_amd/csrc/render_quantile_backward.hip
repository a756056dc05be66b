// Backward pass of Quantile Rendering (Algorithm 1, Sec. 4.2): gradients
// with respect to the decoded float32 features, the 2D means, the conics
// (a, b, c) and the opacities, given g = dL/d(out) per pixel.
//
// With the selected j of a pixel, w_j = T^Q_j alpha'_j (T^Q_j: T^Q before j),
// Z = 1 - T^Q, out = sum_j w_j f_j / Z and d_j = <g, f_j>:
//    dL/df_j      = (w_j / Z) g
//    dL/dalpha'_j = (T^Q_j d_j - (S_j + <g, out> T^Q) / (1 - alpha'_j)) / Z,
//                   S_j = sum_{l > j} w_l d_l,  <g, out> = sum_j w_j d_j / Z,
// and alpha' = o G, G = exp(-(a dx^2 + 2 b dx dy + c dy^2)/2) gives
//    dalpha'/do = G, dalpha'/dpower = alpha' (0 for both if clamped),
//    dpower/da = -dx^2/2, /db = -dx dy, /dc = -dy^2/2,
//    dpower/du = a dx + b dy, /dv = b dx + c dy.
// The selection itself is piecewise constant and passes no gradient.
//
// One workgroup per tile, laid out like the forward:
//  1. the selection walk and the merge of each 4-pixel group's selections
//     (quantile_select.h, the very code of the forward, so the same
//     Gaussians are selected; nothing per pixel is stored by the forward);
//     the tile's distinct selections get slots with LDS accumulators, so
//     that every gradient is summed over the tile before one global atomic
//     per value (tiles select a few dozen distinct Gaussians against about
//     450 group-rows; float atomics to global memory are the expensive part);
//  2. dots d_pj = <g_p, f_j>, per group, wave-wide over 512 columns: the four
//     pixels' rows of dL/d(out) in registers, each distinct row loaded once
//     per group, the four pixels' partial dots summed over the wave together;
//  3. a reverse sweep over each pixel's selections (thread per pixel) turns
//     the dots into dL/dalpha' and the chain rule above, summed per slot;
//  4. feature gradients sum_p (w_pj / Z_p) g_p, per group and distinct row,
//     over column chunks of 128 (dL/d(out) is read a second time), summed
//     per slot and flushed after each chunk.
// T^Q_j is recovered as w_j / alpha'_j (alpha' >= alpha_min > 0 for every
// selection).
#include "quantile_select.h"

namespace qr {

// Gradient outputs of one view (generic pointers, host-constructible).
struct GradPtrs {
  const float* __restrict__ grad_out;
  float* __restrict__ grad_features;
  float* __restrict__ grad_means2d;
  float* __restrict__ grad_co;
};

struct GGrad {
  const QR_GLOBAL float* __restrict__ grad_out;
  QR_GLOBAL float* __restrict__ grad_features;
  QR_GLOBAL float* __restrict__ grad_means2d;
  QR_GLOBAL float* __restrict__ grad_co;
};

__device__ __forceinline__ GGrad to_global(const GradPtrs& g) {
  return GGrad{(const QR_GLOBAL float*)g.grad_out, (QR_GLOBAL float*)g.grad_features,
               (QR_GLOBAL float*)g.grad_means2d, (QR_GLOBAL float*)g.grad_co};
}

__device__ __forceinline__ void atomic_add(QR_GLOBAL float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Four float atomics on consecutive columns.
__device__ __forceinline__ void atomic_add4(QR_GLOBAL float* p, float4 v) {
  atomic_add(p + 0, v.x);
  atomic_add(p + 1, v.y);
  atomic_add(p + 2, v.z);
  atomic_add(p + 3, v.w);
}

template <int kCtrl>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl,
                                                               0xF, 0xF, false));
}

__device__ __forceinline__ uint32_t fbits(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float bitsf(uint32_t x) { return __builtin_bit_cast(float, x); }

// Sums four per-lane partials (one per pixel of a group) over the 64 lanes
// at once, without LDS: v_permlane32_swap exchanges lanes 32..63 of its first
// operand with lanes 0..31 of its second, so after the swap of (p0, p2) the
// sum of the two results holds p0 summed over the two halves in lanes 0..31
// and p2 likewise in lanes 32..63 (the same for p1, p3); v_permlane16_swap
// does the same with odd and even 16-lane rows, leaving row q with pixel q's
// partial sums, which DPP moves add up inside the row. On return lanes
// 16q .. 16q+15 hold the total of partial q.
__device__ __forceinline__ float wave_sum4(float p0, float p1, float p2, float p3) {
  const auto a = __builtin_amdgcn_permlane32_swap(fbits(p0), fbits(p2), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(fbits(p1), fbits(p3), false, false);
  const float x = bitsf(a[0]) + bitsf(a[1]);
  const float y = bitsf(b[0]) + bitsf(b[1]);
  const auto c = __builtin_amdgcn_permlane16_swap(fbits(x), fbits(y), false, false);
  float k = bitsf(c[0]) + bitsf(c[1]);
  k += dpp<0xB1>(k);   // quad_perm [1,0,3,2]
  k += dpp<0x4E>(k);   // quad_perm [2,3,0,1]
  k += dpp<0x124>(k);  // row_ror:4
  k += dpp<0x128>(k);  // row_ror:8
  return k;
}

__device__ __forceinline__ float dot8(float4 a0, float4 a1, float4 b0, float4 b1) {
  return a0.x * b0.x + a0.y * b0.y + a0.z * b0.z + a0.w * b0.w + a1.x * b1.x + a1.y * b1.y +
         a1.z * b1.z + a1.w * b1.w;
}

__device__ __forceinline__ float4 nt_load4(const QR_GLOBAL float* p) {
  const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const QR_GLOBAL f32x4*>(p));
  return make_float4(x.x, x.y, x.z, x.w);
}

// Feature gradients and geometric gradients are summed per tile before they
// reach global memory: the tile's distinct selected list positions get slots
// (in list order, from a bitmap of the selected positions), and each slot
// has LDS accumulators, flushed with one atomic per value at the end.
// Selections past the slot capacity (or past kPosCap in the list) add to
// global memory directly.
constexpr int kAccRegs = 32;    // register sums per lane and column slot
constexpr int kSlotCap = kAccRegs - 1;  // distinct selections of a tile with slots
constexpr int kPosCap = 2048;   // list positions covered by the slot bitmap
constexpr int kChunk = 128;     // feature columns summed per pass
constexpr int kGeo = 6;         // d/d(a, b, c, o, u, v)

struct BwdLds {
  int upos[kGroups * kUCap];        // merged rows' list positions
  int8_t uslot[kGroups * kUCap];    // their slots, kSlotCap if none
  uint32_t udefer[kGroups];         // per group: rows without a slot (bit e)
  uint32_t bm[kPosCap / 32];        // selected positions, relative to the list start
  int bpre[kPosCap / 32];           // slots before each bitmap word
  int sgid[kSlotCap];               // Gaussian id of each slot
  float geo[4][kSlotCap * kGeo];    // geometric gradient sums, per wave
  float acc[kSlotCap * kChunk];     // feature gradient sums of one column chunk
  int nslot;
};

__device__ __forceinline__ int slot_of(const BwdLds& B, int r) {
  if (r >= kPosCap) return -1;
  const int s = B.bpre[r >> 5] + __popc(B.bm[r >> 5] & ((1u << (r & 31)) - 1u));
  return s < kSlotCap ? s : -1;
}

// The two float4 columns (c0, c1) of pixel p's row of dL/d(out), zero for
// columns past dim.
__device__ __forceinline__ void load_grad_row(const GView& v, const GGrad& gg, int p, int tx, int ty,
                                              int c0, int c1, int dim, float4& g0, float4& g1) {
  const int dim4 = dim >> 2;
  const int gx = tx * kTile + (p % kTile), gy = ty * kTile + (p / kTile);
  const QR_GLOBAL float* row = gg.grad_out + (static_cast<int64_t>(gy) * v.W + gx) * dim;
  g0 = c0 < dim4 ? nt_load4(row + 4 * c0) : make_float4(0.f, 0.f, 0.f, 0.f);
  g1 = c1 < dim4 ? nt_load4(row + 4 * c1) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Dots of R distinct rows of a merged group for one pass of 512 columns,
// summed over the wave and stored (first pass) or added to s_d at the row's
// place in each selecting pixel's list (byte q of sel counts the rows pixel
// q selected so far).
template <int DT, int R>
__device__ __forceinline__ void dot_rows(const GView& v, const int* ug, const uint8_t* um, int e0,
                                         int l0, int l1, int dim, const float4 (&g0)[kPG],
                                         const float4 (&g1)[kPG], float* __restrict__ s_d, int p0,
                                         int KP, uint32_t& sel, int lane, bool first) {
  float4 f0[R], f1[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int g = __builtin_amdgcn_readfirstlane(ug[e0 + e]);
    f0[e] = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * l0);
    f1[e] = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * l1);
  }
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const uint32_t mk = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(um[e0 + e]));
    float pd[kPG] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < kPG; ++q)
      if (mk & (1u << q)) pd[q] = dot8(g0[q], g1[q], f0[e], f1[e]);
    const float t = wave_sum4(pd[0], pd[1], pd[2], pd[3]);
    const int q = lane >> 4;
    const int j = static_cast<int>((sel >> (8 * q)) & 0xFFu);
    if ((lane & 15) == 0 && (mk & (1u << q))) {
      float* d = &s_d[(p0 + q) * KP + j];
      *d = first ? t : *d + t;
    }
    sel += (mk & 1u) | ((mk & 2u) << 7) | ((mk & 4u) << 14) | ((mk & 8u) << 21);
  }
}

// d_pj = <g_p, f_j> for every selection of one group's pixels, into s_d.
template <int DT>
__device__ __forceinline__ void group_dots(const GView& v, const GGrad& gg, const QuantileLds& L,
                                           const int* __restrict__ s_sel_pos, int grp, int nu,
                                           int tx, int ty, int lane, int dim,
                                           float* __restrict__ s_d, int KP) {
  const int dim4 = dim >> 2;
  const int p0 = grp * kPG;
  for (int cb = 0; cb < dim4; cb += 128) {
    const int c0 = cb + lane, c1 = cb + 64 + lane;
    const int l0 = min(c0, dim4 - 1), l1 = min(c1, dim4 - 1);
    float4 g0[kPG], g1[kPG];
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      // pixels with no selection (or outside the image) have a constant
      // output: nothing flows back through them
      if (__builtin_amdgcn_readfirstlane(L.ns[p0 + q]) > 0) {
        load_grad_row(v, gg, p0 + q, tx, ty, c0, c1, dim, g0[q], g1[q]);
      } else {
        g0[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        g1[q] = g0[q];
      }
    }
    if (nu >= 0) {
      const int* ug = &L.ugid[grp * kUCap];
      const uint8_t* um = &L.umask[grp * kUCap];
      uint32_t sel = 0u;
      int e0 = 0;
      for (; e0 + 4 <= nu; e0 += 4) dot_rows<DT, 4>(v, ug, um, e0, l0, l1, dim, g0, g1, s_d, p0, KP, sel, lane, cb == 0);
      if (e0 + 2 <= nu) {
        dot_rows<DT, 2>(v, ug, um, e0, l0, l1, dim, g0, g1, s_d, p0, KP, sel, lane, cb == 0);
        e0 += 2;
      }
      if (e0 < nu) dot_rows<DT, 1>(v, ug, um, e0, l0, l1, dim, g0, g1, s_d, p0, KP, sel, lane, cb == 0);
    } else {  // more distinct selections than kUCap: pixel by pixel
#pragma unroll
      for (int q = 0; q < kPG; ++q) {
        const int p = p0 + q;
        const int n = __builtin_amdgcn_readfirstlane(L.ns[p]);
        for (int j = 0; j < n; ++j) {
          const int pos = __builtin_amdgcn_readfirstlane(s_sel_pos[p * KP + j]);
          const int g = static_cast<int>(__builtin_amdgcn_readfirstlane(v.sorted_gid[pos]));
          const float4 f0 = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * l0);
          const float4 f1 = load_feat4_global<DT>(v.feats, v.scale, g, dim, 4 * l1);
          const float t = wave_sum4(dot8(g0[q], g1[q], f0, f1), 0.f, 0.f, 0.f);
          if (lane == 0) s_d[p * KP + j] = cb == 0 ? t : s_d[p * KP + j] + t;
        }
      }
    }
  }
}

// Adds the feature gradient (a0, a1) (columns cb + lane and cb + 64 + lane)
// of a selection to its slot's register sums (slot s, uniform: an indexed
// register move), or to global memory for a selection without a slot
// (Gaussian g).
__device__ __forceinline__ void add_feature_grad(const GGrad& gg, int s, int g, int lane, int cb,
                                                 int dim, float a0, float a1,
                                                 float (&acc0)[kAccRegs], float (&acc1)[kAccRegs]) {
  if (s >= 0) {
    acc0[s] += a0;
    acc1[s] += a1;
  } else {
    QR_GLOBAL float* dst = gg.grad_features + static_cast<int64_t>(g) * dim + cb;
    if (cb + lane < dim) atomic_add(dst + lane, a0);
    if (cb + 64 + lane < dim) atomic_add(dst + 64 + lane, a1);
  }
}

// Columns cb + lane and cb + 64 + lane of the rows of dL/d(out) of batch h
// (kBatch groups) of this wave's groups (the pixels of wave w are tile
// pixels 64 w + lane). Exactly kGradBatchLoads(kBatch) loads are issued, none
// skipped: addresses are clamped into the image and the columns into dim
// (values of pixels outside the image, or with no selection, are never used:
// no merged row carries their mask bit; columns past dim are never
// written), so that a wait for all but the newest batch is a fixed count.
template <int kBatch>
constexpr int kGradBatchLoads = 2 * kBatch * kPG;

template <int kBatch>
__device__ __forceinline__ void load_grad_batch(const GView& v, const GGrad& gg, int wave,
                                                int lane, int tx, int ty, int cb, int dim, int h,
                                                float (&g0)[kBatch][kPG], float (&g1)[kBatch][kPG]) {
  const int c0 = min(cb + lane, dim - 1), c1 = min(cb + 64 + lane, dim - 1);
#pragma unroll
  for (int gi = 0; gi < kBatch; ++gi) {
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      const int p = wave * 64 + (h * kBatch + gi) * kPG + q;
      const int gx = min(tx * kTile + (p % kTile), v.W - 1);
      const int gy = min(ty * kTile + (p / kTile), v.H - 1);
      const QR_GLOBAL float* row = gg.grad_out + (static_cast<int64_t>(gy) * v.W + gx) * dim;
      g0[gi][q] = __builtin_nontemporal_load(row + c0);
      g1[gi][q] = __builtin_nontemporal_load(row + c1);
    }
  }
}

// s_waitcnt vmcnt(n) (gfx9 encoding: vmcnt in bits 3:0 and 15:14; expcnt
// and lgkmcnt left at their maxima, i.e. not waited for).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

// Feature gradients of one group for the chunk of columns [cb, cb + 128):
// sum_p (w_pj / Z_p) g_p per distinct row, into the wave's slot sums. g0 /
// g1: the group's four rows of dL/d(out) at columns cb + lane and
// cb + 64 + lane.
__device__ __forceinline__ void group_feature_grads(const GView& v, const GGrad& gg,
                                                    const QuantileLds& L, const BwdLds& B,
                                                    const int* __restrict__ s_sel_pos,
                                                    const float* __restrict__ s_sel_w, int KP,
                                                    int grp, int lo, int lane, int cb, int dim,
                                                    const float (&g0)[kPG], const float (&g1)[kPG],
                                                    float (&acc0)[kAccRegs], float (&acc1)[kAccRegs]) {
  const int p0 = grp * kPG;
  const int nu = __builtin_amdgcn_readfirstlane(L.unum[grp]);
  if (nu >= 0) {
    const int* ug = &L.ugid[grp * kUCap];
    const float4* uw = &L.uw[grp * kUCap];
    const int8_t* us = &B.uslot[grp * kUCap];
    // a pixel that did not select the row has weight 0: multiplied rather
    // than branched over (fewer instructions than testing its mask bit)
    auto row_grad = [&](int e, float& a0, float& a1) {
      const float4 w = uw[e];
      a0 = w.x * g0[0] + w.y * g0[1] + w.z * g0[2] + w.w * g0[3];
      a1 = w.x * g1[0] + w.y * g1[1] + w.z * g1[2] + w.w * g1[3];
    };
    // Rows are summed into their slot's registers two at a time (their LDS
    // reads issued together); a row without a slot lands in the unused
    // register kSlotCap and goes to global memory after the loop, so that
    // the loop issues no memory operation (and so waits for none).
    int e = 0;
    for (; e + 2 <= nu; e += 2) {
      const int sa = __builtin_amdgcn_readfirstlane(static_cast<int>(us[e]));
      const int sb = __builtin_amdgcn_readfirstlane(static_cast<int>(us[e + 1]));
      float a0, a1, b0, b1;
      row_grad(e, a0, a1);
      row_grad(e + 1, b0, b1);
      acc0[sa] += a0;
      acc1[sa] += a1;
      acc0[sb] += b0;
      acc1[sb] += b1;
    }
    if (e < nu) {
      const int sa = __builtin_amdgcn_readfirstlane(static_cast<int>(us[e]));
      float a0, a1;
      row_grad(e, a0, a1);
      acc0[sa] += a0;
      acc1[sa] += a1;
    }
    uint32_t deferred = __builtin_amdgcn_readfirstlane(B.udefer[grp]);
    while (deferred) {
      const int e = __builtin_ctz(deferred);
      deferred &= deferred - 1u;
      float a0, a1;
      row_grad(e, a0, a1);
      add_feature_grad(gg, -1, __builtin_amdgcn_readfirstlane(ug[e]), lane, cb, dim, a0, a1, acc0, acc1);
    }
  } else {
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      const int p = p0 + q;
      const int n = __builtin_amdgcn_readfirstlane(L.ns[p]);
      const float inv = L.inv[p];
      for (int j = 0; j < n; ++j) {
        const int pos = __builtin_amdgcn_readfirstlane(s_sel_pos[p * KP + j]);
        const int s = slot_of(B, pos - lo);
        const int g = s >= 0 ? 0 : static_cast<int>(__builtin_amdgcn_readfirstlane(v.sorted_gid[pos]));
        const float w = s_sel_w[p * KP + j] * inv;
        add_feature_grad(gg, s, g, lane, cb, dim, w * g0[q], w * g1[q], acc0, acc1);
      }
    }
  }
}

// Backward of one tile (all 256 threads of the workgroup). kBatch: groups
// whose rows of dL/d(out) are requested together in the feature pass;
// kAhead: the next batch is requested while one is summed (more round trips
// overlap, at the cost of registers).
template <int DT, int kBatch, bool kAhead>
__device__ __forceinline__ void quantile_backward_tile(const GView& v, const GGrad& gg, int tile,
                                                       int K, int dim, const qr_params& prm,
                                                       QuantileLds& L, BwdLds& B,
                                                       int* __restrict__ s_sel_pos,
                                                       float* __restrict__ s_sel_w,
                                                       float* __restrict__ s_d) {
  const int tiles_x = (v.W + kTile - 1) / kTile;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: row addresses stay scalar
  constexpr int kWaveGroups = kGroups / 4;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid % kTile);
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < v.W && py < v.H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;
  const int lo = static_cast<int>(v.tile_offsets[tile]);
  const int hi = static_cast<int>(v.tile_offsets[tile + 1]);
  const int KP = (K + 3) & ~3;
  const PixelSel sel =
      quantile_select(v, lo, hi, K, pxc, pyc, inside, prm, L, s_sel_pos, s_sel_w, KP, B.upos);
  const int ns = sel.ns;
  const int* my_pos = s_sel_pos + tid * KP;
  const float* my_w = s_sel_w + tid * KP;
  const bool geo = gg.grad_means2d || gg.grad_co;

  // ---- slots: the tile's distinct selected positions, in list order ----
  if (tid < kPosCap / 32) B.bm[tid] = 0u;
  __syncthreads();
  for (int j = 0; j < ns; ++j) {
    const int r = my_pos[j] - lo;
    if (r < kPosCap) atomicOr(&B.bm[r >> 5], 1u << (r & 31));
  }
  __syncthreads();
  if (tid < kPosCap / 32) {  // wave 0: exclusive prefix of the word populations
    const int c = __popc(B.bm[tid]);
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(incl, off, 64);
      if (lane >= off) incl += u;
    }
    B.bpre[tid] = incl - c;
    if (tid == kPosCap / 32 - 1) B.nslot = min(incl, kSlotCap);
  }
  for (int i = tid; i < 4 * kSlotCap * kGeo; i += kTilePix) (&B.geo[0][0])[i] = 0.f;
  for (int i = tid; i < kSlotCap * kChunk; i += kTilePix) B.acc[i] = 0.f;
  __syncthreads();
  for (int j = 0; j < ns; ++j) {
    const int s = slot_of(B, my_pos[j] - lo);
    if (s >= 0) B.sgid[s] = static_cast<int>(v.sorted_gid[my_pos[j]]);  // same value from every writer
  }
  if (lane < kWaveGroups) {
    const int grp = wave * kWaveGroups + lane;
    const int nu = L.unum[grp];
    uint32_t defer = 0u;
    for (int e = 0; e < nu; ++e) {
      const int sl = slot_of(B, B.upos[grp * kUCap + e] - lo);
      B.uslot[grp * kUCap + e] = static_cast<int8_t>(sl >= 0 ? sl : kSlotCap);
      if (sl < 0) defer |= 1u << e;
    }
    B.udefer[grp] = defer;
  }
  __syncthreads();
  const int nslot = B.nslot;

  if (geo) {
    // ---- dots d_pj (wave-local; the first pass stores every selection's) ----
    for (int gl = 0; gl < kWaveGroups; ++gl) {
      const int grp = wave * kWaveGroups + gl;
      const int nu = __builtin_amdgcn_readfirstlane(L.unum[grp]);
      group_dots<DT>(v, gg, L, s_sel_pos, grp, nu, tx, ty, lane, dim, s_d, KP);
    }
    wave_lds_sync();

    // ---- reverse sweep over this pixel's selections ----
    if (ns > 0) {
      const float TQ = sel.TQ;
      const float invZ = 1.f / (1.f - TQ);
      const float* my_d = s_d + tid * KP;
      float gout = 0.f;  // <g, out>
      for (int j = 0; j < ns; ++j) gout += my_w[j] * my_d[j];
      gout *= invZ;
      float S = 0.f;
      for (int j = ns - 1; j >= 0; --j) {
        const int g = static_cast<int>(v.sorted_gid[my_pos[j]]);
        const f32x2 m = v.means2d[g];
        const f32x4 c = v.conic_opacity[g];
        const AlphaEval e = eval_alpha(make_float2(m.x, m.y), make_float4(c.x, c.y, c.z, c.w), pxc,
                                       pyc, prm.alpha_max);
        const float wj = my_w[j], dj = my_d[j];
        const float tq = wj / e.alpha;  // T^Q before this selection
        const float dL_da = invZ * (tq * dj - (S + gout * TQ) / (1.f - e.alpha));
        S += wj * dj;
        if (e.clamped || dL_da == 0.f) continue;
        const float dpow = dL_da * e.alpha;
        const float gv[kGeo] = {dpow * (-0.5f * e.dx * e.dx), dpow * (-e.dx * e.dy),
                                dpow * (-0.5f * e.dy * e.dy), dL_da * e.G,
                                dpow * (c.x * e.dx + c.y * e.dy), dpow * (c.y * e.dx + c.z * e.dy)};
        const int s = slot_of(B, my_pos[j] - lo);
        if (s >= 0) {
#pragma unroll
          for (int i = 0; i < kGeo; ++i) atomicAdd(&B.geo[wave][s * kGeo + i], gv[i]);
        } else {
          if (gg.grad_co)
            for (int i = 0; i < 4; ++i) atomic_add(gg.grad_co + 4 * g + i, gv[i]);
          if (gg.grad_means2d)
            for (int i = 0; i < 2; ++i) atomic_add(gg.grad_means2d + 2 * g + i, gv[4 + i]);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < nslot * kGeo; i += kTilePix) {
      const float val = B.geo[0][i] + B.geo[1][i] + B.geo[2][i] + B.geo[3][i];
      const int s = i / kGeo, k = i - s * kGeo;
      const int g = B.sgid[s];
      if (val == 0.f) continue;
      if (k < 4) {
        if (gg.grad_co) atomic_add(gg.grad_co + 4 * g + k, val);
      } else if (gg.grad_means2d) {
        atomic_add(gg.grad_means2d + 2 * g + (k - 4), val);
      }
    }
  }

  if (gg.grad_features) {
    // ---- feature gradients, one chunk of columns at a time ----
    // Each wave sums its groups' rows per slot in registers, the four waves'
    // sums meet in LDS, and one atomic per (slot, column) goes to memory.
    for (int cb = 0; cb < dim; cb += kChunk) {
      float acc0[kAccRegs], acc1[kAccRegs];  // [kSlotCap]: rows without a slot
#pragma unroll
      for (int i = 0; i < kAccRegs; ++i) {
        acc0[i] = 0.f;
        acc1[i] = 0.f;
      }
      // rows of dL/d(out) are requested kBatch groups at a time (one batch
      // ahead of the batch being summed if kAhead)
      constexpr int kNB = kWaveGroups / kBatch;
      float gA0[kBatch][kPG], gA1[kBatch][kPG], gB0[kBatch][kPG], gB1[kBatch][kPG];
      if (kAhead) load_grad_batch<kBatch>(v, gg, wave, lane, tx, ty, cb, dim, 0, gA0, gA1);
#pragma unroll 1
      for (int h = 0; h < kNB; ++h) {
        if (!kAhead) {
          load_grad_batch<kBatch>(v, gg, wave, lane, tx, ty, cb, dim, h, gA0, gA1);
        } else if (h + 1 < kNB) {
          load_grad_batch<kBatch>(v, gg, wave, lane, tx, ty, cb, dim, h + 1, gB0, gB1);
          // batch h has arrived once at most the next batch's loads are
          // outstanding
          wait_vmcnt<kGradBatchLoads<kBatch>>();
        }
#pragma unroll
        for (int gi = 0; gi < kBatch; ++gi)
          group_feature_grads(v, gg, L, B, s_sel_pos, s_sel_w, KP, wave * kWaveGroups + h * kBatch + gi,
                              lo, lane, cb, dim, gA0[gi], gA1[gi], acc0, acc1);
        if (kAhead) {
#pragma unroll
          for (int gi = 0; gi < kBatch; ++gi) {
#pragma unroll
            for (int q = 0; q < kPG; ++q) {
              gA0[gi][q] = gB0[gi][q];
              gA1[gi][q] = gB1[gi][q];
            }
          }
        }
      }
      for (int i = 0; i < nslot; ++i) {
        atomicAdd(&B.acc[i * kChunk + lane], acc0[i]);
        atomicAdd(&B.acc[i * kChunk + 64 + lane], acc1[i]);
      }
      __syncthreads();
      for (int i = tid; i < nslot * kChunk; i += kTilePix) {
        const int sl = i / kChunk, c = i - sl * kChunk;
        const float val = B.acc[i];
        B.acc[i] = 0.f;
        if (val != 0.f && cb + c < dim)
          atomic_add(gg.grad_features + static_cast<int64_t>(B.sgid[sl]) * dim + cb + c, val);
      }
      __syncthreads();
    }
  }
}

// Two workgroups per CU: the backward keeps a third [256][K] array (the dots)
// in LDS.
constexpr int kBwdWavesPerSimd = 2;

__device__ __forceinline__ size_t bwd_sel_floats(int K) { return static_cast<size_t>(kTilePix) * ((K + 3) & ~3); }

template <int DT>
__global__ void __launch_bounds__(kTilePix, kBwdWavesPerSimd)
quantile_backward_kernel(ViewArgs v, GradPtrs gp, int n_tiles, qr_params prm, int K, int dim) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ QuantileLds L;
  __shared__ BwdLds B;
  const size_t n = bwd_sel_floats(K);
  int* s_sel_pos = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + n;
  float* s_d = s_sel_w + n;
  quantile_backward_tile<DT, 2, true>(to_global(v), to_global(gp), xcd_remap(blockIdx.x, n_tiles), K, dim,
                             prm, L, B, s_sel_pos, s_sel_w, s_d);
}

__device__ __forceinline__ GradPtrs grad_ptrs(const qr_view_grad& g) {
  return GradPtrs{g.grad_out, g.grad_features, g.grad_means2d, g.grad_conic_opacity};
}

// Many views in one launch, one workgroup per (view, tile) item, items dealt
// to the XCDs in contiguous runs of the schedule.
template <int DT>
__global__ void __launch_bounds__(kTilePix, kBwdWavesPerSimd)
quantile_backward_batched_grid_kernel(const qr_view* __restrict__ views,
                                      const qr_view_grad* __restrict__ grads,
                                      const uint32_t* __restrict__ schedule, int n_items,
                                      qr_params prm, int K, int dim) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ QuantileLds L;
  __shared__ BwdLds B;
  const size_t n = bwd_sel_floats(K);
  int* s_sel_pos = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + n;
  float* s_d = s_sel_w + n;
  const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[xcd_remap(blockIdx.x, n_items)]);
  const uint32_t vi = packed >> kViewShift;
  quantile_backward_tile<DT, 1, true>(to_global(view_args(views[vi])), to_global(grad_ptrs(grads[vi])),
                             static_cast<int>(packed & kTileMask), K, dim, prm, L, B, s_sel_pos,
                             s_sel_w, s_d);
}

// Many views in one persistent launch: items are taken from per-XCD ranges
// of the schedule exactly as by the persistent forward renderer.
constexpr int kBwdXcdQueues = 8;

__device__ __forceinline__ uint32_t bwd_queue_begin(int64_t n_items, int q) {
  return static_cast<uint32_t>(n_items * q / kBwdXcdQueues);
}

template <int DT>
__global__ void __launch_bounds__(kTilePix, kBwdWavesPerSimd)
quantile_backward_batched_kernel(const qr_view* __restrict__ views,
                                 const qr_view_grad* __restrict__ grads,
                                 const uint32_t* __restrict__ schedule, int64_t n_items,
                                 uint32_t* __restrict__ counter, qr_params prm, int K, int dim) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ QuantileLds L;
  __shared__ BwdLds B;
  __shared__ uint32_t s_item[2];
  const size_t n = bwd_sel_floats(K);
  int* s_sel_pos = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + n;
  float* s_d = s_sel_w + n;
  const int home = static_cast<int>(blockIdx.x % kBwdXcdQueues);
  // the item word alternates as in the forward: a wave running ahead writes
  // the other word
  for (int it = 0;; it ^= 1) {
    if (threadIdx.x == 0) {
      uint32_t item = 0xFFFFFFFFu;
      for (int d = 0; d < kBwdXcdQueues; ++d) {
        const int q = (home + d) % kBwdXcdQueues;
        const uint32_t b = bwd_queue_begin(n_items, q), e = bwd_queue_begin(n_items, q + 1);
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
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item[it]);
    if (item >= n_items) break;
    const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[item]);
    const uint32_t vi = packed >> kViewShift;
    quantile_backward_tile<DT, 1, false>(to_global(view_args(views[vi])), to_global(grad_ptrs(grads[vi])),
                               static_cast<int>(packed & kTileMask), K, dim, prm, L, B, s_sel_pos,
                               s_sel_w, s_d);
  }
}

__global__ void reset_bwd_counter_kernel(uint32_t* __restrict__ c) {
  if (threadIdx.x < kBwdXcdQueues) c[threadIdx.x] = 0u;
}

inline size_t bwd_dynamic_lds(int K) {
  return static_cast<size_t>(kTilePix) * ((K + 3) & ~3) * 3 * sizeof(float);
}

}  // namespace qr

using namespace qr;

extern "C" int qr_render_quantile_backward(void* stream, int32_t width, int32_t height,
                                           const qr_params* prm, int32_t K,
                                           const uint32_t* tile_offsets, const uint32_t* sorted_gid,
                                           const float* means2d, const float* conic_opacity,
                                           const void* features, int32_t dtype,
                                           const float* feature_scale, int32_t dim,
                                           const float* grad_out, float* grad_features,
                                           float* grad_means2d, float* grad_conic_opacity) {
  int rc = validate_render("qr_render_quantile_backward", width, height, prm, tile_offsets,
                           sorted_gid, means2d, conic_opacity, features, dtype, feature_scale, dim,
                           grad_out);
  if (rc != QR_OK) return rc;
  if (K < 1 || K > QR_MAX_K)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_backward: K = %d outside [1, %d]", K, QR_MAX_K);
  const int tiles_x = static_cast<int>(ceil_div(width, kTile));
  const int tiles_y = static_cast<int>(ceil_div(height, kTile));
  const int n_tiles = tiles_x * tiles_y;
  hipStream_t s = as_stream(stream);
  const ViewArgs v{width, height, tile_offsets, sorted_gid, reinterpret_cast<const float2*>(means2d),
                   reinterpret_cast<const float4*>(conic_opacity), features, feature_scale,
                   nullptr, nullptr, nullptr};
  const GradPtrs gp{grad_out, grad_features, grad_means2d, grad_conic_opacity};
  const size_t lds = bwd_dynamic_lds(K);
#define QR_LAUNCH(DT)                                                                             \
  hipLaunchKernelGGL(quantile_backward_kernel<DT>, dim3(n_tiles), dim3(kTilePix), lds, s, v, gp, \
                     n_tiles, *prm, K, dim)
  switch (dtype) {
    case QR_F32: QR_LAUNCH(QR_F32); break;
    case QR_BF16: QR_LAUNCH(QR_BF16); break;
    default: QR_LAUNCH(QR_FP8_E4M3); break;
  }
#undef QR_LAUNCH
  return check_launch("qr_render_quantile_backward");
}

extern "C" int qr_render_quantile_batched_backward(void* stream, int32_t n_views,
                                                   const qr_view* views, const qr_view_grad* grads,
                                                   const qr_params* prm, int32_t K, int32_t dtype,
                                                   int32_t dim, const uint32_t* schedule,
                                                   int64_t n_items, int32_t n_workgroups,
                                                   void* workspace, size_t workspace_bytes) {
  const char* name = "qr_render_quantile_batched_backward";
  if (n_views <= 0 || n_views > (1 << (32 - kViewShift)))
    return fail(QR_ERR_INVALID_ARG, "%s: n_views = %d out of range", name, n_views);
  if (!views || !grads || !schedule || !prm) return fail(QR_ERR_INVALID_ARG, "%s: null pointer", name);
  if (n_workgroups < 0) return fail(QR_ERR_INVALID_ARG, "%s: n_workgroups < 0", name);
  if (n_workgroups > 0 && (!workspace || workspace_bytes < kBwdXcdQueues * sizeof(uint32_t)))
    return fail(QR_ERR_CAPACITY, "%s: persistent mode needs a %d-byte workspace", name,
                static_cast<int>(kBwdXcdQueues * sizeof(uint32_t)));
  if (n_items < 0 || n_items >= (1ll << 31)) return fail(QR_ERR_INVALID_ARG, "%s: bad item count", name);
  if (K < 1 || K > QR_MAX_K)
    return fail(QR_ERR_UNSUPPORTED, "%s: K = %d outside [1, %d]", name, K, QR_MAX_K);
  if (dtype != QR_F32 && dtype != QR_BF16 && dtype != QR_FP8_E4M3)
    return fail(QR_ERR_UNSUPPORTED, "%s: unknown dtype %d", name, dtype);
  if (dim <= 0 || dim % 16 != 0 || dim > QR_MAX_DIM)
    return fail(QR_ERR_UNSUPPORTED, "%s: dim = %d", name, dim);
  if (!(prm->alpha_min > 0.f) || !(prm->alpha_max >= prm->alpha_min) || !(prm->alpha_max < 1.f))
    return fail(QR_ERR_INVALID_ARG, "%s: need 0 < alpha_min <= alpha_max < 1", name);
  if (n_items == 0) return QR_OK;
  hipStream_t s = as_stream(stream);
  const size_t lds = bwd_dynamic_lds(K);
  if (n_workgroups == 0) {
    const int ni = static_cast<int>(n_items);
#define QR_LAUNCH(DT)                                                                        \
  hipLaunchKernelGGL(quantile_backward_batched_grid_kernel<DT>, dim3(ni), dim3(kTilePix), lds, \
                     s, views, grads, schedule, ni, *prm, K, dim)
    switch (dtype) {
      case QR_F32: QR_LAUNCH(QR_F32); break;
      case QR_BF16: QR_LAUNCH(QR_BF16); break;
      default: QR_LAUNCH(QR_FP8_E4M3); break;
    }
#undef QR_LAUNCH
    return check_launch(name);
  }
  auto* counter = static_cast<uint32_t*>(workspace);
  hipLaunchKernelGGL(reset_bwd_counter_kernel, dim3(1), dim3(64), 0, s, counter);
#define QR_LAUNCH(DT)                                                                         \
  hipLaunchKernelGGL(quantile_backward_batched_kernel<DT>, dim3(n_workgroups), dim3(kTilePix), \
                     lds, s, views, grads, schedule, n_items, counter, *prm, K, dim)
  switch (dtype) {
    case QR_F32: QR_LAUNCH(QR_F32); break;
    case QR_BF16: QR_LAUNCH(QR_BF16); break;
    default: QR_LAUNCH(QR_FP8_E4M3); break;
  }
#undef QR_LAUNCH
  return check_launch(name);
}
