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
// One workgroup per tile:
//  1. the selection walk (quantile_select.h, the very code of the forward,
//     so the same Gaussians are selected; nothing per pixel is stored by the
//     forward): each pixel's selected list positions and weights w^Q in LDS.
//     A tile selects a few dozen distinct Gaussians (about 20 on the room
//     scenes, against about 1,200 pixel selections): they get slots 0 .. 31
//     in list order, and each pixel a 32-bit mask of the slots it selected;
//  2. feature gradients dF = W^T G: [slots x 256 px] . [256 px x dim] on
//     v_mfma_f32_16x16x32_bf16 (each wave a quarter of the columns),
//     W[p][s] = w_ps / Z_p, one atomic per (slot, column);
//  3. dots D = G F^T: [256 px x dim] . [dim x slots] on the same MFMA (each
//     wave its 64 pixels), with d_pj read out at the selected (pixel, slot)
//     pairs and written over the weights, which step 2 no longer needs (so
//     a selection costs 8 bytes of LDS and K up to 64 fits);
//  4. a sweep over each pixel's selections (thread per pixel) recomputes
//     alpha'_j, w_j and T^Q_j from the records with the walk's own float
//     operations and turns the dots into dL/dalpha' and the chain rule
//     above, summed per slot in LDS and added to global memory once per
//     (slot, value). The tail sums S_j are the total minus the running
//     prefix, both kept in double.
// Both products take float32 operands split into bfloat16 pairs
// x = x_hi + x_lo and form hi.hi + hi.lo + lo.hi with float32 accumulation
// (relative error below 2^-16 per product). Selections without a slot (a
// tile with more than 32 distinct selections, or a position past kPosCap)
// are handled by a plain wave-wide path.
#include "quantile_select.h"
#include "wave_ops.h"

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

// Eight consecutive decoded features (columns c .. c+7) of Gaussian g.
template <int DT>
__device__ __forceinline__ void load_feat8(const GView& v, int64_t g, int dim, int c, float (&f)[8]) {
  const float4 a = load_feat4_global<DT>(v.feats, v.scale, g, dim, c);
  const float4 b = load_feat4_global<DT>(v.feats, v.scale, g, dim, c + 4);
  f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
  f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
}

constexpr int kSlots = 32;      // distinct selections of a tile given slots
constexpr int kPosCap = 2048;   // list positions covered by the slot bitmap
constexpr int kGeo = 6;         // d/d(a, b, c, o, u, v)
constexpr int kNB = 4;          // 16-column MFMA blocks per wave and round

// LDS of the backward (the walk's staging and per-pixel scalars, then the
// slot map and the geometric sums).
struct BwdLds {
  float2 mean[kTilePix];
  float4 co[kTilePix];
  float thr[QR_MAX_K + 1];
  float inv[kTilePix];
  int ns[kTilePix];
  uint32_t smask[kTilePix];         // per pixel: slots it selected
  uint32_t bm[kPosCap / 32];        // selected positions, relative to the list start
  int bpre[kPosCap / 32];           // slots before each bitmap word
  int sgid[kSlots];                 // Gaussian id of each slot
  float geo[4][kSlots * kGeo];      // geometric gradient sums, per wave
  int nslot;
};

__device__ __forceinline__ int slot_of(const BwdLds& B, int r) {
  if (r >= kPosCap) return -1;
  const int s = B.bpre[r >> 5] + __popc(B.bm[r >> 5] & ((1u << (r & 31)) - 1u));
  return s < kSlots ? s : -1;
}

// Row of dL/d(out) of tile pixel p (clamped into the image: rows of pixels
// outside it are never used).
__device__ __forceinline__ const QR_GLOBAL float* grad_row(const GView& v, const GGrad& gg, int tx,
                                                           int ty, int p, int dim) {
  const int gx = min(tx * kTile + (p % kTile), v.W - 1);
  const int gy = min(ty * kTile + (p / kTile), v.H - 1);
  return gg.grad_out + (static_cast<int64_t>(gy) * v.W + gx) * dim;
}

// Raw operands of one 32-column step of slot_dots.
struct DotStep {
  f32x4 a[4][2];  // g_p, columns c .. c+7, of the lane's pixel in each 16-pixel block
  float f[2][8];  // f_s, columns c .. c+7, of the lane's slot in each 16-slot block
};

// D[p][s] = <g_p, f_s> for the wave's 64 pixels and the tile's slots, stored
// to s_d at the place of slot s in pixel p's selection list. The operands of
// step k+1 are requested before step k is multiplied (a fixed number of
// loads per step, every address clamped into range).
template <int DT>
__device__ __forceinline__ void slot_dots(const GView& v, const GGrad& gg, const BwdLds& B,
                                          int nslot, int tx, int ty, int wave, int lane, int dim,
                                          float* __restrict__ s_d, int KP) {
  const int row = lane & 15, kq = (lane >> 4) * 8;
  const int n_nb = (nslot + 15) >> 4;  // 1 or 2 blocks of 16 slots
  int gid[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) gid[nb] = B.sgid[min(nb * 16 + row, nslot - 1)];
  const QR_GLOBAL float* arow[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) arow[mb] = grad_row(v, gg, tx, ty, wave * 64 + mb * 16 + row, dim);
  floatx4 acc[4][2];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nk = (dim + 31) >> 5;
  auto load = [&](int k, DotStep& o) {
    const int c = min(k * 32 + kq, dim - 8);  // dim is a multiple of 8
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      o.a[mb][0] = *reinterpret_cast<const QR_GLOBAL f32x4*>(arow[mb] + c);
      o.a[mb][1] = *reinterpret_cast<const QR_GLOBAL f32x4*>(arow[mb] + c + 4);
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) load_feat8<DT>(v, gid[nb], dim, c, o.f[nb]);
  };
  auto multiply = [&](int k, const DotStep& o) {
    const bool live = k * 32 + kq < dim;  // columns past dim contribute zero
    bf16x8 ahi[4], alo[4], bhi[2], blo[2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      float x[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = live ? o.a[mb][0][i] : 0.f;
        x[4 + i] = live ? o.a[mb][1][i] : 0.f;
      }
      split8(x, ahi[mb], alo[mb]);
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) split8(o.f[nb], bhi[nb], blo[nb]);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      if (nb >= n_nb) continue;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mb], bhi[nb], acc[mb][nb], 0, 0, 0);
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[mb], bhi[nb], acc[mb][nb], 0, 0, 0);
        if (DT != QR_BF16)  // bf16 features are exact in their high part
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mb], blo[nb], acc[mb][nb], 0, 0, 0);
      }
    }
  };
  DotStep X, Y;
  load(0, X);
  for (int k = 0; k < nk; k += 2) {
    load(min(k + 1, nk - 1), Y);
    multiply(k, X);
    load(min(k + 2, nk - 1), X);
    if (k + 1 < nk) multiply(k + 1, Y);
  }
  // accumulator layout: lane holds D[4 (lane / 16) + i][lane % 16]
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = wave * 64 + mb * 16 + 4 * (lane >> 4) + i;
      const uint32_t m = B.smask[p];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int sl = nb * 16 + row;
        if (sl < nslot && ((m >> sl) & 1u)) s_d[p * KP + __popc(m & ((1u << sl) - 1u))] = acc[mb][nb][i];
      }
    }
  }
}

// dF[s][c] = sum_p (w_ps / Z_p) g_p[c] for the tile's slots and this wave's
// column blocks, added to grad_features. A wave takes kNB consecutive
// 16-column blocks per round (blocks 4 kNB r + kNB wave .. + kNB - 1 in round
// r), so its loads of one pixel row cover whole 128-byte lines instead of the
// halves that alternating waves would request at different times. The
// dL/d(out) operand of step k+1 is requested before step k is multiplied.
__device__ __forceinline__ void slot_feature_grads(const GView& v, const GGrad& gg, const BwdLds& B,
                                                   const float* __restrict__ s_sel_w, int nslot,
                                                   int tx, int ty, int wave, int lane, int dim,
                                                   int KP) {
  const int row = lane & 15, kq = (lane >> 4) * 8;
  const int n_mb = (nslot + 15) >> 4;
  const int n_blk = dim >> 4;
  constexpr int kSteps = kTilePix / 32;
  for (int b0 = wave * kNB; b0 < n_blk; b0 += 4 * kNB) {
    floatx4 acc[2][kNB];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < kNB; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    int col[kNB];
#pragma unroll
    for (int nb = 0; nb < kNB; ++nb) col[nb] = min(b0 + nb, n_blk - 1) * 16 + row;  // clamped
    // B = G: pixels k*32 + kq .. + 7, column col[nb]. Plain (caching) loads:
    // the dots pass reads the same rows next and finds them in the caches
    // (with non-temporal loads the backward took 8% longer).
    auto load = [&](int k, float (&x)[kNB][8]) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const QR_GLOBAL float* r = grad_row(v, gg, tx, ty, k * 32 + kq + t, dim);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) x[nb][t] = r[col[nb]];
      }
    };
    auto multiply = [&](int k, const float (&x)[kNB][8]) {
      // A = W^T: slot mb * 16 + row, pixels k*32 + kq .. + 7
      bf16x8 ahi[2], alo[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int sl = mb * 16 + row;
        float w[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int p = k * 32 + kq + t;
          const uint32_t m = B.smask[p];
          w[t] = ((m >> sl) & 1u) ? s_sel_w[p * KP + __popc(m & ((1u << sl) - 1u))] * B.inv[p] : 0.f;
        }
        split8(w, ahi[mb], alo[mb]);
      }
#pragma unroll
      for (int nb = 0; nb < kNB; ++nb) {
        bf16x8 bhi, blo;
        split8(x[nb], bhi, blo);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          if (mb >= n_mb) continue;
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mb], bhi, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[mb], bhi, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mb], blo, acc[mb][nb], 0, 0, 0);
        }
      }
    };
    float X[kNB][8], Y[kNB][8];
    load(0, X);
#pragma unroll 1
    for (int k = 0; k < kSteps; k += 2) {
      load(k + 1, Y);
      multiply(k, X);
      load(min(k + 2, kSteps - 1), X);
      multiply(k + 1, Y);
    }
    // lane holds dF[4 (lane / 16) + i][lane % 16] of each block
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int sl = mb * 16 + 4 * (lane >> 4) + i;
        if (sl >= nslot) continue;
        QR_GLOBAL float* dst = gg.grad_features + static_cast<int64_t>(B.sgid[sl]) * dim + row;
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
          const int blk = b0 + nb;
          if (blk < n_blk && acc[mb][nb][i] != 0.f) atomic_add(dst + blk * 16, acc[mb][nb][i]);
        }
      }
    }
  }
}

// Selections without a slot, for the wave's pixels, one selection at a time
// over the wave's lanes. DOTS = false: feature gradients w g / Z added to
// global memory (reads the weights); DOTS = true: the dots <g, f_j>, written
// over the weight of the same selection (s_d aliases s_sel_w).
template <int DT, bool DOTS>
__device__ __forceinline__ void slotless(const GView& v, const GGrad& gg, const BwdLds& B,
                                         const int* __restrict__ s_sel_pos,
                                         float* __restrict__ s_sel_w, int tx, int ty, int wave,
                                         int lane, int dim, int ns, int KP) {
  const int p_own = wave * 64 + lane;
  const int nfree = ns - __popc(B.smask[p_own]);  // slotted selections come first
  uint64_t todo = __ballot(nfree > 0);
  while (todo) {
    const int l = __builtin_ctzll(todo);
    todo &= todo - 1ull;
    const int p = wave * 64 + l;
    const int n = __builtin_amdgcn_readfirstlane(B.ns[p]);
    const int j0 = __popc(B.smask[p]);
    const float inv = B.inv[p];
    const QR_GLOBAL float* grow = grad_row(v, gg, tx, ty, p, dim);
    for (int j = j0; j < n; ++j) {
      const int pos = __builtin_amdgcn_readfirstlane(s_sel_pos[p * KP + j]);
      const int g = static_cast<int>(__builtin_amdgcn_readfirstlane(v.sorted_gid[pos]));
      if constexpr (DOTS) {
        float dot = 0.f;
        for (int c = 4 * lane; c < dim; c += 256) {
          const f32x4 gx = *reinterpret_cast<const QR_GLOBAL f32x4*>(grow + c);
          const float4 f = load_feat4_global<DT>(v.feats, v.scale, g, dim, c);
          dot += gx.x * f.x + gx.y * f.y + gx.z * f.z + gx.w * f.w;
        }
        const float t = wave_sum(dot);
        if (lane == 0) s_sel_w[p * KP + j] = t;
      } else {
        const float w = s_sel_w[p * KP + j] * inv;
        QR_GLOBAL float* dst = gg.grad_features + static_cast<int64_t>(g) * dim;
        for (int c = 4 * lane; c < dim; c += 256) {
          const f32x4 gx = *reinterpret_cast<const QR_GLOBAL f32x4*>(grow + c);
          atomic_add(dst + c + 0, w * gx.x);
          atomic_add(dst + c + 1, w * gx.y);
          atomic_add(dst + c + 2, w * gx.z);
          atomic_add(dst + c + 3, w * gx.w);
        }
      }
    }
  }
}

// Backward of one tile (all 256 threads of the workgroup). Per-pixel LDS:
// the walk's selected positions and weights ([256][KP] each); once the
// feature gradients (which read the weights) are done, the dots d_j are
// written over the weights, and the sweep recomputes each weight and T^Q_j
// from the records with the walk's own float operations.
template <int DT>
__device__ __forceinline__ void quantile_backward_tile(const GView& v, const GGrad& gg, int tile,
                                                       int K, int dim, const qr_params& prm,
                                                       BwdLds& B, int* __restrict__ s_sel_pos,
                                                       float* __restrict__ s_sel_w) {
  const int tiles_x = (v.W + kTile - 1) / kTile;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: addresses stay scalar
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid % kTile);
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < v.W && py < v.H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;
  const int lo = static_cast<int>(v.tile_offsets[tile]);
  const int hi = static_cast<int>(v.tile_offsets[tile + 1]);
  const int KP = (K + 3) & ~3;
  const PixelSel sel = quantile_walk<QR_SELECT_QUANTILE>(v, lo, hi, K, pxc, pyc, inside, prm, B, s_sel_pos, s_sel_w, KP);
  const int ns = sel.ns;
  const int* my_pos = s_sel_pos + tid * KP;
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
    if (tid == kPosCap / 32 - 1) B.nslot = min(incl, kSlots);
  }
  for (int i = tid; i < 4 * kSlots * kGeo; i += kTilePix) (&B.geo[0][0])[i] = 0.f;
  __syncthreads();
  {
    uint32_t m = 0u;
    for (int j = 0; j < ns; ++j) {
      const int s = slot_of(B, my_pos[j] - lo);
      if (s < 0) break;  // slots are ranks in list order: the slotted selections come first
      m |= 1u << s;
      B.sgid[s] = static_cast<int>(v.sorted_gid[my_pos[j]]);  // same value from every writer
    }
    B.smask[tid] = m;
  }
  __syncthreads();
  const int nslot = B.nslot;

  if (gg.grad_features) {
    // ---- feature gradients (read every pixel's weights) ----
    if (nslot > 0) slot_feature_grads(v, gg, B, s_sel_w, nslot, tx, ty, wave, lane, dim, KP);
    slotless<DT, false>(v, gg, B, s_sel_pos, s_sel_w, tx, ty, wave, lane, dim, ns, KP);
  }
  if (!geo) return;
  __syncthreads();  // every wave is done with the weights before they are overwritten

  // ---- dots d_pj, written over the weights (wave-local) ----
  float* s_d = s_sel_w;
  if (nslot > 0) slot_dots<DT>(v, gg, B, nslot, tx, ty, wave, lane, dim, s_d, KP);
  slotless<DT, true>(v, gg, B, s_sel_pos, s_sel_w, tx, ty, wave, lane, dim, ns, KP);
  wave_lds_sync();

  // ---- sweep over this pixel's selections ----
  // Weights and T^Q_j are recomputed front to back exactly as the walk formed
  // them; the tail sums S_j = sum_{l > j} w_l d_l are taken as the total
  // minus the running prefix, both in double.
  if (ns > 0) {
    const float TQ = sel.TQ;
    const float invZ = 1.f / (1.f - TQ);
    const float* my_d = s_d + tid * KP;
    double tot = 0.0;
    {
      float tq = 1.f;
      for (int j = 0; j < ns; ++j) {
        const int g = static_cast<int>(v.sorted_gid[my_pos[j]]);
        const f32x2 m = v.means2d[g];
        const f32x4 c = v.conic_opacity[g];
        const float a = gauss_alpha(make_float2(m.x, m.y), make_float4(c.x, c.y, c.z, c.w), pxc, pyc,
                                    prm.alpha_max);
        tot += static_cast<double>(tq * a) * my_d[j];
        tq = tq * (1.f - a);
      }
    }
    const float gout = static_cast<float>(tot) * invZ;  // <g, out>
    float tq = 1.f;
    double pre = 0.0;
    for (int j = 0; j < ns; ++j) {
      const int g = static_cast<int>(v.sorted_gid[my_pos[j]]);
      const f32x2 m = v.means2d[g];
      const f32x4 c = v.conic_opacity[g];
      const AlphaEval e = eval_alpha(make_float2(m.x, m.y), make_float4(c.x, c.y, c.z, c.w), pxc,
                                     pyc, prm.alpha_max);
      const float wj = tq * e.alpha, dj = my_d[j];
      pre += static_cast<double>(wj) * dj;
      const float S = static_cast<float>(tot - pre);  // sum over the later selections
      const float dL_da = invZ * (tq * dj - (S + gout * TQ) / (1.f - e.alpha));
      tq = tq * (1.f - e.alpha);
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

// Two waves per SIMD (registers of the MFMA operands and accumulators).
constexpr int kBwdWavesPerSimd = 2;

__device__ __forceinline__ size_t bwd_sel_floats(int K) { return static_cast<size_t>(kTilePix) * ((K + 3) & ~3); }

template <int DT>
__global__ void __launch_bounds__(kTilePix, kBwdWavesPerSimd)
quantile_backward_kernel(ViewArgs v, GradPtrs gp, int n_tiles, qr_params prm, int K, int dim) {
  extern __shared__ unsigned char dyn_lds[];
  __shared__ BwdLds B;
  const size_t n = bwd_sel_floats(K);
  int* s_sel_pos = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + n;
  quantile_backward_tile<DT>(to_global(v), to_global(gp), xcd_remap(blockIdx.x, n_tiles), K, dim,
                             prm, B, s_sel_pos, s_sel_w);
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
  __shared__ BwdLds B;
  const size_t n = bwd_sel_floats(K);
  int* s_sel_pos = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + n;
  const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[xcd_remap(blockIdx.x, n_items)]);
  const uint32_t vi = packed >> kViewShift;
  quantile_backward_tile<DT>(to_global(view_args(views[vi])), to_global(grad_ptrs(grads[vi])),
                             static_cast<int>(packed & kTileMask), K, dim, prm, B, s_sel_pos,
                             s_sel_w);
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
  __shared__ BwdLds B;
  __shared__ uint32_t s_item[2];
  const size_t n = bwd_sel_floats(K);
  int* s_sel_pos = reinterpret_cast<int*>(dyn_lds);
  float* s_sel_w = reinterpret_cast<float*>(dyn_lds) + n;
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
    quantile_backward_tile<DT>(to_global(view_args(views[vi])), to_global(grad_ptrs(grads[vi])),
                               static_cast<int>(packed & kTileMask), K, dim, prm, B, s_sel_pos,
                               s_sel_w);
  }
}

__global__ void reset_bwd_counter_kernel(uint32_t* __restrict__ c) {
  if (threadIdx.x < kBwdXcdQueues) c[threadIdx.x] = 0u;
}

inline size_t bwd_dynamic_lds(int K) {
  return static_cast<size_t>(kTilePix) * ((K + 3) & ~3) * 2 * sizeof(float);
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
  if (prm->selection != QR_SELECT_QUANTILE)
    return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_backward: the quantile selection only");
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
  if (prm->selection != QR_SELECT_QUANTILE)
    return fail(QR_ERR_UNSUPPORTED, "%s: the quantile selection only", name);
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
