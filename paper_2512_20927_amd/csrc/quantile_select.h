// Selection phase of Quantile Rendering (Algorithm 1, Sec. 4.2) for one
// 16x16 tile, shared by the forward renderer and its backward pass so that
// both make exactly the same selections:
//  - the walk: the tile's depth-sorted list is staged into LDS in batches of
//    256 projected records and every pixel (one thread each) runs the
//    transmittance chain T_test = T (1 - alpha') with the threshold test
//    T_test < t_{k+1}, recording the <= K selected list positions and their
//    weights w^Q = T^Q alpha'; a pixel is done once all K thresholds are
//    consumed (the same event as the stop test T_test < 1/(K+1)) and the
//    workgroup leaves the list once every pixel is done;
//  - the merge: each group of four adjacent pixels (a row segment of the
//    tile) has its four selection lists, ordered by list position, merged
//    into its distinct selections, each carrying the four pixels' weights
//    divided by the pixel's 1 - T^Q (0 where a pixel did not select it) and a
//    mask of the pixels that selected it. The pixels of wave w are tile rows
//    4w .. 4w+3, exactly the pixels of the groups it merges, so the merge and
//    everything after it are wave-local.
#pragma once

#include "common.h"
#include "render_common.h"

namespace qr {

constexpr int kViewShift = QR_BATCH_TILE_BITS;
constexpr uint32_t kTileMask = (1u << QR_BATCH_TILE_BITS) - 1u;

constexpr int kPG = 4;                     // pixels gathered together
constexpr int kGroups = kTilePix / kPG;    // 64 pixel groups per tile
// Distinct selections kept per merged group: 16, or 32 for 24 < K <= 52,
// where the selection lists already hold the kernel to one workgroup per CU
// (at K = 40 about 44% of the room workload's groups have more than 16
// distinct selections and 0.1% more than 32).
constexpr int kUCap = 16;
constexpr int kUCapLarge = 32;
constexpr int kUCapLargeMinK = 25;
constexpr int kUCapLargeMaxK = 52;
__host__ __device__ constexpr int ucap_for(int K) {
  return K >= kUCapLargeMinK && K <= kUCapLargeMaxK ? kUCapLarge : kUCap;
}
// Three 45 KB workgroups fill a CU's LDS: registers are bounded to match
// (three waves per SIMD).
constexpr int kWavesPerSimd = 3;

// LDS of one workgroup: record staging, thresholds, per-pixel scalars and
// the merged groups of up to UCAP distinct selections (each pixel's [K]
// selections live in dynamic LDS).
template <int UCAP>
struct QuantileLdsT {
  static constexpr int kCap = UCAP;
  float2 mean[kTilePix];
  float4 co[kTilePix];
  float thr[QR_MAX_K + 1];
  double zq[QR_MAX_K];                     // Stratified-K: z_m, m = 1..K
  float inv[kTilePix];
  int ns[kTilePix];
  int unum[kGroups];                       // distinct entries per group, -1 if over UCAP
  int ugid[kGroups * UCAP];                // a group's distinct selections (list positions until converted)
  float4 uw[kGroups * UCAP];               // their weights for the group's four pixels, x = first pixel
  uint8_t umask[kGroups * UCAP];           // bit q: pixel q of the group selected the entry
};
using QuantileLds = QuantileLdsT<kUCap>;

struct ViewArgs {
  int W, H;
  const uint32_t* __restrict__ tile_offsets;
  const uint32_t* __restrict__ sorted_gid;
  const float2* __restrict__ means2d;
  const float4* __restrict__ conic_opacity;
  const void* __restrict__ feats;
  const float* __restrict__ scale;
  float* __restrict__ out;
  float* __restrict__ T_q;
  int32_t* __restrict__ n_sel;
};

// The same view with global-memory pointers (see QR_GLOBAL), as the tile
// code uses it.
struct GView {
  int W, H;
  const QR_GLOBAL uint32_t* __restrict__ tile_offsets;
  const QR_GLOBAL uint32_t* __restrict__ sorted_gid;
  const QR_GLOBAL f32x2* __restrict__ means2d;
  const QR_GLOBAL f32x4* __restrict__ conic_opacity;
  const QR_GLOBAL void* __restrict__ feats;
  const QR_GLOBAL float* __restrict__ scale;
  QR_GLOBAL float* __restrict__ out;
  QR_GLOBAL float* __restrict__ T_q;
  QR_GLOBAL int32_t* __restrict__ n_sel;
};

__device__ __forceinline__ GView to_global(const ViewArgs& v) {
  return GView{v.W, v.H,
               (const QR_GLOBAL uint32_t*)v.tile_offsets, (const QR_GLOBAL uint32_t*)v.sorted_gid,
               (const QR_GLOBAL f32x2*)v.means2d, (const QR_GLOBAL f32x4*)v.conic_opacity,
               (const QR_GLOBAL void*)v.feats, (const QR_GLOBAL float*)v.scale,
               (QR_GLOBAL float*)v.out, (QR_GLOBAL float*)v.T_q, (QR_GLOBAL int32_t*)v.n_sel};
}

// Orders this wave's LDS writes before its later LDS reads (all lanes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ ViewArgs view_args(const qr_view& qv) {
  return ViewArgs{qv.width, qv.height, qv.tile_offsets, qv.sorted_gid,
                  reinterpret_cast<const float2*>(qv.means2d),
                  reinterpret_cast<const float4*>(qv.conic_opacity), qv.features,
                  qv.feature_scale, qv.out, qv.T_q, qv.n_sel};
}

// What the walk leaves in registers for the calling thread's pixel.
struct PixelSel {
  int ns;    // selections (0 outside the image)
  float TQ;  // T^Q after the last selection
  float T;   // Algorithm 1: full transmittance when the walk ends (the stop
             // test breaks before T takes the stopping entry's T_test)
  int last;  // Algorithm 1: list position + 1 of the last on-ray entry examined
};

// The walk for one tile (all 256 threads of the workgroup). Selections go to
// s_sel_pos / s_sel_w ([256][KP], as absolute positions in sorted_gid and
// w^Q); L (any LDS struct with the staging arrays mean, co, the thresholds
// thr and the per-pixel ns, inv) receives ns (-1 outside the image) and
// 1 / (1 - T^Q). Workgroup barriers occur only around the staging of record
// batches; the record batch is only rewritten after a barrier that every
// wave reaches once it has finished the previous tile.
// MODE QR_SELECT_QUANTILE: Algorithm 1's thresholds t_m = 1 - m/(K+1).
// MODE QR_SELECT_STRATIFIED (Stratified-K, Appendix): a first pass over the
// list estimates the mean and spread of the ray's transmittance values (T_0 =
// 1 and T after every Gaussian the dense blend composites, with its T_eps
// stop; sums in double) and the thresholds are the ray's own; the second
// pass examines the same Gaussians (it also ends at the dense stop).
// MODE QR_SELECT_TOPK (the Top-K sampler the paper compares with): the
// candidates are the Gaussians the dense blend composites (same T_eps stop),
// each with its dense weight T alpha'; the K largest are kept (equal weights:
// the earlier position), then put back in list order; 1 / (1 - T^Q) becomes
// 1 / (sum of the kept weights) and T^Q reports 1 - that sum. A pixel is done
// once its list is full and T alpha_max is no larger than the smallest kept
// weight: no later weight can exceed it.
template <int MODE, class WalkLds>
__device__ __forceinline__ PixelSel quantile_walk(const GView& v, int lo, int hi, int K, float pxc,
                                                  float pyc, bool inside, const qr_params& prm,
                                                  WalkLds& L, int* __restrict__ s_sel_pos,
                                                  float* __restrict__ s_sel_w, int KP) {
  const int tid = threadIdx.x;
  // thr[k] = t_{k+1}; thr[K] = 0 (identical for every tile of a launch)
  if (MODE == QR_SELECT_QUANTILE && tid <= K) L.thr[tid] = quantile_threshold(tid + 1, K);
  if constexpr (MODE == QR_SELECT_STRATIFIED) {
    if (tid < K) L.zq[tid] = stratified_z(tid + 1, K);  // read after the barrier below
    __syncthreads();
  }
  const float amin = prm.alpha_min, amax = prm.alpha_max;

  double mu = 0.0, sigma = 0.0;
  if constexpr (MODE == QR_SELECT_STRATIFIED) {
    double s1 = 1.0, s2 = 1.0;  // T_0 = 1
    int n = 1;
    float T1 = 1.f;
    bool stop = !inside;
    for (int batch = lo; batch < hi; batch += kTilePix) {
      if (__syncthreads_count(!stop) == 0) break;
      const int idx = batch + tid;
      if (idx < hi) {
        const int g = static_cast<int>(v.sorted_gid[idx]);
        const f32x2 m = v.means2d[g];
        const f32x4 c = v.conic_opacity[g];
        L.mean[tid] = make_float2(m.x, m.y);
        L.co[tid] = make_float4(c.x, c.y, c.z, c.w);
      } else {  // padding record: opacity 0 is below alpha_min on every ray
        L.mean[tid] = make_float2(0.f, 0.f);
        L.co[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      __syncthreads();
      constexpr int kU = 8;  // records read from LDS per round trip
      const int cnt_pad = (min(kTilePix, hi - batch) + kU - 1) & ~(kU - 1);
      for (int j = 0; j < cnt_pad; j += kU) {
        if (__all(stop)) break;
        float2 rm[kU];
        float4 rc[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          rm[u] = L.mean[j + u];
          rc[u] = L.co[j + u];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const float alpha = gauss_alpha(rm[u], rc[u], pxc, pyc, amax);
          if (stop || alpha < amin) continue;
          const float T_test = T1 * (1.f - alpha);
          if (T_test < prm.T_eps) {
            stop = true;
          } else {
            T1 = T_test;
            s1 += T1;
            s2 += static_cast<double>(T1) * T1;
            ++n;
          }
        }
      }
    }
    mu = s1 / n;
    sigma = sqrt(fmax(s2 / n - mu * mu, 0.0));
  }
  auto threshold = [&](int kk) -> float {  // t_{kk+1}; past t_K none is crossed
    if constexpr (MODE == QR_SELECT_STRATIFIED) return kk < K ? stratified_threshold_z(L.zq[kk], mu, sigma) : -1.f;
    else return L.thr[kk];
  };

  float T = 1.f, TQ = 1.f;
  int k = 0, ns = 0, last = 0;
  bool done = !inside;
  // t_{k+1}: changes only at a crossing
  float thr_k;
  if constexpr (MODE == QR_SELECT_STRATIFIED) thr_k = threshold(0);
  else thr_k = quantile_threshold(1, K);
  int* my_pos = s_sel_pos + tid * KP;
  float* my_w = s_sel_w + tid * KP;
  float wmin = 0.f;  // Top-K: the worst kept entry (smallest weight, later position among equals)
  int imin = 0;

  for (int batch = lo; batch < hi; batch += kTilePix) {
    if (__syncthreads_count(!done) == 0) break;
    const int idx = batch + tid;
    if (idx < hi) {
      const int g = static_cast<int>(v.sorted_gid[idx]);
      const f32x2 m = v.means2d[g];
      const f32x4 c = v.conic_opacity[g];
      L.mean[tid] = make_float2(m.x, m.y);
      L.co[tid] = make_float4(c.x, c.y, c.z, c.w);
    } else {  // padding record: opacity 0 is below alpha_min on every ray
      L.mean[tid] = make_float2(0.f, 0.f);
      L.co[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    // kWalkUnroll records are read from LDS before any is used (one LDS round
    // trip per group of records; the padding makes every group whole)
    constexpr int kWalkUnroll = 8;
    const int cnt_pad = (min(kTilePix, hi - batch) + kWalkUnroll - 1) & ~(kWalkUnroll - 1);
    for (int j = 0; j < cnt_pad; j += kWalkUnroll) {
      if (__all(done)) break;
      float2 rm[kWalkUnroll];
      float4 rc[kWalkUnroll];
#pragma unroll
      for (int u = 0; u < kWalkUnroll; ++u) {
        rm[u] = L.mean[j + u];
        rc[u] = L.co[j + u];
      }
#pragma unroll
      for (int u = 0; u < kWalkUnroll; ++u) {
        const float alpha = gauss_alpha(rm[u], rc[u], pxc, pyc, amax);
        if (done || alpha < amin) continue;  // finished, or not on this pixel's ray
        const float T_test = T * (1.f - alpha);
        if constexpr (MODE == QR_SELECT_TOPK) {
          if (T_test < prm.T_eps) {  // the dense blend stops before this Gaussian
            done = true;
            continue;
          }
          const float w = T * alpha;
          const int pos = batch + j + u;
          if (ns < K) {
            my_pos[ns] = pos;
            my_w[ns] = w;
            if (ns == 0 || w <= wmin) {
              wmin = w;
              imin = ns;
            }
            ++ns;
          } else if (w > wmin) {
            my_pos[imin] = pos;
            my_w[imin] = w;
            int pmin = my_pos[0];
            wmin = my_w[0];
            imin = 0;
            for (int e = 1; e < K; ++e) {
              const float we = my_w[e];
              const int pe = my_pos[e];
              if (we < wmin || (we == wmin && pe > pmin)) {
                wmin = we;
                imin = e;
                pmin = pe;
              }
            }
          }
          T = T_test;
          if (ns == K && T * amax <= wmin) done = true;
          continue;
        }
        if (MODE == QR_SELECT_STRATIFIED && T_test < prm.T_eps) {  // the sampled ray ends here
          done = true;
          continue;
        }
        if constexpr (MODE == QR_SELECT_QUANTILE) last = batch + j + u - lo + 1;
        if (T_test < thr_k) {  // crossing: a quantile Gaussian
          my_pos[ns] = batch + j + u;
          my_w[ns] = TQ * alpha;
          ++ns;
          TQ = TQ * (1.f - alpha);
          ++k;
          while (k < K && T_test < threshold(k)) ++k;  // thresholds crossed by the same step
          thr_k = threshold(k);
          if (k == K) done = true;
        }
        // Algorithm 1 leaves T at the stopping entry (the stop test comes first)
        if (MODE != QR_SELECT_QUANTILE || !done) T = T_test;
      }
    }
  }
  if constexpr (MODE == QR_SELECT_TOPK) {
    // back to list order (insertion sort of at most K entries), weight sum
    for (int a = 1; a < ns; ++a) {
      const int p = my_pos[a];
      const float w = my_w[a];
      int b = a - 1;
      while (b >= 0 && my_pos[b] > p) {
        my_pos[b + 1] = my_pos[b];
        my_w[b + 1] = my_w[b];
        --b;
      }
      my_pos[b + 1] = p;
      my_w[b + 1] = w;
    }
    float sum = 0.f;
    for (int a = 0; a < ns; ++a) sum += my_w[a];
    TQ = 1.f - sum;
    L.ns[tid] = inside ? ns : -1;
    L.inv[tid] = ns > 0 ? 1.f / sum : 0.f;
    wave_lds_sync();
    return PixelSel{ns, TQ, T, last};
  }
  L.ns[tid] = inside ? ns : -1;
  L.inv[tid] = ns > 0 ? 1.f / (1.f - TQ) : 0.f;
  wave_lds_sync();

  return PixelSel{ns, TQ, T, last};
}

// The merge for one tile (all 256 threads; wave-local), after the walk.
template <class Lds>
__device__ __forceinline__ void merge_groups(const GView& v, Lds& L,
                                             const int* __restrict__ s_sel_pos,
                                             const float* __restrict__ s_sel_w, int KP) {
  constexpr int kCap = Lds::kCap;
  const int tid = threadIdx.x;
  // The merge, wave-local: adjacent pixels select mostly the same
  // Gaussians, so a group's distinct selections are far fewer than its
  // pixels' selections. Lane l < 16 merges group 16 w + l.
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int kWaveGroups = kGroups / 4;
  if (lane < kWaveGroups) {
    const int grp = wave * kWaveGroups + lane;
    const int p0 = grp * kPG;
    // each pixel's next selection (list position and weight) kept in registers
    // (weights are stored already divided by the pixel's 1 - T^Q)
    int n[kPG], idx[kPG], head[kPG];
    float hw[kPG], inv[kPG];
#pragma unroll
    for (int q = 0; q < kPG; ++q) {
      n[q] = max(L.ns[p0 + q], 0);
      inv[q] = L.inv[p0 + q];
      idx[q] = 0;
      head[q] = n[q] > 0 ? s_sel_pos[(p0 + q) * KP] : 0x7fffffff;
      hw[q] = n[q] > 0 ? s_sel_w[(p0 + q) * KP] * inv[q] : 0.f;
    }
    int cnt = 0;
    for (;;) {
      const int best = min(min(head[0], head[1]), min(head[2], head[3]));
      if (best == 0x7fffffff) break;
      if (cnt == kCap) {
        cnt = -1;
        break;
      }
      float wq[kPG];
      uint32_t mk = 0u;
#pragma unroll
      for (int q = 0; q < kPG; ++q) {
        wq[q] = 0.f;
        if (head[q] == best) {
          wq[q] = hw[q];
          mk |= 1u << q;
          ++idx[q];
          head[q] = idx[q] < n[q] ? s_sel_pos[(p0 + q) * KP + idx[q]] : 0x7fffffff;
          hw[q] = idx[q] < n[q] ? s_sel_w[(p0 + q) * KP + idx[q]] * inv[q] : 0.f;
        }
      }
      L.ugid[grp * kCap + cnt] = best;  // position for now
      L.uw[grp * kCap + cnt] = make_float4(wq[0], wq[1], wq[2], wq[3]);
      L.umask[grp * kCap + cnt] = static_cast<uint8_t>(mk);
      ++cnt;
    }
    L.unum[grp] = cnt;
    // positions -> Gaussian ids, 16 at a time: all loads of a batch issued
    // before any result is used
#pragma unroll
    for (int e0 = 0; e0 < kCap; e0 += 16) {
      if (e0 >= cnt) break;
      int pos[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) pos[e] = e0 + e < cnt ? L.ugid[grp * kCap + e0 + e] : -1;
      uint32_t gid[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) gid[e] = pos[e] >= 0 ? v.sorted_gid[pos[e]] : 0u;
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (e0 + e < cnt) L.ugid[grp * kCap + e0 + e] = static_cast<int>(gid[e]);
    }
  }
  wave_lds_sync();
}

// Walk and merge (the forward renderer's selection phase).
template <int MODE, class Lds>
__device__ __forceinline__ PixelSel quantile_select(const GView& v, int lo, int hi, int K,
                                                    float pxc, float pyc, bool inside,
                                                    const qr_params& prm, Lds& L,
                                                    int* __restrict__ s_sel_pos,
                                                    float* __restrict__ s_sel_w, int KP) {
  const PixelSel sel = quantile_walk<MODE>(v, lo, hi, K, pxc, pyc, inside, prm, L, s_sel_pos, s_sel_w, KP);
  merge_groups(v, L, s_sel_pos, s_sel_w, KP);
  return sel;
}

}  // namespace qr
