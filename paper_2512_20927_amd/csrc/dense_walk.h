// The transmittance walk of the dense blend (Eq. 1) over one batch of 32
// list entries split over the four waves of a workgroup, eight entries each,
// with one pixel per lane (the same pixel in every wave). Shared by the
// forward strip kernel and the backward, so that both form bit-identical
// weights:
//   1. each wave takes alpha' of its eight entries and the product of their
//      (1 - alpha') (walk_alpha8);
//   2. with the products of the earlier waves, each wave knows T at the
//      start of its eight entries and forms their weights in list order with
//      the stop test (walk_weights8). A stop in an earlier eight leaves T
//      below T_eps there, so a later eight stops at its first entry (its T
//      differs from the sequential chain's only in rounding, and one more
//      factor 1 - alpha' <= 1 - alpha_min keeps it below T_eps);
//   3. every wave folds the four results into the pixel's T, stop flag and
//      last blended position identically (walk_fold).
#pragma once

#include "render_common.h"

namespace qr {

constexpr int kWalkBatch = 32;        // list entries per batch
constexpr int kWalkQ = 8;             // entries per wave
constexpr uint32_t kWalkStop = 0x100u;  // stop flag of a wave's result word

// alpha' of entries e0 .. e0 + 7 (0 below alpha_min, past cnt or once the
// pixel is done) and the product of their (1 - alpha').
__device__ __forceinline__ float walk_alpha8(const float2* mean, const float4* co, int e0, int cnt,
                                             bool done, float pxc, float pyc, const qr_params& prm,
                                             float (&al)[kWalkQ]) {
  float part = 1.f;
#pragma unroll
  for (int j = 0; j < kWalkQ; ++j) {
    const int e = e0 + j;
    al[j] = 0.f;
    if (e < cnt && !done) {
      const float a = gauss_alpha(mean[e], co[e], pxc, pyc, prm.alpha_max);
      if (a >= prm.alpha_min) {
        al[j] = a;
        part *= 1.f - a;
      }
    }
  }
  return part;
}

// Weights of the eight entries from T at their start (Tl, updated to T after
// the last blended one), in list order with the stop test. Returns the
// index of the last blended entry (0xFF: none) with kWalkStop if the stop
// test fired.
__device__ __forceinline__ uint32_t walk_weights8(float& Tl, const float (&al)[kWalkQ], float T_eps,
                                                  float (&w)[kWalkQ]) {
  bool stopped = false;
  uint32_t last = 0xFFu;
#pragma unroll
  for (int j = 0; j < kWalkQ; ++j) {
    w[j] = 0.f;
    if (al[j] > 0.f && !stopped) {
      const float T_test = Tl * (1.f - al[j]);
      if (T_test < T_eps) {
        stopped = true;
      } else {
        w[j] = al[j] * Tl;
        Tl = T_test;
        last = static_cast<uint32_t>(j);
      }
    }
  }
  return last | (stopped ? kWalkStop : 0u);
}

// The pixel's state after the batch from the four waves' results (tend[q]:
// T after wave q's entries, info[q]: walk_weights8's word), in list order.
// T moves only with a blended entry (T_test >= T_eps), so it never falls
// below T_eps. ncon: list position + 1 (from the batch start `base`) of the
// last blended entry.
__device__ __forceinline__ void walk_fold(const float* tend, const uint32_t* info, int stride,
                                          int lane, int base, float& T, bool& done, int& ncon) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!done) {
      const uint32_t inf = info[q * stride + lane];
      if ((inf & 0xFFu) != 0xFFu) {
        ncon = base + kWalkQ * q + static_cast<int>(inf & 0xFFu) + 1;
        T = tend[q * stride + lane];
      }
      if (inf & kWalkStop) done = true;
    }
  }
}

}  // namespace qr
