// Dense alpha-blend forward (Eq. 1: out = sum_i T_i alpha'_i f_i over every
// Gaussian on the ray, stopping before T drops below T_eps).
//
// Per tile the output is a contraction W [px x G] . F [G x D] where
// W[p, g] = T_{p,g} alpha'_{p,g} (zero off the ray or after the stop) and F
// holds the feature rows of the tile's depth-sorted list. The unit of work is
// a strip of 64 pixels (4 rows of a 16x16 tile) over all D columns, so every
// pixel's transmittance chain is walked once:
//   - each lane of each wave owns one pixel of the strip (the same pixel in
//     all four waves); the list is taken 32 entries at a time and wave q
//     evaluates alpha' of entries 8q .. 8q+7 for its lane's pixel. The four
//     partial products of (1 - alpha') are exchanged through LDS, so each wave
//     knows T at the start of its eight entries and forms their weights; the
//     stop test is applied in list order within the eight, and a stop in an
//     earlier eight leaves T below T_eps there, which stops the later ones at
//     their first entry too (their T differs from the sequential chain's only
//     in rounding, and one more factor (1 - alpha') <= 1 - alpha_min takes it
//     below T_eps). Every wave then folds the four results into the pixel's
//     T, stop flag and last blended position identically;
//   - the weights go to LDS as bfloat16 pairs w = w_hi + w_lo; each wave
//     contracts them with its own column groups of F on
//     v_mfma_f32_16x16x32_bf16 as out^T = F^T W^T, both operands split into
//     bfloat16 pairs and the product formed as F_hi W_hi + F_lo W_hi +
//     F_hi W_lo with float32 accumulation (bfloat16 features are exact in
//     F_hi, so their F_lo term is dropped): float32-class accuracy (below
//     2^-16 of each product) at the bfloat16 matrix rate;
//   - the MFMA rows of a 64-column group are permuted (row i of column tile c
//     is column 16 (i % 4) + 4 (i / 4) + c), so that a lane's operand values
//     for the group's four column tiles are four consecutive features of one
//     row (one 16-byte load per list entry) and its results for one pixel are
//     four consecutive features (one 16-byte store);
//   - feature rows of a batch are requested before the walk, so their loads
//     overlap it; 16-pixel rows of the strip that take nothing from a batch
//     skip their MFMAs; the strip leaves the list once all 64 pixels stopped.
// Widths above 512 are rendered in passes of 512 columns, each walking again.
// Widths up to 64 take the tile kernels further down (dense_tile_narrow):
// one workgroup per tile, one sequential walk per pixel, one barrier per batch.
#include "common.h"
#include "dense_walk.h"
#include "quantile_select.h"
#include "render_common.h"

namespace qr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kStripRows = 4;                      // tile rows per strip
constexpr int kStripPix = kTile * kStripRows;      // 64: one pixel per lane
constexpr int kStrips = kTile / kStripRows;        // 4 strips per tile
constexpr int kDB = 32;                            // list entries per batch (MFMA K)
constexpr int kDQ = kDB / 4;                       // entries each wave walks per batch
constexpr int kGrpCols = 64;                       // columns of a group (4 MFMA column tiles)
constexpr int kWaveGroups = 2;                     // groups per wave and pass
constexpr int kPassCols = 4 * kWaveGroups * kGrpCols;  // 512 columns per pass
constexpr int kWS = kDB + 8;                       // LDS row stride (bf16) of a pixel's weights
static_assert(kDB == kWalkBatch && kDQ == kWalkQ, "the strip's batches are the split walk's");

struct DenseLds {
  __attribute__((aligned(16))) __bf16 whi[kStripPix * kWS];
  __attribute__((aligned(16))) __bf16 wlo[kStripPix * kWS];
  float2 mean[kDB];
  float4 co[kDB];
  // ids of the batch, double-buffered by batch parity: the second column
  // group's loads read them after the last barrier of the batch, while wave
  // 0 may already be staging the next batch
  __attribute__((aligned(16))) uint32_t gid[2][kDB];
  float part[4][kStripPix];   // product of (1 - alpha') over a wave's eight entries
  float tend[4][kStripPix];   // T after a wave's eight entries (before its stop)
  uint32_t info[4][kStripPix];  // walk_weights8's result word per wave
  unsigned long long busy[4];   // pixels with a non-zero weight, per wave
};

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  lo = static_cast<__bf16>(x - static_cast<float>(hi));
}

// Four consecutive features (d .. d+3) of row g as raw loads: float32 values,
// or bfloat16 codes in the low 8 bytes.
template <int DT>
__device__ __forceinline__ f32x4 load_raw4(const GView& v, uint32_t g, int dim, int d) {
  const uint64_t off = static_cast<uint64_t>(g) * static_cast<uint32_t>(dim) + static_cast<uint32_t>(d);
  if constexpr (DT == QR_F32) {
    return *reinterpret_cast<const QR_GLOBAL f32x4*>(static_cast<const QR_GLOBAL float*>(v.feats) + off);
  } else if constexpr (DT == QR_BF16) {
    const u32x2 r = *reinterpret_cast<const QR_GLOBAL u32x2*>(
        static_cast<const QR_GLOBAL uint16_t*>(v.feats) + off);
    return f32x4{__uint_as_float(r.x), __uint_as_float(r.y), 0.f, 0.f};
  } else {
    const uint32_t r = *reinterpret_cast<const QR_GLOBAL uint32_t*>(
        static_cast<const QR_GLOBAL uint8_t*>(v.feats) + off);
    const float4 x = e4m3x4_to_f32(r, v.scale[g]);
    return f32x4{x.x, x.y, x.z, x.w};
  }
}

// A operands (bfloat16 pairs) of one column group from its raw rows: column
// tile c takes component c of the lane's eight rows.
template <int DT>
__device__ __forceinline__ void convert_group(const f32x4 (&raw)[8], bf16x8 (&ahi)[4],
                                              bf16x8 (&alo)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if constexpr (DT != QR_BF16) {
        __bf16 h, l;
        split_bf16(raw[t][c], h, l);
        ahi[c][t] = h;
        alo[c][t] = l;
      } else {
        // bfloat16 codes: two per 32-bit word, column c in word c / 2
        const uint32_t word = __float_as_uint(raw[t][c >> 1]);
        const uint16_t code = static_cast<uint16_t>((c & 1) ? (word >> 16) : (word & 0xFFFFu));
        ahi[c][t] = __builtin_bit_cast(__bf16, code);
      }
    }
  }
}

// acc[c][p] += F^T W^T for one column group (4 column tiles) and the 4 pixel
// rows of 16 of a strip whose weights (bfloat16 pairs, row stride kWS) are at
// whi / wlo; pixel rows with no weight in `busy` are skipped.
template <int DT>
__device__ __forceinline__ void mfma_group(f32x4 (&acc)[4][4], const bf16x8 (&ahi)[4],
                                           const bf16x8 (&alo)[4], const __bf16* whi,
                                           const __bf16* wlo, unsigned long long busy, int ci,
                                           int kb) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (((busy >> (16 * p)) & 0xFFFFull) == 0ull) continue;
    const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(&whi[(16 * p + ci) * kWS + 8 * kb]);
    const bf16x8 blo = *reinterpret_cast<const bf16x8*>(&wlo[(16 * p + ci) * kWS + 8 * kb]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      acc[c][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[c], bhi, acc[c][p], 0, 0, 0);
      acc[c][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[c], blo, acc[c][p], 0, 0, 0);
      if constexpr (DT != QR_BF16)
        acc[c][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[c], bhi, acc[c][p], 0, 0, 0);
    }
  }
}

// Stores one column group (columns gbase .. gbase + gw) of a strip's 64
// pixels. Lane (kb, ci) holds, for pixel row p of the strip and column tile
// c, out^T rows 4 kb + r (r = 0..3), i.e. columns 16 r + 4 kb + c of pixel
// ci: four consecutive columns per (r, p). A 128-byte line of a pixel (32
// columns, r = 2m and 2m + 1) is spread over 8 lanes and two values; lanes ci
// and ci ^ 8 swap one value (DPP rotation by 8 within each row of 16 lanes),
// so that each store instruction writes whole lines: 8 pixels x 128 bytes.
// (With 64-byte pieces the memory side read back and rewrote half lines:
// about 1.5x the map's bytes.) Called by every lane of the wave.
__device__ __forceinline__ void store_group(const GView& v, const f32x4 (&acc)[4][4], int tx,
                                            int ty, int strip, int gbase, int gw, int dim, int ci,
                                            int kb) {
  const bool left = ci < 8;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int oy = ty * kTile + strip * kStripRows + p;
    const int xa = tx * kTile + (left ? ci : ci - 8);  // pixel of the first store
    const int xb = xa + 8;                              // of the second
    const int64_t rowpix = static_cast<int64_t>(oy) * v.W;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float a4[4], b4[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float lo4 = acc[c][p][2 * m], hi4 = acc[c][p][2 * m + 1];
        const float send = left ? hi4 : lo4;
        const float recv = __int_as_float(
            __builtin_amdgcn_mov_dpp(__float_as_int(send), 0x128, 0xF, 0xF, false));
        a4[c] = left ? lo4 : recv;
        b4[c] = left ? recv : hi4;
      }
      const int col = 32 * m + (left ? 0 : 16) + 4 * kb;
      if (oy < v.H && col < gw) {
        QR_GLOBAL float* base = v.out + gbase + col;
        if (xa < v.W)
          store_stream(reinterpret_cast<QR_GLOBAL float4*>(base + (rowpix + xa) * dim),
                       make_float4(a4[0], a4[1], a4[2], a4[3]));
        if (xb < v.W)
          store_stream(reinterpret_cast<QR_GLOBAL float4*>(base + (rowpix + xb) * dim),
                       make_float4(b4[0], b4[1], b4[2], b4[3]));
      }
    }
  }
}

// One 64-pixel strip of one tile: Eq. 1 for its pixels, all `dim` columns.
// Called by all 256 threads; every barrier is reached by every wave the same
// number of times (loop bounds and exits are uniform over the workgroup).
// rgid, rmean, rco: threads 0..31 carry the records of the batch being
// requested (with `preloaded`, the caller has already requested the first
// batch's); before_stores is called by every thread once, right before the
// map stores of the last pass (a persistent caller requests its next unit's
// first records there: a load issued after a store waits for it).
struct NoHook {
  __device__ void operator()() const {}
};

template <int DT, class Hook = NoHook>
__device__ void dense_strip(const GView& v, int tile, int strip, int dim, const qr_params& prm,
                            DenseLds& L, int& rgid, f32x2& rmean, f32x4& rco, bool preloaded,
                            const Hook& before_stores = Hook()) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kb = lane >> 4;  // MFMA k-block of the lane: entries 8 kb .. 8 kb + 7
  const int ci = lane & 15;  // MFMA row / column index of the lane
  const int W = v.W, H = v.H;
  const int tiles_x = (W + kTile - 1) / kTile;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  // the lane's pixel in the walk (the same in every wave)
  const int px = tx * kTile + ci;
  const int py = ty * kTile + strip * kStripRows + kb;
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;
  const int lo = static_cast<int>(v.tile_offsets[tile]);
  const int hi = static_cast<int>(v.tile_offsets[tile + 1]);
  const int coff = 16 * (ci & 3) + 4 * (ci >> 2);  // the lane's columns in a group
  int par = 0;  // parity of the batches staged so far (selects the id buffer)
  // The next batch's ids and records are requested by threads 0..31 while
  // the current batch is contracted, and staged into LDS at the top of the
  // next iteration.
  for (int c0 = 0; c0 < dim; c0 += kPassCols) {
    // this wave's column groups in the pass: base column and width (0: none)
    int gbase[kWaveGroups], gw[kWaveGroups];
#pragma unroll
    for (int k = 0; k < kWaveGroups; ++k) {
      gbase[k] = c0 + (wave + 4 * k) * kGrpCols;
      gw[k] = max(0, min(kGrpCols, dim - gbase[k]));
    }
    float T = 1.f;
    bool done = !inside;
    int ncon = 0;
    f32x4 acc[kWaveGroups][4][4];
#pragma unroll
    for (int k = 0; k < kWaveGroups; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[k][c][p] = f32x4{0.f, 0.f, 0.f, 0.f};

    // the pixel states are identical in every wave: uniform exits
    const bool first = lo < hi && __ballot(!done) != 0ull;  // uniform
    if (first && tid < kDB && lo + tid < hi && !(preloaded && c0 == 0)) {
      rgid = static_cast<int>(v.sorted_gid[lo + tid]);
      rmean = v.means2d[rgid];
      rco = v.conic_opacity[rgid];
    }
    for (int batch = lo; batch < hi; batch += kDB) {
      if (__ballot(!done) == 0ull) break;
      const int cnt = min(kDB, hi - batch);
      const int nb = batch + kDB;
      // records of the batch (the previous batch's were last read before the
      // second barrier of its iteration, which every wave has passed; its ids
      // are in the other buffer)
      uint32_t* const gid = L.gid[par];
      par ^= 1;
      // every id slot holds a valid row: slots past the list repeat the
      // batch's first id (their weights are zero)
      const int g0 = __shfl(rgid, 0);
      if (tid < kDB) gid[tid] = static_cast<uint32_t>(tid < cnt ? rgid : g0);
      if (tid < cnt) {
        L.mean[tid] = make_float2(rmean.x, rmean.y);
        L.co[tid] = make_float4(rco.x, rco.y, rco.z, rco.w);
      }
      __syncthreads();

      // feature rows of the batch for this wave's first group, requested now
      // so that the loads overlap the walk (the second group's are requested
      // before the first group's MFMAs). No branches: ids past the list are
      // valid rows (weight 0), columns past the width of a partial group are
      // clamped to its first, and a group past the width (no MFMAs, nothing
      // stored) reads column 0 (their results are never stored).
      f32x4 raw[8];
      const auto load_group = [&](int k) {
        const int col = gw[k] > 0 ? gbase[k] + (coff < gw[k] ? coff : 0) : 0;
        const u32x4 ga = *reinterpret_cast<const u32x4*>(&gid[8 * kb]);
        const u32x4 gb = *reinterpret_cast<const u32x4*>(&gid[8 * kb + 4]);
        const uint32_t g8[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
#pragma unroll
        for (int t = 0; t < 8; ++t) raw[t] = load_raw4<DT>(v, g8[t], dim, col);
      };
      load_group(0);

      // walk (the split walk of dense_walk.h): alpha' of this wave's eight
      // entries and the product of their (1 - alpha')
      float al[kDQ];
      L.part[wave][lane] = walk_alpha8(L.mean, L.co, kDQ * wave, cnt, done, pxc, pyc, prm, al);
      __syncthreads();

      // T at the start of the eight entries, their weights in list order
      // with the stop test
      float Tl = T;
      for (int q = 0; q < wave; ++q) Tl *= L.part[q][lane];
      float w8[kDQ];
      const uint32_t inf = walk_weights8(Tl, al, prm.T_eps, w8);
      bool any = false;
      bf16x8 whi, wlo;
#pragma unroll
      for (int j = 0; j < kDQ; ++j) {
        any |= w8[j] != 0.f;
        __bf16 h, l;
        split_bf16(w8[j], h, l);
        whi[j] = h;
        wlo[j] = l;
      }
      *reinterpret_cast<bf16x8*>(&L.whi[lane * kWS + kDQ * wave]) = whi;
      *reinterpret_cast<bf16x8*>(&L.wlo[lane * kWS + kDQ * wave]) = wlo;
      L.tend[wave][lane] = Tl;
      L.info[wave][lane] = inf;
      const unsigned long long b = __ballot(any);
      if (lane == 0) L.busy[wave] = b;
      __syncthreads();

      // the pixel's state after the batch (the same in every wave)
      walk_fold(&L.tend[0][0], &L.info[0][0], kStripPix, lane, batch - lo, T, done, ncon);
      const unsigned long long busy = L.busy[0] | L.busy[1] | L.busy[2] | L.busy[3];
      // the next batch's ids (its records are requested after the first
      // group's MFMAs, once the ids have arrived)
      const bool more = nb < hi && __ballot(!done) != 0ull;  // uniform: another batch follows
      const bool prefetch = more && tid < kDB && nb + tid < hi;
      if (prefetch) rgid = static_cast<int>(v.sorted_gid[nb + tid]);

      // F^T W^T on the matrix cores, one column group at a time: A = this
      // wave's features (rows permuted within the group), B = the weights of
      // 16 pixels
#pragma unroll
      for (int k = 0; k < kWaveGroups; ++k) {
        if (k == 1 && prefetch) {
          // the next batch's records (their ids, requested before the first
          // group's MFMAs, have arrived)
          rmean = v.means2d[rgid];
          rco = v.conic_opacity[rgid];
        }
        if (gw[k] == 0) continue;
        bf16x8 ahi[4], alo[4];
        convert_group<DT>(raw, ahi, alo);
        mfma_group<DT>(acc[k], ahi, alo, L.whi, L.wlo, busy, ci, kb);
        if (k + 1 < kWaveGroups) load_group(k + 1);
      }
    }

    if (c0 + kPassCols >= dim) before_stores();
#pragma unroll
    for (int k = 0; k < kWaveGroups; ++k)
      if (gw[k] > 0) store_group(v, acc[k], tx, ty, strip, gbase[k], gw[k], dim, ci, kb);
    if (c0 == 0 && wave == 0 && inside) {
      const int pix = py * W + px;
      if (v.T_q) v.T_q[pix] = T;
      if (v.n_sel) v.n_sel[pix] = ncon;
    }
  }
}

// Narrow features (dim <= 64: one column group). The strip decomposition
// above splits each batch's walk over four waves and pays three barriers and a
// cross-wave fold per batch for it; with one column group there is little
// MFMA work to hide that behind. Here one workgroup takes a whole tile: wave w
// owns strip w (tile rows 4w .. 4w + 3), each lane walks its pixel's chain
// over all 32 entries of a batch in list order (the transmittance recursion
// of Eq. 1 exactly as written, no reassociation), writes its weights to the
// wave's own LDS rows and the wave contracts them with the batch's feature
// rows. Records are double-buffered, so one barrier per batch both publishes
// the staged records and tests whether any pixel of the tile is still live.
struct DenseNarrowLds {
  __attribute__((aligned(16))) __bf16 whi[4][kStripPix * kWS];
  __attribute__((aligned(16))) __bf16 wlo[4][kStripPix * kWS];
  float2 mean[2][kDB];
  float4 co[2][kDB];
  __attribute__((aligned(16))) uint32_t gid[2][kDB];
};

// One column of row g (dim == 16 layout): float32 value, or the bfloat16 code
// in the low half.
template <int DT>
__device__ __forceinline__ float load_raw1(const GView& v, uint32_t g, int d) {
  const uint64_t off = static_cast<uint64_t>(g) * 16u + static_cast<uint32_t>(d);
  if constexpr (DT == QR_F32) {
    return static_cast<const QR_GLOBAL float*>(v.feats)[off];
  } else if constexpr (DT == QR_BF16) {
    return __uint_as_float(static_cast<const QR_GLOBAL uint16_t*>(v.feats)[off]);
  } else {
    const uint32_t r = static_cast<const QR_GLOBAL uint8_t*>(v.feats)[off];
    return __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(r), false)[0] * v.scale[g];
  }
}

// kOne: dim == 16, one MFMA column tile in natural order (row i = column i);
// a lane loads its column of eight entries and stores four consecutive
// columns of one pixel, and a store instruction covers 16 whole pixels (1 KB
// contiguous). Otherwise (16 < dim <= 64) one permuted column group as in the
// strip kernel.
template <int DT, bool kOne>
__device__ void dense_tile_narrow(const GView& v, int tile, int dim, const qr_params& prm,
                                  DenseNarrowLds& L) {
  constexpr int NC = kOne ? 1 : 4;  // MFMA column tiles
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kb = lane >> 4;
  const int ci = lane & 15;
  const int W = v.W, H = v.H;
  const int tiles_x = (W + kTile - 1) / kTile;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  // the lane's pixel: row kb, column ci of the wave's strip (so that its
  // weights are row `lane` of the wave's B operand)
  const int px = tx * kTile + ci;
  const int py = ty * kTile + wave * kStripRows + kb;
  const bool inside = px < W && py < H;
  const float pxc = px + 0.5f, pyc = py + 0.5f;
  const int lo = static_cast<int>(v.tile_offsets[tile]);
  const int hi = static_cast<int>(v.tile_offsets[tile + 1]);
  // permuted layout: the lane's four columns (clamped to the group's first
  // past the width: loaded, never stored)
  const int coff = 16 * (ci & 3) + 4 * (ci >> 2);
  const int col = coff < dim ? coff : 0;
  __bf16* const whi = L.whi[wave];
  __bf16* const wlo = L.wlo[wave];

  float T = 1.f;
  bool done = !inside;
  int ncon = 0;
  f32x4 acc[NC][4];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[c][p] = f32x4{0.f, 0.f, 0.f, 0.f};

  // records of the next batch, requested by threads 0..31 one batch ahead
  int rgid = -1;
  f32x2 rmean = f32x2{0.f, 0.f};
  f32x4 rco = f32x4{0.f, 0.f, 0.f, 0.f};
  if (tid < kDB && lo + tid < hi) {
    rgid = static_cast<int>(v.sorted_gid[lo + tid]);
    rmean = v.means2d[rgid];
    rco = v.conic_opacity[rgid];
  }
  int par = 0;
  for (int batch = lo; batch < hi; batch += kDB, par ^= 1) {
    const int cnt = min(kDB, hi - batch);
    const int nb = batch + kDB;
    // stage the batch into buffer `par` (its previous contents, two batches
    // back, were last read before the previous iteration's barrier); id
    // slots past the list repeat the batch's first id (weight 0)
    const int g0 = __shfl(rgid, 0);
    if (tid < kDB) {
      L.gid[par][tid] = static_cast<uint32_t>(tid < cnt ? rgid : g0);
      L.mean[par][tid] = make_float2(rmean.x, rmean.y);
      L.co[par][tid] = make_float4(rco.x, rco.y, rco.z, rco.w);
    }
    // publishes the records; uniform exit once every pixel has stopped
    if (__syncthreads_count(!done) == 0) break;
    const bool prefetch = tid < kDB && nb + tid < hi;
    if (prefetch) rgid = static_cast<int>(v.sorted_gid[nb + tid]);
    if (__ballot(!done) == 0ull) {  // uniform per wave: its strip has finished
      if (prefetch) {
        rmean = v.means2d[rgid];
        rco = v.conic_opacity[rgid];
      }
      continue;
    }

    // the batch's feature rows (ids past the list are valid rows), requested
    // before the walk so that the loads overlap it
    const u32x4 ga = *reinterpret_cast<const u32x4*>(&L.gid[par][8 * kb]);
    const u32x4 gb = *reinterpret_cast<const u32x4*>(&L.gid[par][8 * kb + 4]);
    const uint32_t g8[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
    f32x4 raw[kOne ? 1 : 8];
    float raw1[kOne ? 8 : 1];
    if constexpr (kOne) {
#pragma unroll
      for (int t = 0; t < 8; ++t) raw1[t] = load_raw1<DT>(v, g8[t], ci);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) raw[t] = load_raw4<DT>(v, g8[t], dim, col);
    }

    // Eq. 1 along the lane's ray, in list order
    bool any = false;
#pragma unroll 1
    for (int q = 0; q < kDB / 8; ++q) {
      bf16x8 bh, bl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = 8 * q + j;
        float w = 0.f;
        if (e < cnt && !done) {
          const float a = gauss_alpha(L.mean[par][e], L.co[par][e], pxc, pyc, prm.alpha_max);
          if (a >= prm.alpha_min) {
            const float T_test = T * (1.f - a);
            if (T_test < prm.T_eps) {
              done = true;
            } else {
              w = a * T;
              T = T_test;
              ncon = batch - lo + e + 1;
            }
          }
        }
        any |= w != 0.f;
        __bf16 h, l;
        split_bf16(w, h, l);
        bh[j] = h;
        bl[j] = l;
      }
      *reinterpret_cast<bf16x8*>(&whi[lane * kWS + 8 * q]) = bh;
      *reinterpret_cast<bf16x8*>(&wlo[lane * kWS + 8 * q]) = bl;
    }
    if (prefetch) {
      rmean = v.means2d[rgid];
      rco = v.conic_opacity[rgid];
    }
    const unsigned long long busy = __ballot(any);
    wave_lds_sync();  // the wave's weights, written by all its lanes
    if (busy == 0ull) continue;
    if constexpr (kOne) {
      bf16x8 ahi, alo;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if constexpr (DT != QR_BF16) {
          __bf16 h, l;
          split_bf16(raw1[t], h, l);
          ahi[t] = h;
          alo[t] = l;
        } else {
          ahi[t] = __builtin_bit_cast(__bf16, static_cast<uint16_t>(__float_as_uint(raw1[t])));
        }
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (((busy >> (16 * p)) & 0xFFFFull) == 0ull) continue;
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(&whi[(16 * p + ci) * kWS + 8 * kb]);
        const bf16x8 blo = *reinterpret_cast<const bf16x8*>(&wlo[(16 * p + ci) * kWS + 8 * kb]);
        acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[0][p], 0, 0, 0);
        acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[0][p], 0, 0, 0);
        if constexpr (DT != QR_BF16)
          acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[0][p], 0, 0, 0);
      }
    } else {
      bf16x8 ahi[4], alo[4];
      convert_group<DT>(raw, ahi, alo);
      mfma_group<DT>(acc, ahi, alo, whi, wlo, busy, ci, kb);
    }
  }

  if constexpr (kOne) {
    // lane (kb, ci) holds columns 4 kb .. 4 kb + 3 of pixel ci of row p
    const int ox = tx * kTile + ci;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int oy = ty * kTile + wave * kStripRows + p;
      if (ox < W && oy < H)
        store_stream(reinterpret_cast<QR_GLOBAL float4*>(
                         v.out + (static_cast<int64_t>(oy) * W + ox) * 16 + 4 * kb),
                     make_float4(acc[0][p][0], acc[0][p][1], acc[0][p][2], acc[0][p][3]));
    }
  } else {
    store_group(v, acc, tx, ty, wave, 0, dim, dim, ci, kb);
  }
  if (inside) {
    const int pix = py * W + px;
    if (v.T_q) v.T_q[pix] = T;
    if (v.n_sel) v.n_sel[pix] = ncon;
  }
}

// One view: one workgroup per (tile, strip); the four strips of a tile are
// consecutive units and every XCD receives a contiguous run of units.
template <int DT>
__global__ void __launch_bounds__(kTilePix, 2)
render_dense_kernel(ViewArgs v, int n_units, int dim, qr_params prm) {
  __shared__ DenseLds L;
  const int u = xcd_remap(blockIdx.x, n_units);
  int rgid = -1;
  f32x2 rmean = f32x2{0.f, 0.f};
  f32x4 rco = f32x4{0.f, 0.f, 0.f, 0.f};
  dense_strip<DT>(to_global(v), u / kStrips, u % kStrips, dim, prm, L, rgid, rmean, rco, false);
}

// Many views, one workgroup per (item, strip) unit of the schedule.
template <int DT>
__global__ void __launch_bounds__(kTilePix, 2)
render_dense_batched_grid_kernel(const qr_view* __restrict__ views,
                                 const uint32_t* __restrict__ schedule, int n_units, int dim,
                                 qr_params prm) {
  __shared__ DenseLds L;
  const int u = xcd_remap(blockIdx.x, n_units);
  const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[u / kStrips]);
  const GView v = to_global(view_args(views[packed >> kViewShift]));
  int rgid = -1;
  f32x2 rmean = f32x2{0.f, 0.f};
  f32x4 rco = f32x4{0.f, 0.f, 0.f, 0.f};
  dense_strip<DT>(v, static_cast<int>(packed & kTileMask), u % kStrips, dim, prm, L, rgid, rmean, rco,
                  false);
}

// Many views, persistent workgroups over (item, strip) units through one
// work counter per XCD (the same queue discipline as the batched Q-Render
// launch: a workgroup takes units of its XCD's contiguous range of the
// schedule, then of the others').
constexpr int kDenseQueues = 8;

__device__ __forceinline__ uint32_t dense_queue_begin(int64_t n_units, int q) {
  return static_cast<uint32_t>(n_units * q / kDenseQueues);
}

template <int DT>
__global__ void __launch_bounds__(kTilePix, 2)
render_dense_batched_kernel(const qr_view* __restrict__ views, const uint32_t* __restrict__ schedule,
                            int64_t n_units, uint32_t* __restrict__ counter, int dim, qr_params prm) {
  __shared__ DenseLds L;
  __shared__ uint32_t s_unit[2];
  const int home = static_cast<int>(blockIdx.x % kDenseQueues);
  const auto claim = [&]() {
    uint32_t unit = 0xFFFFFFFFu;
    for (int d = 0; d < kDenseQueues; ++d) {
      const int q = (home + d) % kDenseQueues;
      const uint32_t b = dense_queue_begin(n_units, q), e = dense_queue_begin(n_units, q + 1);
      if (b == e) continue;
      const uint32_t i = atomicAdd(&counter[q], 1u);
      if (i < e - b) {
        unit = b + i;
        break;
      }
    }
    return unit;
  };
  if (threadIdx.x == 0) s_unit[0] = claim();
  // the first records of the next unit, requested by wave 0 before the
  // current unit's map stores (a load issued after a store waits for it)
  int rgid = -1;
  f32x2 rmean = f32x2{0.f, 0.f};
  f32x4 rco = f32x4{0.f, 0.f, 0.f, 0.f};
  bool preloaded = false;
  for (int it = 0;; it ^= 1) {
    __syncthreads();
    const uint32_t unit = __builtin_amdgcn_readfirstlane(s_unit[it]);
    if (unit >= n_units) break;
    const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[unit / kStrips]);
    const GView v = to_global(view_args(views[packed >> kViewShift]));
    const int slot = it ^ 1;
    const auto before_stores = [&]() {
      uint32_t next = 0xFFFFFFFFu;
      if (threadIdx.x == 0) {
        next = claim();
        s_unit[slot] = next;
      }
      preloaded = false;
      if (threadIdx.x < 64) {
        const uint32_t nu = __builtin_amdgcn_readfirstlane(next);
        if (nu < n_units) {
          const uint32_t np = __builtin_amdgcn_readfirstlane(schedule[nu / kStrips]);
          const GView nv = to_global(view_args(views[np >> kViewShift]));
          const int nt = static_cast<int>(np & kTileMask);
          const int lo = static_cast<int>(nv.tile_offsets[nt]);
          const int hi = static_cast<int>(nv.tile_offsets[nt + 1]);
          if (threadIdx.x < kDB && lo + static_cast<int>(threadIdx.x) < hi) {
            rgid = static_cast<int>(nv.sorted_gid[lo + threadIdx.x]);
            rmean = nv.means2d[rgid];
            rco = nv.conic_opacity[rgid];
          }
          preloaded = true;
        }
      }
    };
    dense_strip<DT>(v, static_cast<int>(packed & kTileMask), static_cast<int>(unit % kStrips), dim,
                    prm, L, rgid, rmean, rco, preloaded, before_stores);
  }
}

// The narrow-feature kernels: one workgroup per tile (single view), per
// schedule item (batched grid), or persistent over items.
template <int DT, bool kOne>
__global__ void __launch_bounds__(kTilePix, kOne ? 3 : 2)
render_dense_narrow_kernel(ViewArgs v, int n_tiles, int dim, qr_params prm) {
  __shared__ DenseNarrowLds L;
  dense_tile_narrow<DT, kOne>(to_global(v), xcd_remap(blockIdx.x, n_tiles), dim, prm, L);
}

template <int DT, bool kOne>
__global__ void __launch_bounds__(kTilePix, kOne ? 3 : 2)
render_dense_narrow_batched_grid_kernel(const qr_view* __restrict__ views,
                                        const uint32_t* __restrict__ schedule, int n_items,
                                        int dim, qr_params prm) {
  __shared__ DenseNarrowLds L;
  const int u = xcd_remap(blockIdx.x, n_items);
  const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[u]);
  const GView v = to_global(view_args(views[packed >> kViewShift]));
  dense_tile_narrow<DT, kOne>(v, static_cast<int>(packed & kTileMask), dim, prm, L);
}

template <int DT, bool kOne>
__global__ void __launch_bounds__(kTilePix, kOne ? 3 : 2)
render_dense_narrow_batched_kernel(const qr_view* __restrict__ views,
                                   const uint32_t* __restrict__ schedule, int64_t n_items,
                                   uint32_t* __restrict__ counter, int dim, qr_params prm) {
  __shared__ DenseNarrowLds L;
  __shared__ uint32_t s_unit[2];
  const int home = static_cast<int>(blockIdx.x % kDenseQueues);
  for (int it = 0;; it ^= 1) {
    if (threadIdx.x == 0) {
      uint32_t unit = 0xFFFFFFFFu;
      for (int d = 0; d < kDenseQueues; ++d) {
        const int q = (home + d) % kDenseQueues;
        const uint32_t b = dense_queue_begin(n_items, q), e = dense_queue_begin(n_items, q + 1);
        if (b == e) continue;
        const uint32_t i = atomicAdd(&counter[q], 1u);
        if (i < e - b) {
          unit = b + i;
          break;
        }
      }
      s_unit[it] = unit;
    }
    __syncthreads();
    const uint32_t unit = __builtin_amdgcn_readfirstlane(s_unit[it]);
    if (unit >= n_items) break;
    const uint32_t packed = __builtin_amdgcn_readfirstlane(schedule[unit]);
    const GView v = to_global(view_args(views[packed >> kViewShift]));
    dense_tile_narrow<DT, kOne>(v, static_cast<int>(packed & kTileMask), dim, prm, L);
  }
}

__global__ void reset_dense_counter_kernel(uint32_t* __restrict__ c) {
  if (threadIdx.x < kDenseQueues) c[threadIdx.x] = 0u;
}

}  // namespace qr

using namespace qr;

#define QR_DENSE_DISPATCH(dt)                         \
  switch (dt) {                                       \
    case QR_F32: QR_LAUNCH(QR_F32); break;            \
    case QR_BF16: QR_LAUNCH(QR_BF16); break;          \
    default: QR_LAUNCH(QR_FP8_E4M3); break;           \
  }

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
  const int64_t n_tiles = ceil_div(width, kTile) * ceil_div(height, kTile);
  if (n_tiles * kStrips >= (1ll << 31)) return fail(QR_ERR_UNSUPPORTED, "qr_render_dense: image too large");
  const int n_units = static_cast<int>(n_tiles * kStrips);
  hipStream_t s = as_stream(stream);
  const ViewArgs v{width, height, tile_offsets, sorted_gid, reinterpret_cast<const float2*>(means2d),
                   reinterpret_cast<const float4*>(conic_opacity), features, feature_scale, out,
                   T_final, n_contrib};
  if (dim <= kGrpCols) {
    const int nt = static_cast<int>(n_tiles);
#define QR_LAUNCH(DT)                                                                           \
  if (dim == 16)                                                                                \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(render_dense_narrow_kernel<DT, true>), dim3(nt),          \
                       dim3(kTilePix), 0, s, v, nt, dim, *prm);                                 \
  else                                                                                          \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(render_dense_narrow_kernel<DT, false>), dim3(nt),         \
                       dim3(kTilePix), 0, s, v, nt, dim, *prm)
    QR_DENSE_DISPATCH(dtype);
#undef QR_LAUNCH
    return check_launch("qr_render_dense");
  }
#define QR_LAUNCH(DT) \
  hipLaunchKernelGGL(render_dense_kernel<DT>, dim3(n_units), dim3(kTilePix), 0, s, v, n_units, dim, *prm)
  QR_DENSE_DISPATCH(dtype);
#undef QR_LAUNCH
  return check_launch("qr_render_dense");
}

extern "C" int qr_render_dense_batched(void* stream, int32_t n_views, const qr_view* views,
                                       const qr_params* prm, int32_t dtype, int32_t dim,
                                       const uint32_t* schedule, int64_t n_items,
                                       int32_t n_workgroups, void* workspace,
                                       size_t workspace_bytes) {
  const char* name = "qr_render_dense_batched";
  if (n_views <= 0 || n_views > (1 << (32 - kViewShift)))
    return fail(QR_ERR_INVALID_ARG, "%s: n_views = %d out of range", name, n_views);
  if (!views || !schedule || !prm) return fail(QR_ERR_INVALID_ARG, "%s: null pointer", name);
  if (n_workgroups < 0) return fail(QR_ERR_INVALID_ARG, "%s: n_workgroups < 0", name);
  if (n_workgroups > 0 && (!workspace || workspace_bytes < kDenseQueues * sizeof(uint32_t)))
    return fail(QR_ERR_CAPACITY, "%s: persistent mode needs a %d-byte workspace", name,
                static_cast<int>(kDenseQueues * sizeof(uint32_t)));
  if (n_items < 0 || n_items * kStrips >= (1ll << 31))
    return fail(QR_ERR_INVALID_ARG, "%s: bad item count", name);
  if (dtype != QR_F32 && dtype != QR_BF16 && dtype != QR_FP8_E4M3)
    return fail(QR_ERR_UNSUPPORTED, "%s: unknown dtype %d", name, dtype);
  if (dim <= 0 || dim % 16 != 0 || dim > QR_MAX_DIM)
    return fail(QR_ERR_UNSUPPORTED, "%s: dim = %d", name, dim);
  if (!(prm->alpha_min > 0.f) || !(prm->alpha_max >= prm->alpha_min) || !(prm->alpha_max < 1.f))
    return fail(QR_ERR_INVALID_ARG, "%s: need 0 < alpha_min <= alpha_max < 1", name);
  if (!(prm->T_eps >= 0.f)) return fail(QR_ERR_INVALID_ARG, "%s: T_eps must be >= 0", name);
  if (prm->out_dtype != QR_F32) return fail(QR_ERR_UNSUPPORTED, "%s: float32 output only", name);
  if (n_items == 0) return QR_OK;
  hipStream_t s = as_stream(stream);
  const bool narrow = dim <= kGrpCols;  // one workgroup per item, else per (item, strip)
  const int64_t n_units = narrow ? n_items : n_items * kStrips;
  if (n_workgroups == 0) {
    const int nu = static_cast<int>(n_units);
#define QR_LAUNCH(DT)                                                                          \
  if (narrow && dim == 16)                                                                     \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(render_dense_narrow_batched_grid_kernel<DT, true>),       \
                       dim3(nu), dim3(kTilePix), 0, s, views, schedule, nu, dim, *prm);         \
  else if (narrow)                                                                             \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(render_dense_narrow_batched_grid_kernel<DT, false>),      \
                       dim3(nu), dim3(kTilePix), 0, s, views, schedule, nu, dim, *prm);         \
  else                                                                                         \
    hipLaunchKernelGGL(render_dense_batched_grid_kernel<DT>, dim3(nu), dim3(kTilePix), 0, s,    \
                       views, schedule, nu, dim, *prm)
    QR_DENSE_DISPATCH(dtype);
#undef QR_LAUNCH
    return check_launch(name);
  }
  auto* counter = static_cast<uint32_t*>(workspace);
  hipLaunchKernelGGL(reset_dense_counter_kernel, dim3(1), dim3(64), 0, s, counter);
#define QR_LAUNCH(DT)                                                                           \
  if (narrow && dim == 16)                                                                      \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(render_dense_narrow_batched_kernel<DT, true>),             \
                       dim3(n_workgroups), dim3(kTilePix), 0, s, views, schedule, n_units,       \
                       counter, dim, *prm);                                                      \
  else if (narrow)                                                                              \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(render_dense_narrow_batched_kernel<DT, false>),            \
                       dim3(n_workgroups), dim3(kTilePix), 0, s, views, schedule, n_units,       \
                       counter, dim, *prm);                                                      \
  else                                                                                          \
    hipLaunchKernelGGL(render_dense_batched_kernel<DT>, dim3(n_workgroups), dim3(kTilePix), 0, s, \
                       views, schedule, n_units, counter, dim, *prm)
  QR_DENSE_DISPATCH(dtype);
#undef QR_LAUNCH
  return check_launch(name);
}
