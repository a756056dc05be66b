// Tile binning: per-tile, depth-ordered Gaussian lists.
//
// The ray list of Eq. 1 is the depth-ordered sequence of Gaussians covering
// the pixel; as in 3D-GS it is built per 16x16 tile by sorting (tile, depth)
// pairs. Steps, all on the caller's stream without a host round trip:
//   1. exclusive scan of tiles_touched -> pair offsets (and the pair count)
//   2. emit one 64-bit key (tile << 32 | float bits of depth) + Gaussian id
//      per covered tile, in Gaussian-id order
//   3. stable LSD radix sort, 8 bits per pass, over only the key bits that can
//      be non-zero (32 depth bits + ceil(log2(tiles)) tile bits); stability
//      makes equal (tile, depth) keys keep Gaussian-id order
//   4. tile ranges: CSR offsets from the boundaries of the sorted tile ids.
// Depth is positive (z > z_near > 0), so its IEEE bit pattern orders like the
// value. Every kernel reads the pair count from device memory; grids are
// sized by the caller's capacity so no synchronisation is needed.
#include <algorithm>

#include "common.h"

namespace qr {

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 8;
constexpr int kScanItems = kScanThreads * kScanPerThread;  // 2048
constexpr int kSortThreads = 256;
constexpr int kSortPerThread = 16;
constexpr int kSortItems = kSortThreads * kSortPerThread;  // 4096 keys per block
constexpr int kRadix = 256;

// ---- block-wide exclusive scan of one value per thread (256 threads) -----
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds4,
                                                          uint32_t* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) lds4[wave] = inc;
  __syncthreads();
  uint32_t wave_base = 0;
  for (int w = 0; w < wave; ++w) wave_base += lds4[w];
  if (total) *total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return wave_base + inc - v;
}

// scan phase 1: per-block sums
__global__ void __launch_bounds__(kScanThreads)
scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ part) {
  __shared__ uint32_t lds4[4];
  const int64_t base = blockIdx.x * static_cast<int64_t>(kScanItems);
  uint32_t s = 0;
  for (int j = 0; j < kScanPerThread; ++j) {
    const int64_t i = base + j * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t total;
  block_exclusive_scan(s, lds4, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// scan phase 2: one block scans the block sums in chunks; part[nb] = total,
// and out[n] = total when `out_total` is given.
__global__ void __launch_bounds__(kScanThreads)
scan_top_kernel(uint32_t* __restrict__ part, int64_t nb, uint32_t* __restrict__ out_total) {
  __shared__ uint32_t lds4[4];
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += kScanThreads) {
    const int64_t i = c + threadIdx.x;
    const uint32_t v = i < nb ? part[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, lds4, &total);
    if (i < nb) part[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    part[nb] = carry;
    if (out_total) *out_total = carry;
  }
}

// scan phase 3: exclusive scan inside each block plus the block's offset.
// in == out is allowed (each thread reads its items before writing).
__global__ void __launch_bounds__(kScanThreads)
scan_down_kernel(const uint32_t* in, int64_t n, const uint32_t* __restrict__ part,
                 uint32_t* out) {
  __shared__ uint32_t lds4[4];
  const int64_t base = blockIdx.x * static_cast<int64_t>(kScanItems) +
                       threadIdx.x * static_cast<int64_t>(kScanPerThread);
  uint32_t v[kScanPerThread];
  uint32_t s = 0;
  for (int j = 0; j < kScanPerThread; ++j) {
    const int64_t i = base + j;
    v[j] = i < n ? in[i] : 0u;
    s += v[j];
  }
  uint32_t run = part[blockIdx.x] + block_exclusive_scan(s, lds4, nullptr);
  for (int j = 0; j < kScanPerThread; ++j) {
    const int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
}

// Exclusive scan of n u32 values into out[0..n]; out[n] = total.
// `part` needs scan_parts(n) + 1 entries.
static int64_t scan_parts(int64_t n) { return std::max<int64_t>(ceil_div(n, kScanItems), 1); }

static void scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* part,
                           hipStream_t s) {
  const int64_t nb = scan_parts(n);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, s,
                     in, n, part);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, part, nb, out + n);
  hipLaunchKernelGGL(scan_down_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, s,
                     in, n, part, out);
}

// ---- emit ------------------------------------------------------------------
__global__ void __launch_bounds__(256)
emit_kernel(int64_t n, const int4* __restrict__ rect, const uint32_t* __restrict__ touched,
            const float* __restrict__ depth, const uint32_t* __restrict__ pair_off,
            int tiles_x, int64_t capacity, unsigned long long* __restrict__ keys,
            uint32_t* __restrict__ vals) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n || touched[i] == 0) return;
  const int4 r = rect[i];
  const unsigned long long dbits = __float_as_uint(depth[i]);
  int64_t k = pair_off[i];
  for (int ty = r.y; ty < r.w; ++ty) {
    for (int tx = r.x; tx < r.z; ++tx, ++k) {
      if (k >= capacity) return;
      const unsigned long long tile = static_cast<unsigned long long>(ty * tiles_x + tx);
      keys[k] = (tile << 32) | dbits;
      vals[k] = static_cast<uint32_t>(i);
    }
  }
}

__device__ __forceinline__ int64_t pair_count(const uint32_t* total, int64_t capacity) {
  return std::min<int64_t>(static_cast<int64_t>(*total), capacity);
}

// ---- radix sort ------------------------------------------------------------
// Histogram of one 8-bit digit per block of 4096 keys, stored digit-major
// (hist[digit * nblocks + block]) so that one exclusive scan of the whole
// array yields each (digit, block) pair's first output position.
__global__ void __launch_bounds__(kSortThreads)
radix_hist_kernel(const unsigned long long* __restrict__ keys, const uint32_t* __restrict__ total,
                  int64_t capacity, int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t P = pair_count(total, capacity);
  const int64_t base = blockIdx.x * static_cast<int64_t>(kSortItems);
  for (int j = 0; j < kSortPerThread; ++j) {
    const int64_t i = base + j * kSortThreads + threadIdx.x;
    if (i < P) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * static_cast<int64_t>(gridDim.x) + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter. Keys are visited in index order (rounds of 256, thread
// order inside a round); within a wave, the rank among lanes with the same
// digit comes from eight ballots, and across the four waves from per-wave
// digit counts in LDS.
__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const unsigned long long* __restrict__ keys_in,
                     const uint32_t* __restrict__ vals_in, const uint32_t* __restrict__ total,
                     int64_t capacity, int shift, const uint32_t* __restrict__ hist_scanned,
                     unsigned long long* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t run[kRadix];
  __shared__ uint32_t wcnt[4][kRadix];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  run[threadIdx.x] = hist_scanned[threadIdx.x * static_cast<int64_t>(gridDim.x) + blockIdx.x];
  for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t P = pair_count(total, capacity);
  const int64_t base = blockIdx.x * static_cast<int64_t>(kSortItems);
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  for (int j = 0; j < kSortPerThread; ++j) {
    const int64_t i = base + j * kSortThreads + threadIdx.x;
    const bool valid = i < P;
    unsigned long long key = 0;
    uint32_t val = 0;
    uint32_t digit = 0;
    if (valid) {
      key = keys_in[i];
      val = vals_in[i];
      digit = static_cast<uint32_t>(key >> shift) & 0xFFu;
    }
    unsigned long long eq = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (digit >> b) & 1u;
      const unsigned long long m = __ballot(valid && bit);
      eq &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(eq & lt_mask);
    if (valid && rank == 0) wcnt[wave][digit] = __popcll(eq);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[digit] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][digit];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                        wcnt[3][threadIdx.x];
    for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
  }
}

// ---- tile ranges -----------------------------------------------------------
__global__ void __launch_bounds__(256)
tile_ranges_kernel(const unsigned long long* __restrict__ keys, const uint32_t* __restrict__ total,
                   int64_t capacity, int n_tiles, uint32_t* __restrict__ offsets) {
  const int64_t P = pair_count(total, capacity);
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (P == 0) {
    // no pairs: every tile list is empty
    for (int64_t t = i; t <= n_tiles; t += 256LL * gridDim.x) offsets[t] = 0;
    return;
  }
  if (i >= P) return;
  const int t = static_cast<int>(keys[i] >> 32);
  const int prev = i == 0 ? -1 : static_cast<int>(keys[i - 1] >> 32);
  for (int tt = prev + 1; tt <= t; ++tt) offsets[tt] = static_cast<uint32_t>(i);
  if (i == P - 1)
    for (int tt = t + 1; tt <= n_tiles; ++tt) offsets[tt] = static_cast<uint32_t>(P);
}

__global__ void copy_total_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  *dst = *src;
}

__global__ void set_u32_kernel(uint32_t* __restrict__ dst, uint32_t v) { *dst = v; }

// ---- workspace layout --------------------------------------------------------
struct Layout {
  size_t pair_off, scan_part, keys0, keys1, vals0, vals1, hist, hist_part, bytes;
  int64_t nb_sort, hist_len;
};

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

static Layout layout(int64_t n, int64_t capacity) {
  Layout L{};
  size_t o = 0;
  L.pair_off = o;  o = align256(o + sizeof(uint32_t) * (n + 1));
  L.scan_part = o; o = align256(o + sizeof(uint32_t) * (scan_parts(n) + 1));
  L.keys0 = o;     o = align256(o + sizeof(uint64_t) * std::max<int64_t>(capacity, 1));
  L.keys1 = o;     o = align256(o + sizeof(uint64_t) * std::max<int64_t>(capacity, 1));
  L.vals0 = o;     o = align256(o + sizeof(uint32_t) * std::max<int64_t>(capacity, 1));
  L.vals1 = o;     o = align256(o + sizeof(uint32_t) * std::max<int64_t>(capacity, 1));
  L.nb_sort = std::max<int64_t>(ceil_div(capacity, kSortItems), 1);
  L.hist_len = kRadix * L.nb_sort;
  L.hist = o;      o = align256(o + sizeof(uint32_t) * (L.hist_len + 1));
  L.hist_part = o; o = align256(o + sizeof(uint32_t) * (scan_parts(L.hist_len) + 1));
  L.bytes = o;
  return L;
}

static int tile_bits(int64_t n_tiles) {
  int b = 0;
  while ((1ll << b) < n_tiles) ++b;
  return b;
}

}  // namespace qr

using namespace qr;

extern "C" int qr_bin_sort_workspace_size(int64_t n, int32_t tiles_x, int32_t tiles_y,
                                          int64_t capacity, size_t* bytes) {
  if (!bytes) return fail(QR_ERR_INVALID_ARG, "qr_bin_sort_workspace_size: null result pointer");
  if (n < 0 || capacity < 0 || tiles_x <= 0 || tiles_y <= 0)
    return fail(QR_ERR_INVALID_ARG, "qr_bin_sort_workspace_size: bad sizes");
  *bytes = layout(n, capacity).bytes;
  return QR_OK;
}

extern "C" int qr_bin_sort(void* stream, int64_t n, int32_t tiles_x, int32_t tiles_y,
                           const int32_t* tile_rect, const uint32_t* tiles_touched,
                           const float* depth, int64_t capacity, void* workspace,
                           size_t workspace_bytes, uint32_t* sorted_gid, uint64_t* sorted_keys,
                           uint32_t* tile_offsets, uint32_t* total_pairs) {
  if (n < 0 || capacity < 0) return fail(QR_ERR_INVALID_ARG, "qr_bin_sort: negative size");
  if (tiles_x <= 0 || tiles_y <= 0) return fail(QR_ERR_INVALID_ARG, "qr_bin_sort: bad tile grid");
  const int64_t n_tiles = static_cast<int64_t>(tiles_x) * tiles_y;
  if (n_tiles >= (1ll << 31)) return fail(QR_ERR_UNSUPPORTED, "qr_bin_sort: too many tiles");
  if (n >= (1ll << 32) || capacity >= (1ll << 32) - 1)
    return fail(QR_ERR_UNSUPPORTED, "qr_bin_sort: n and capacity must be below 2^32 - 1");
  if (!tile_offsets || !total_pairs || !workspace)
    return fail(QR_ERR_INVALID_ARG, "qr_bin_sort: null output or workspace");
  if (n > 0 && (!tile_rect || !tiles_touched || !depth))
    return fail(QR_ERR_INVALID_ARG, "qr_bin_sort: null input pointer");
  if (capacity > 0 && !sorted_gid) return fail(QR_ERR_INVALID_ARG, "qr_bin_sort: null sorted_gid");
  const Layout L = layout(n, capacity);
  if (workspace_bytes < L.bytes)
    return fail(QR_ERR_CAPACITY, "qr_bin_sort: workspace needs %zu bytes, got %zu", L.bytes,
                workspace_bytes);

  hipStream_t s = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  auto* pair_off = reinterpret_cast<uint32_t*>(ws + L.pair_off);
  auto* scan_part = reinterpret_cast<uint32_t*>(ws + L.scan_part);
  auto* keys0 = reinterpret_cast<unsigned long long*>(ws + L.keys0);
  auto* keys1 = reinterpret_cast<unsigned long long*>(ws + L.keys1);
  auto* vals0 = reinterpret_cast<uint32_t*>(ws + L.vals0);
  auto* vals1 = reinterpret_cast<uint32_t*>(ws + L.vals1);
  auto* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  auto* hist_part = reinterpret_cast<uint32_t*>(ws + L.hist_part);
  const uint32_t* d_total = pair_off + n;

  // 1. pair offsets and total
  if (n > 0) {
    scan_exclusive(tiles_touched, pair_off, n, scan_part, s);
  } else {
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(1), 0, s, pair_off, 0u);
  }
  hipLaunchKernelGGL(copy_total_kernel, dim3(1), dim3(1), 0, s, d_total, total_pairs);

  // 2. emit keys in Gaussian order
  if (n > 0 && capacity > 0)
    hipLaunchKernelGGL(emit_kernel, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, s, n,
                       reinterpret_cast<const int4*>(tile_rect), tiles_touched, depth, pair_off,
                       tiles_x, capacity, keys0, vals0);

  // 3. LSD radix sort over the significant bits
  const int key_bits = 32 + tile_bits(n_tiles);
  const int passes = (key_bits + 7) / 8;
  unsigned long long* ksrc = keys0;
  uint32_t* vsrc = vals0;
  unsigned long long* kfinal = sorted_keys ? reinterpret_cast<unsigned long long*>(sorted_keys) : nullptr;
  for (int p = 0; p < passes && capacity > 0; ++p) {
    const bool last = p == passes - 1;
    unsigned long long* kdst = (ksrc == keys0) ? keys1 : keys0;
    uint32_t* vdst = (vsrc == vals0) ? vals1 : vals0;
    if (last) {
      vdst = sorted_gid;
      if (kfinal) kdst = kfinal;
    }
    const int shift = 8 * p;
    const unsigned nb = static_cast<unsigned>(L.nb_sort);
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kSortThreads), 0, s, ksrc, d_total,
                       capacity, shift, hist);
    scan_exclusive(hist, hist, L.hist_len, hist_part, s);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kSortThreads), 0, s, ksrc, vsrc,
                       d_total, capacity, shift, hist, kdst, vdst);
    ksrc = kdst;
    vsrc = vdst;
  }

  // 4. tile ranges
  const int64_t grid = std::max<int64_t>(ceil_div(std::max<int64_t>(capacity, n_tiles + 1), 256), 1);
  hipLaunchKernelGGL(tile_ranges_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, ksrc,
                     d_total, capacity, static_cast<int>(n_tiles), tile_offsets);
  return check_launch("qr_bin_sort");
}
