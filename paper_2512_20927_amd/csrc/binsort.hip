// Tile binning: per-tile, depth-ordered Gaussian lists.
//
// The ray list of Eq. 1 is the depth-ordered sequence of Gaussians covering
// the pixel; as in 3D-GS it is built per 16x16 tile. Instead of one global
// sort of (tile, depth) keys this is a bucket sort by tile followed by an
// independent sort of each tile's bucket in LDS:
//   1. count: every (Gaussian, covered tile) pair increments its tile's
//      counter (each wave spreads one Gaussian's tiles over its lanes);
//   2. exclusive scan of the counts -> tile_offsets (CSR) and the pair count;
//   3. scatter: each pair claims a slot in its tile's bucket with an atomic
//      cursor and stores the 64-bit key (float bits of depth << 32 | id);
//   4. sort: one workgroup per tile sorts its bucket. The keys are unique
//      (they contain the id), so the result is the exact (depth, id) order
//      whatever order step 3 produced. Buckets of up to 256 keys are
//      bitonic-sorted one key per thread (lane shuffles inside a wave, LDS
//      across waves), up to kLdsItems in LDS; longer ones take a
//      single-workgroup LSD radix sort through a workspace segment.
// Depth is positive (z > z_near > 0), so its IEEE bit pattern orders like
// the value. No kernel synchronises with the host: grids are sized by the
// caller's capacity and every kernel reads the pair count from device memory.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace qr {

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 8;
constexpr int kScanItems = kScanThreads * kScanPerThread;  // 2048
// 16 KB of keys: the kernel's whole LDS (about 21 KB) fits beside a
// renderer's workgroups on a CU, so binning of the next views can overlap
// rendering
constexpr int kLdsItems = 2048;
constexpr int kRadix = 256;

// ---- device-wide exclusive scan (u32) --------------------------------------
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
  block_scan_exclusive(s, lds4, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one block scans the block sums in chunks; part[nb] = out_total[0] = total
// (out_total2 receives a second copy when given)
__global__ void __launch_bounds__(kScanThreads)
scan_top_kernel(uint32_t* __restrict__ part, int64_t nb, uint32_t* __restrict__ out_total,
                uint32_t* __restrict__ out_total2) {
  __shared__ uint32_t lds4[4];
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += kScanThreads) {
    const int64_t i = c + threadIdx.x;
    const uint32_t v = i < nb ? part[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_scan_exclusive(v, lds4, &total);
    if (i < nb) part[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    part[nb] = carry;
    *out_total = carry;
    if (out_total2) *out_total2 = carry;
  }
}

__global__ void __launch_bounds__(kScanThreads)
scan_down_kernel(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ part,
                 uint32_t* __restrict__ out) {
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
  uint32_t run = part[blockIdx.x] + block_scan_exclusive(s, lds4, nullptr);
  for (int j = 0; j < kScanPerThread; ++j) {
    const int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
}

// The whole scan in one workgroup, chunk after chunk with a running carry:
// for short arrays (the per-tile counters of an image) one launch instead of
// three. out[n] = total (and *total2 if given).
__global__ void __launch_bounds__(kScanThreads)
scan_small_kernel(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ out,
                  uint32_t* __restrict__ total2) {
  __shared__ uint32_t lds4[4];
  uint32_t carry = 0;
  for (int64_t c = 0; c < n; c += kScanItems) {
    const int64_t base = c + threadIdx.x * static_cast<int64_t>(kScanPerThread);
    uint32_t v[kScanPerThread];
    uint32_t s = 0;
    for (int j = 0; j < kScanPerThread; ++j) {
      const int64_t i = base + j;
      v[j] = i < n ? in[i] : 0u;
      s += v[j];
    }
    uint32_t total;
    uint32_t run = carry + block_scan_exclusive(s, lds4, &total);
    for (int j = 0; j < kScanPerThread; ++j) {
      const int64_t i = base + j;
      if (i < n) out[i] = run;
      run += v[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    out[n] = carry;
    if (total2) *total2 = carry;
  }
}

constexpr int64_t kSmallScanMax = 16 * kScanItems;  // 32768 entries

static int64_t scan_parts(int64_t n) { return std::max<int64_t>(ceil_div(n, kScanItems), 1); }

// out[0..n) = exclusive scan of in, out[n] = total (and *total2 if given).
// `part` needs scan_parts(n) + 1 entries; in and out must not overlap.
static void scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* part,
                           uint32_t* total2, hipStream_t s) {
  if (n <= kSmallScanMax) {
    hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(kScanThreads), 0, s, in, n, out, total2);
    return;
  }
  const int64_t nb = scan_parts(n);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, s,
                     in, n, part);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, part, nb, out + n, total2);
  hipLaunchKernelGGL(scan_down_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, s,
                     in, n, part, out);
}

// ---- bucket by tile ----------------------------------------------------------
__global__ void __launch_bounds__(256)
zero_u32_kernel(uint32_t* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) a[i] = 0u;
}

// Each wave takes 64 consecutive projected records and visits them one
// after the other; the covered tiles of the current record are spread over
// the 64 lanes, so a Gaussian that covers a thousand tiles costs sixteen
// lane-rounds instead of a thousand serial iterations of one thread, and no
// per-pair index (and no scan of per-record pair counts) is needed.
// Records come in views of n_per_view (record i is Gaussian i % n_per_view
// seen from view i / n_per_view); view v's tile grid is stacked below view
// v-1's (tile rows v*tiles_y ..), and the key carries the view-local id.
template <bool kScatter>
__global__ void __launch_bounds__(256)
tile_pairs_kernel(int64_t n, int64_t n_per_view, const int4* __restrict__ rect,
                  const uint32_t* __restrict__ touched, const float* __restrict__ depth,
                  int tiles_x, int tiles_y, uint32_t* __restrict__ cnt,
                  const uint32_t* __restrict__ offsets, int64_t capacity,
                  unsigned long long* __restrict__ bucket) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (blockIdx.x * 256LL + threadIdx.x) - lane;  // first Gaussian of this wave
  const int64_t mine = base + lane;
  uint32_t my_cnt = 0;
  int4 my_r = make_int4(0, 0, 0, 0);
  uint32_t my_d = 0;
  int my_row0 = 0;       // first stacked tile row of this record's footprint
  uint32_t my_local = 0;  // view-local Gaussian id
  if (mine < n) {
    my_cnt = touched[mine];
    if (my_cnt) {
      my_r = rect[mine];
      if (kScatter) my_d = __float_as_uint(depth[mine]);
      const int64_t view = mine / n_per_view;
      my_local = static_cast<uint32_t>(mine - view * n_per_view);
      my_row0 = static_cast<int>(view) * tiles_y + my_r.y;
    }
  }
  unsigned long long todo = __ballot(my_cnt != 0);
  while (todo) {
    const int j = __ffsll(static_cast<long long>(todo)) - 1;
    todo &= todo - 1;
    const uint32_t c = __shfl(my_cnt, j, 64);
    const int rx = __shfl(my_r.x, j, 64), rz = __shfl(my_r.z, j, 64);
    const int row0 = __shfl(my_row0, j, 64);
    const int w = rz - rx;
    const unsigned long long key = kScatter
        ? ((static_cast<unsigned long long>(__shfl(my_d, j, 64)) << 32) | __shfl(my_local, j, 64))
        : 0ull;
    for (uint32_t k = lane; k < c; k += 64) {
      const int t = (row0 + static_cast<int>(k) / w) * tiles_x + rx + static_cast<int>(k) % w;
      if (kScatter) {
        const int64_t slot = static_cast<int64_t>(offsets[t]) + atomicAdd(&cnt[t], 1u);
        if (slot < capacity) bucket[slot] = key;
      } else {
        atomicAdd(&cnt[t], 1u);
      }
    }
  }
}

// ---- per-tile sort -------------------------------------------------------------
// Stable scatter of one round of 256 keys (thread order) by an 8-bit digit:
// rank among equal digits within the wave from eight ballots, across waves
// from per-wave digit counts. `run` holds each digit's next output position.
__device__ __forceinline__ void stable_scatter_round(bool valid, unsigned long long key, int shift,
                                                     uint32_t* run, uint32_t (*wcnt)[kRadix],
                                                     unsigned long long* __restrict__ dst) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint32_t digit = valid ? static_cast<uint32_t>(key >> shift) & 0xFFu : 0u;
  unsigned long long eq = __ballot(valid);
  for (int b = 0; b < 8; ++b) {
    const bool bit = (digit >> b) & 1u;
    const unsigned long long m = __ballot(valid && bit);
    eq &= bit ? m : ~m;
  }
  const uint32_t rank = __popcll(eq & ((1ull << lane) - 1ull));
  if (valid && rank == 0) wcnt[wave][digit] = __popcll(eq);
  __syncthreads();
  if (valid) {
    uint32_t pos = run[digit] + rank;
    for (int w = 0; w < wave; ++w) pos += wcnt[w][digit];
    dst[pos] = key;
  }
  __syncthreads();
  run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                      wcnt[3][threadIdx.x];
  for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int mask) {
  const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v & 0xFFFFFFFFull), mask, 64));
  const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v >> 32), mask, 64));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__global__ void __launch_bounds__(256)
tile_sort_kernel(int n_tiles, const uint32_t* __restrict__ offsets, int64_t capacity,
                 int gid_bits, unsigned long long* __restrict__ bucket,
                 unsigned long long* __restrict__ radix_tmp, uint32_t* __restrict__ sorted_gid,
                 unsigned long long* __restrict__ sorted_keys) {
  __shared__ unsigned long long s_key[kLdsItems];
  __shared__ uint32_t run[kRadix];
  __shared__ uint32_t wcnt[4][kRadix];
  __shared__ uint32_t lds4[4];
  const int t = blockIdx.x;
  const int64_t lo = std::min<int64_t>(offsets[t], capacity);
  const int64_t hi = std::min<int64_t>(offsets[t + 1], capacity);
  const int n = static_cast<int>(hi - lo);
  if (n <= 0) return;
  const unsigned long long tile_hi = static_cast<unsigned long long>(t) << 32;

  if (n <= 256) {
    // bitonic sort with one key per thread (padded with the largest key):
    // partners in the same wave (distance < 64) are read with lane
    // shuffles, so only the few steps across waves go through LDS and a
    // workgroup barrier
    const int i = threadIdx.x;
    int size = 1;
    while (size < n) size <<= 1;
    unsigned long long key = i < n ? bucket[lo + i] : ~0ull;
    for (int k = 2; k <= size; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        unsigned long long other;
        if (j < 64) {
          other = shfl_xor_u64(key, j);
        } else {
          s_key[i] = key;
          __syncthreads();
          other = s_key[i ^ j];
          __syncthreads();
        }
        const bool ascending = (i & k) == 0;
        const bool lower = (i & j) == 0;  // i is the smaller index of the pair
        key = (lower == ascending) ? (key < other ? key : other) : (key < other ? other : key);
      }
    }
    if (i < n) {
      sorted_gid[lo + i] = static_cast<uint32_t>(key);
      if (sorted_keys) sorted_keys[lo + i] = tile_hi | (key >> 32);
    }
    return;
  }

  if (n <= kLdsItems) {
    // bitonic sort in LDS, padded to a power of two with the largest key
    int size = 1;
    while (size < n) size <<= 1;
    for (int i = threadIdx.x; i < size; i += 256) s_key[i] = i < n ? bucket[lo + i] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= size; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < size; i += 256) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const unsigned long long a = s_key[i], b = s_key[ixj];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
              s_key[i] = b;
              s_key[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < n; i += 256) {
      const unsigned long long key = s_key[i];
      sorted_gid[lo + i] = static_cast<uint32_t>(key);
      if (sorted_keys) sorted_keys[lo + i] = tile_hi | (key >> 32);
    }
    return;
  }

  // long bucket: LSD radix sort, one workgroup, ping-pong between the bucket
  // and the radix_tmp segment. Digits cover the id bits (0 .. gid_bits-1) and
  // the depth bits (32 .. 63); bits gid_bits .. 31 are zero in every key.
  unsigned long long* src = bucket + lo;
  unsigned long long* dst = radix_tmp + lo;
  const int gid_passes = (gid_bits + 7) / 8;
  const int passes = gid_passes + 4;
  for (int p = 0; p < passes; ++p) {
    const int shift = p < gid_passes ? 8 * p : 32 + 8 * (p - gid_passes);
    run[threadIdx.x] = 0;
    for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) atomicAdd(&run[(src[i] >> shift) & 0xFF], 1u);
    __syncthreads();
    const uint32_t c = run[threadIdx.x];
    __syncthreads();
    run[threadIdx.x] = block_scan_exclusive(c, lds4, nullptr);
    __syncthreads();
    for (int base = 0; base < n; base += 256) {
      const int i = base + threadIdx.x;
      const bool valid = i < n;
      stable_scatter_round(valid, valid ? src[i] : 0ull, shift, run, wcnt, dst);
    }
    unsigned long long* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (int i = threadIdx.x; i < n; i += 256) {
    const unsigned long long key = src[i];
    sorted_gid[lo + i] = static_cast<uint32_t>(key);
    if (sorted_keys) sorted_keys[lo + i] = tile_hi | (key >> 32);
  }
}

// ---- workspace layout --------------------------------------------------------
struct Layout {
  size_t cnt, cursor, part, bucket, radix_tmp, bytes;
};

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

static Layout layout(int64_t n_tiles, int64_t capacity) {
  Layout L{};
  size_t o = 0;
  L.cnt = o;     o = align256(o + sizeof(uint32_t) * (n_tiles + 1));
  L.cursor = o;  o = align256(o + sizeof(uint32_t) * (n_tiles + 1));
  L.part = o;    o = align256(o + sizeof(uint32_t) * (scan_parts(n_tiles) + 1));
  L.bucket = o;  o = align256(o + sizeof(uint64_t) * std::max<int64_t>(capacity, 1));
  L.radix_tmp = o; o = align256(o + sizeof(uint64_t) * std::max<int64_t>(capacity, 1));
  L.bytes = o;
  return L;
}

static int bits_for(int64_t n) {
  int b = 0;
  while ((1ll << b) < n) ++b;
  return b;
}

}  // namespace qr

using namespace qr;

extern "C" int qr_bin_sort_workspace_size(int64_t n, int32_t tiles_x, int32_t tiles_y,
                                          int64_t capacity, size_t* bytes) {
  if (!bytes) return fail(QR_ERR_INVALID_ARG, "qr_bin_sort_workspace_size: null result pointer");
  if (n < 0 || capacity < 0 || tiles_x <= 0 || tiles_y <= 0)
    return fail(QR_ERR_INVALID_ARG, "qr_bin_sort_workspace_size: bad sizes");
  *bytes = layout(static_cast<int64_t>(tiles_x) * tiles_y, capacity).bytes;
  return QR_OK;
}

// Bins the records of n_views views (n_per_view each) into the stacked tile
// grid of all views: one launch sequence for the whole batch.
static int bin_sort_impl(const char* name, void* stream, int64_t n_views, int64_t n_per_view,
                         int32_t tiles_x, int32_t tiles_y, const int32_t* tile_rect,
                         const uint32_t* tiles_touched, const float* depth, int64_t capacity,
                         void* workspace, size_t workspace_bytes, uint32_t* sorted_gid,
                         uint64_t* sorted_keys, uint32_t* tile_offsets, uint32_t* total_pairs) {
  if (n_views <= 0 || n_per_view < 0 || capacity < 0) return fail(QR_ERR_INVALID_ARG, "%s: negative size", name);
  if (tiles_x <= 0 || tiles_y <= 0) return fail(QR_ERR_INVALID_ARG, "%s: bad tile grid", name);
  const int64_t n_tiles = static_cast<int64_t>(tiles_x) * tiles_y * n_views;
  if (n_tiles >= (1ll << 31)) return fail(QR_ERR_UNSUPPORTED, "%s: too many tiles", name);
  const int64_t n = n_views * n_per_view;
  if (n_per_view >= (1ll << 32) || n >= (1ll << 40) || capacity >= (1ll << 32) - 1)
    return fail(QR_ERR_UNSUPPORTED, "%s: n and capacity must be below 2^32 - 1", name);
  if (!tile_offsets || !total_pairs || !workspace)
    return fail(QR_ERR_INVALID_ARG, "%s: null output or workspace", name);
  if (n > 0 && (!tile_rect || !tiles_touched || !depth))
    return fail(QR_ERR_INVALID_ARG, "%s: null input pointer", name);
  if (capacity > 0 && !sorted_gid) return fail(QR_ERR_INVALID_ARG, "%s: null sorted_gid", name);
  const Layout L = layout(n_tiles, capacity);
  if (workspace_bytes < L.bytes)
    return fail(QR_ERR_CAPACITY, "%s: workspace needs %zu bytes, got %zu", name, L.bytes,
                workspace_bytes);

  hipStream_t s = as_stream(stream);
  char* ws = static_cast<char*>(workspace);
  auto* cnt = reinterpret_cast<uint32_t*>(ws + L.cnt);
  auto* cursor = reinterpret_cast<uint32_t*>(ws + L.cursor);
  auto* part = reinterpret_cast<uint32_t*>(ws + L.part);
  auto* bucket = reinterpret_cast<unsigned long long*>(ws + L.bucket);
  auto* radix_tmp = reinterpret_cast<unsigned long long*>(ws + L.radix_tmp);

  // counters and cursors are adjacent in the layout: one fill clears both
  const int64_t zero_n = static_cast<int64_t>((L.part - L.cnt) / sizeof(uint32_t));
  hipLaunchKernelGGL(zero_u32_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div(zero_n, 256), 1024))),
                     dim3(256), 0, s, cnt, zero_n);
  const unsigned gblocks = static_cast<unsigned>(std::max<int64_t>(ceil_div(n, 256), 1));
  const int64_t npv = std::max<int64_t>(n_per_view, 1);
  if (n > 0)
    hipLaunchKernelGGL(tile_pairs_kernel<false>, dim3(gblocks), dim3(256), 0, s, n, npv,
                       reinterpret_cast<const int4*>(tile_rect), tiles_touched, depth, tiles_x,
                       tiles_y, cnt, nullptr, capacity, nullptr);
  scan_exclusive(cnt, tile_offsets, n_tiles, part, total_pairs, s);
  if (n > 0 && capacity > 0)
    hipLaunchKernelGGL(tile_pairs_kernel<true>, dim3(gblocks), dim3(256), 0, s, n, npv,
                       reinterpret_cast<const int4*>(tile_rect), tiles_touched, depth, tiles_x,
                       tiles_y, cursor, tile_offsets, capacity, bucket);
  if (capacity > 0)
    hipLaunchKernelGGL(tile_sort_kernel, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s,
                       static_cast<int>(n_tiles), tile_offsets, capacity, bits_for(n_per_view), bucket,
                       radix_tmp, sorted_gid, reinterpret_cast<unsigned long long*>(sorted_keys));
  return check_launch(name);
}

extern "C" int qr_bin_sort(void* stream, int64_t n, int32_t tiles_x, int32_t tiles_y,
                           const int32_t* tile_rect, const uint32_t* tiles_touched,
                           const float* depth, int64_t capacity, void* workspace,
                           size_t workspace_bytes, uint32_t* sorted_gid, uint64_t* sorted_keys,
                           uint32_t* tile_offsets, uint32_t* total_pairs) {
  if (n < 0) return fail(QR_ERR_INVALID_ARG, "qr_bin_sort: negative size");
  if (n >= (1ll << 32)) return fail(QR_ERR_UNSUPPORTED, "qr_bin_sort: n and capacity must be below 2^32 - 1");
  return bin_sort_impl("qr_bin_sort", stream, 1, n, tiles_x, tiles_y, tile_rect, tiles_touched,
                       depth, capacity, workspace, workspace_bytes, sorted_gid, sorted_keys,
                       tile_offsets, total_pairs);
}

// ---- zero-allocation variant ------------------------------------------------
namespace qr {

// The workspace of qr_bin_sort_noalloc: one copy per GPU, allocated when the
// library's code object is loaded on that GPU and held until the process
// ends. In host code `scratch` only names the symbol; its device address is
// looked up once per device (hipGetSymbolAddress) and only that address is
// passed to kernels.
static __device__ __align__(256) unsigned char scratch[QR_BIN_SORT_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_addr[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first
// call for each device).
static int scratch_address(const char* name, void** addr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(QR_ERR_HIP, "%s: hipGetDevice: %s", name, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(QR_ERR_UNSUPPORTED, "%s: device index %d beyond %d", name, dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(QR_ERR_HIP, "%s: hipGetSymbolAddress of the scratch array on device %d: %s",
                  name, dev, hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *addr = g_scratch_addr[dev];
  return QR_OK;
}

}  // namespace qr

extern "C" int qr_bin_sort_noalloc(void* stream, int64_t n, int32_t tiles_x, int32_t tiles_y,
                                   const int32_t* tile_rect, const uint32_t* tiles_touched,
                                   const float* depth, int64_t capacity, uint32_t* sorted_gid,
                                   uint64_t* sorted_keys, uint32_t* tile_offsets,
                                   uint32_t* total_pairs) {
  const char* name = "qr_bin_sort_noalloc";
  if (n < 0 || capacity < 0 || tiles_x <= 0 || tiles_y <= 0)
    return fail(QR_ERR_INVALID_ARG, "%s: bad sizes", name);
  // checked before the layout is computed, so that the sizes below cannot
  // overflow
  if (capacity > static_cast<int64_t>(QR_BIN_SORT_SCRATCH_BYTES) ||
      static_cast<int64_t>(tiles_x) * tiles_y > static_cast<int64_t>(QR_BIN_SORT_SCRATCH_BYTES))
    return fail(QR_ERR_CAPACITY, "%s: capacity %lld pairs over %lld tiles exceeds the %d-byte scratch",
                name, static_cast<long long>(capacity),
                static_cast<long long>(tiles_x) * tiles_y, QR_BIN_SORT_SCRATCH_BYTES);
  const size_t need = layout(static_cast<int64_t>(tiles_x) * tiles_y, capacity).bytes;
  if (need > static_cast<size_t>(QR_BIN_SORT_SCRATCH_BYTES))
    return fail(QR_ERR_CAPACITY,
                "%s: capacity %lld pairs over %lld tiles needs %zu bytes of scratch, the maximum "
                "is %d",
                name, static_cast<long long>(capacity), static_cast<long long>(tiles_x) * tiles_y,
                need, QR_BIN_SORT_SCRATCH_BYTES);
  if (n >= (1ll << 32)) return fail(QR_ERR_UNSUPPORTED, "%s: n must be below 2^32 - 1", name);
  void* ws = nullptr;
  const int rc = scratch_address(name, &ws);
  if (rc != QR_OK) return rc;
  return bin_sort_impl(name, stream, 1, n, tiles_x, tiles_y, tile_rect, tiles_touched, depth,
                       capacity, ws, static_cast<size_t>(QR_BIN_SORT_SCRATCH_BYTES), sorted_gid,
                       sorted_keys, tile_offsets, total_pairs);
}

extern "C" int qr_bin_sort_views(void* stream, int32_t n_views, int64_t n_per_view,
                                 int32_t tiles_x, int32_t tiles_y, const int32_t* tile_rect,
                                 const uint32_t* tiles_touched, const float* depth,
                                 int64_t capacity, void* workspace, size_t workspace_bytes,
                                 uint32_t* sorted_gid, uint64_t* sorted_keys,
                                 uint32_t* tile_offsets, uint32_t* total_pairs) {
  return bin_sort_impl("qr_bin_sort_views", stream, n_views, n_per_view, tiles_x, tiles_y,
                       tile_rect, tiles_touched, depth, capacity, workspace, workspace_bytes,
                       sorted_gid, sorted_keys, tile_offsets, total_pairs);
}
