// Device-side work schedule for the batched renderer: (view, tile) items
// ordered longest tile list first, in power-of-two length classes
// (longest-processing-time-first list scheduling, approximated by buckets so
// that it needs three small kernels and no host round trip).
#include "common.h"

namespace qr {

constexpr int kBuckets = 32;

__device__ __forceinline__ void item_of(int64_t i, int n_views, const int32_t* __restrict__ view_first,
                                        int* view, int* tile) {
  int lo = 0, hi = n_views;  // last v with view_first[v] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (view_first[mid] <= i) lo = mid; else hi = mid;
  }
  *view = lo;
  *tile = static_cast<int>(i - view_first[lo]);
}

__device__ __forceinline__ int heavy_rank(const qr_view* __restrict__ views, int v, int t) {
  const uint32_t len = views[v].tile_offsets[t + 1] - views[v].tile_offsets[t];
  return __clz(len + 1u);  // longer list -> smaller rank (0 .. 31)
}

__global__ void __launch_bounds__(256)
schedule_zero_kernel(uint32_t* __restrict__ a) {
  if (threadIdx.x < 2 * kBuckets) a[threadIdx.x] = 0u;
}

// Per-workgroup histogram in LDS, then one global atomic per non-empty
// bucket: a batch has few length classes, so per-item global atomics would
// all land on a handful of words.
__global__ void __launch_bounds__(256)
schedule_count_kernel(int64_t n_items, int n_views, const int32_t* __restrict__ view_first,
                      const qr_view* __restrict__ views, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[kBuckets];
  if (threadIdx.x < kBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n_items) {
    int v, t;
    item_of(i, n_views, view_first, &v, &t);
    atomicAdd(&h[heavy_rank(views, v, t)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBuckets && h[threadIdx.x] != 0u) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

__global__ void schedule_scan_kernel(uint32_t* __restrict__ cnt) {
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < kBuckets; ++b) {
      const uint32_t c = cnt[b];
      cnt[b] = run;  // exclusive start of bucket b
      run += c;
    }
  }
}

// Items of a workgroup take consecutive slots of their bucket: local ranks
// from LDS atomics, one global reservation per bucket and workgroup. The
// order inside a bucket is unspecified.
__global__ void __launch_bounds__(256)
schedule_scatter_kernel(int64_t n_items, int n_views, const int32_t* __restrict__ view_first,
                        const qr_view* __restrict__ views, const uint32_t* __restrict__ start,
                        uint32_t* __restrict__ cursor, uint32_t* __restrict__ schedule) {
  __shared__ uint32_t h[kBuckets];
  __shared__ uint32_t base[kBuckets];
  if (threadIdx.x < kBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  int v = 0, t = 0, b = 0;
  uint32_t local = 0u;
  if (i < n_items) {
    item_of(i, n_views, view_first, &v, &t);
    b = heavy_rank(views, v, t);
    local = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBuckets && h[threadIdx.x] != 0u)
    base[threadIdx.x] = start[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (i < n_items)
    schedule[base[b] + local] = (static_cast<uint32_t>(v) << QR_BATCH_TILE_BITS) | static_cast<uint32_t>(t);
}

}  // namespace qr

using namespace qr;

extern "C" int qr_batch_schedule(void* stream, int32_t n_views, const qr_view* views,
                                 const int32_t* view_first, int64_t n_items, uint32_t* schedule,
                                 void* workspace, size_t workspace_bytes) {
  if (n_views <= 0 || n_views > (1 << (32 - QR_BATCH_TILE_BITS)))
    return fail(QR_ERR_INVALID_ARG, "qr_batch_schedule: n_views = %d out of range", n_views);
  if (!views || !view_first || !schedule || !workspace)
    return fail(QR_ERR_INVALID_ARG, "qr_batch_schedule: null pointer");
  if (workspace_bytes < 2 * kBuckets * sizeof(uint32_t))
    return fail(QR_ERR_CAPACITY, "qr_batch_schedule: workspace needs %d bytes",
                static_cast<int>(2 * kBuckets * sizeof(uint32_t)));
  if (n_items < 0 || n_items >= (1ll << 32))
    return fail(QR_ERR_INVALID_ARG, "qr_batch_schedule: bad item count");
  if (n_items == 0) return QR_OK;
  hipStream_t s = as_stream(stream);
  auto* cnt = static_cast<uint32_t*>(workspace);
  uint32_t* cursor = cnt + kBuckets;
  const unsigned blocks = static_cast<unsigned>(ceil_div(n_items, 256));
  hipLaunchKernelGGL(schedule_zero_kernel, dim3(1), dim3(256), 0, s, cnt);
  hipLaunchKernelGGL(schedule_count_kernel, dim3(blocks), dim3(256), 0, s, n_items, n_views,
                     view_first, views, cnt);
  hipLaunchKernelGGL(schedule_scan_kernel, dim3(1), dim3(64), 0, s, cnt);
  hipLaunchKernelGGL(schedule_scatter_kernel, dim3(blocks), dim3(256), 0, s, n_items, n_views,
                     view_first, views, cnt, cursor, schedule);
  return check_launch("qr_batch_schedule");
}
