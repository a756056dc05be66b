// Error state, version and small host entry points of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>

#include "common.h"

namespace qr {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return QR_OK;
}

// Sum of tiles_touched into a 64-bit counter: per-block reduction through
// wave shuffles, one atomic per block.
__global__ void __launch_bounds__(256)
count_pairs_kernel(int64_t n, const uint32_t* __restrict__ touched,
                   unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[4];
  unsigned long long acc = 0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    acc += touched[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(total, part[0] + part[1] + part[2] + part[3]);
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

}  // namespace qr

using namespace qr;

extern "C" const char* qr_version(void) { return "qrender 0.1.0 (gfx950)"; }

extern "C" const char* qr_last_error(void) { return g_last_error.c_str(); }

extern "C" int qr_count_pairs(void* stream, int64_t n, const uint32_t* tiles_touched,
                              void* workspace, size_t workspace_bytes, uint64_t* total) {
  if (n < 0) return fail(QR_ERR_INVALID_ARG, "qr_count_pairs: n < 0");
  if (!total) return fail(QR_ERR_INVALID_ARG, "qr_count_pairs: null result pointer");
  if (n == 0) {
    *total = 0;
    return QR_OK;
  }
  if (!tiles_touched || !workspace)
    return fail(QR_ERR_INVALID_ARG, "qr_count_pairs: null device pointer");
  if (workspace_bytes < sizeof(unsigned long long))
    return fail(QR_ERR_CAPACITY, "qr_count_pairs: workspace needs 8 bytes, got %zu", workspace_bytes);
  auto* d_total = static_cast<unsigned long long*>(workspace);
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, d_total);
  const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 2048);
  hipLaunchKernelGGL(count_pairs_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, n,
                     tiles_touched, d_total);
  int rc = check_launch("qr_count_pairs");
  if (rc != QR_OK) return rc;
  unsigned long long h = 0;
  hipError_t e = hipMemcpyAsync(&h, d_total, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(QR_ERR_HIP, "qr_count_pairs: %s", hipGetErrorString(e));
  *total = h;
  return QR_OK;
}
