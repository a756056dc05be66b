// Launch-shape autotuner of the batched renderers (host code): times every
// (schedule, workgroups per CU) candidate of qr_render_quantile_batched (or,
// with K = 0, of qr_render_dense_batched) with HIP events on the caller's
// stream and reports the fastest.
#include <vector>

#include "common.h"

using namespace qr;

extern "C" int qr_autotune_batched(void* stream, int32_t n_views, const qr_view* views,
                                   const qr_params* prm, int32_t K, int32_t dtype, int32_t dim,
                                   const uint32_t* const* schedules, int32_t n_sched,
                                   int64_t n_items, const int32_t* wg_per_cu, int32_t n_wg,
                                   int32_t reps, void* workspace, size_t workspace_bytes,
                                   float* timings_ms, int32_t* best_schedule,
                                   int32_t* best_wg_per_cu) {
  const char* name = "qr_autotune_batched";
  if (!schedules || !wg_per_cu || !timings_ms || !best_schedule || !best_wg_per_cu)
    return fail(QR_ERR_INVALID_ARG, "%s: null host pointer", name);
  if (n_sched <= 0 || n_wg <= 0 || reps <= 0)
    return fail(QR_ERR_INVALID_ARG, "%s: need n_sched, n_wg, reps >= 1", name);
  for (int i = 0; i < n_sched; ++i)
    if (!schedules[i]) return fail(QR_ERR_INVALID_ARG, "%s: schedule %d is null", name, i);
  for (int j = 0; j < n_wg; ++j)
    if (wg_per_cu[j] < 0 || wg_per_cu[j] > 64)
      return fail(QR_ERR_INVALID_ARG, "%s: wg_per_cu[%d] = %d outside [0, 64]", name, j, wg_per_cu[j]);
  int dev = 0;
  hipDeviceProp_t props;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&props, dev) != hipSuccess)
    return fail(QR_ERR_HIP, "%s: no device properties", name);
  const int n_cu = props.multiProcessorCount;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return fail(QR_ERR_HIP, "%s: cannot create events", name);
  }
  int rc = QR_OK;
  float best = 0.f;
  for (int i = 0; i < n_sched && rc == QR_OK; ++i) {
    for (int j = 0; j < n_wg && rc == QR_OK; ++j) {
      const int nwg = wg_per_cu[j] * n_cu;
      auto launch = [&]() {
        if (K == 0)
          return qr_render_dense_batched(stream, n_views, views, prm, dtype, dim, schedules[i],
                                         n_items, nwg, workspace, workspace_bytes);
        return qr_render_quantile_batched(stream, n_views, views, prm, K, dtype, dim, schedules[i],
                                          n_items, nwg, workspace, workspace_bytes);
      };
      rc = launch();  // warm-up (and argument validation)
      if (rc != QR_OK) break;
      if (hipEventRecord(a, s) != hipSuccess) rc = fail(QR_ERR_HIP, "%s: event record", name);
      for (int r = 0; r < reps && rc == QR_OK; ++r) rc = launch();
      if (rc != QR_OK) break;
      float ms = 0.f;
      if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        rc = fail(QR_ERR_HIP, "%s: event timing failed", name);
        break;
      }
      ms /= static_cast<float>(reps);
      timings_ms[i * n_wg + j] = ms;
      if ((i == 0 && j == 0) || ms < best) {
        best = ms;
        *best_schedule = i;
        *best_wg_per_cu = wg_per_cu[j];
      }
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}
