// Backward passes of the two renderers (in progress).
#include "common.h"
#include "render_common.h"

using namespace qr;

extern "C" int qr_render_dense_backward(void*, int32_t, int32_t, const qr_params*, const uint32_t*,
                                        const uint32_t*, const float*, const float*, const void*,
                                        int32_t, const float*, int32_t, const float*, const float*,
                                        float*, float*, float*) {
  return fail(QR_ERR_UNSUPPORTED, "qr_render_dense_backward: not built yet");
}

extern "C" int qr_render_quantile_backward(void*, int32_t, int32_t, const qr_params*, int32_t,
                                           const uint32_t*, const uint32_t*, const float*,
                                           const float*, const void*, int32_t, const float*,
                                           int32_t, const float*, float*, float*, float*) {
  return fail(QR_ERR_UNSUPPORTED, "qr_render_quantile_backward: not built yet");
}
