// View-dependent RGB of Gaussians from real spherical-harmonic coefficients
// (the colour model of 3D-GS scenes, for the RGB use of Q-Render, Appendix
// "Rendering RGB"): colour = sum_{l <= L} sum_m k_lm Y_lm(d) + 1/2, clipped
// below at 0, d the unit vector from the camera centre to the mean (zero for
// a mean at the centre); Y_lm the real orthonormal harmonics carrying the
// Condon-Shortley phase (-1)^m (the sign convention of 3D-GS coefficients),
// m = -l .. l, coefficient index l^2 + l + m. One thread per Gaussian; the colour goes to
// columns 0..2 of an out_dim-wide feature row (the rest zero) so that the
// renderers take it as a feature table.
#include "common.h"

namespace qr {

__global__ void __launch_bounds__(256)
sh_to_rgb_kernel(int64_t n, int degree, const float* __restrict__ means3d,
                 const float* __restrict__ sh, int coef_stride, float cx, float cy, float cz,
                 float* __restrict__ out, int out_dim) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  float x = means3d[3 * i + 0] - cx, y = means3d[3 * i + 1] - cy, z = means3d[3 * i + 2] - cz;
  const float r = sqrtf(x * x + y * y + z * z);
  const float inv = r > 0.f ? 1.f / r : 0.f;
  x *= inv;
  y *= inv;
  z *= inv;
  constexpr float kPi = 3.14159265358979323846f;
  float Y[16];
  Y[0] = 0.5f / sqrtf(kPi);
  if (degree >= 1) {
    const float k = sqrtf(3.f / (4.f * kPi));
    Y[1] = -k * y;
    Y[2] = k * z;
    Y[3] = -k * x;
  }
  if (degree >= 2) {
    const float a = 0.5f * sqrtf(15.f / kPi), b = 0.25f * sqrtf(5.f / kPi), c = 0.25f * sqrtf(15.f / kPi);
    Y[4] = a * x * y;
    Y[5] = -a * y * z;
    Y[6] = b * (3.f * z * z - 1.f);
    Y[7] = -a * x * z;
    Y[8] = c * (x * x - y * y);
  }
  if (degree >= 3) {
    const float a = 0.25f * sqrtf(35.f / (2.f * kPi)), b = 0.5f * sqrtf(105.f / kPi);
    const float c = 0.25f * sqrtf(21.f / (2.f * kPi)), e = 0.25f * sqrtf(7.f / kPi);
    const float f = 0.25f * sqrtf(105.f / kPi);
    Y[9] = -a * y * (3.f * x * x - y * y);
    Y[10] = b * x * y * z;
    Y[11] = -c * y * (5.f * z * z - 1.f);
    Y[12] = e * (5.f * z * z * z - 3.f * z);
    Y[13] = -c * x * (5.f * z * z - 1.f);
    Y[14] = f * z * (x * x - y * y);
    Y[15] = -a * x * (x * x - 3.f * y * y);
  }
  const int nc = (degree + 1) * (degree + 1);
  const float* k = sh + i * coef_stride * 3;
  float rgb[3] = {0.5f, 0.5f, 0.5f};
  for (int j = 0; j < nc; ++j)
    for (int ch = 0; ch < 3; ++ch) rgb[ch] += Y[j] * k[3 * j + ch];
  float* o = out + i * out_dim;
  for (int ch = 0; ch < 3; ++ch) o[ch] = fmaxf(rgb[ch], 0.f);
  for (int ch = 3; ch < out_dim; ++ch) o[ch] = 0.f;
}

}  // namespace qr

using namespace qr;

extern "C" int qr_sh_to_rgb(void* stream, int64_t n, int32_t degree, const float* means3d,
                            const float* sh, int32_t coef_stride, const qr_camera* cam,
                            float* out, int32_t out_dim) {
  const char* name = "qr_sh_to_rgb";
  if (n < 0) return fail(QR_ERR_INVALID_ARG, "%s: n < 0", name);
  if (degree < 0 || degree > 3) return fail(QR_ERR_UNSUPPORTED, "%s: degree %d outside [0, 3]", name, degree);
  if (coef_stride < (degree + 1) * (degree + 1))
    return fail(QR_ERR_INVALID_ARG, "%s: coef_stride %d < (degree + 1)^2", name, coef_stride);
  if (out_dim < 3) return fail(QR_ERR_INVALID_ARG, "%s: out_dim %d < 3", name, out_dim);
  if (!cam) return fail(QR_ERR_INVALID_ARG, "%s: null camera", name);
  if (n == 0) return QR_OK;
  if (!means3d || !sh || !out) return fail(QR_ERR_INVALID_ARG, "%s: null array pointer", name);
  if (n >= (1ll << 31) * 256) return fail(QR_ERR_UNSUPPORTED, "%s: n too large", name);
  // camera centre c = -R^T t
  const float* R = cam->R_cw;
  const float* t = cam->t;
  const float cx = -(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]);
  const float cy = -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]);
  const float cz = -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]);
  hipLaunchKernelGGL(sh_to_rgb_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     as_stream(stream), n, degree, means3d, sh, coef_stride, cx, cy, cz, out, out_dim);
  return check_launch(name);
}
