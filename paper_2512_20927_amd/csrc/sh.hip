// View-dependent RGB of Gaussians from real spherical-harmonic coefficients
// (the colour model of 3D-GS scenes, for the RGB use of Q-Render, Appendix
// "Rendering RGB"): colour = sum_{l <= L} sum_m k_lm Y_lm(d) + 1/2, clipped
// below at 0, d the unit vector from the camera centre to the mean (zero for
// a mean at the centre); Y_lm the real orthonormal harmonics carrying the
// Condon-Shortley phase (-1)^m (the sign convention of 3D-GS coefficients),
// m = -l .. l, coefficient index l^2 + l + m. The colour goes to columns
// 0..2 of an out_dim-wide feature row (the rest zero) so that the renderers
// take it as a feature table: one thread per Gaussian for one camera, or
// out_dim / 4 lanes per Gaussian for a batch of cameras.
#include "common.h"
#include "render_common.h"

namespace qr {

// Y[0 .. (degree+1)^2) at the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(int degree, float x, float y, float z, float (&Y)[16]) {
  constexpr float kPi = 3.14159265358979323846f;
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
}

// Colour of one Gaussian (mean m, coefficients k) seen from centre c, into
// o[0 .. out_dim): colour in columns 0..2, zeros after.
// k: a pointer to the coefficients, or a register array of 48 of them.
template <class KT>
__device__ __forceinline__ void sh_colour(int degree, const float (&m)[3], const KT& k, float cx,
                                          float cy, float cz, float* __restrict__ o, int out_dim) {
  float x = m[0] - cx, y = m[1] - cy, z = m[2] - cz;
  const float r = sqrtf(x * x + y * y + z * z);
  const float inv = r > 0.f ? 1.f / r : 0.f;
  float Y[16];
  sh_basis(degree, x * inv, y * inv, z * inv, Y);
  const int nc = (degree + 1) * (degree + 1);
  float rgb[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (j < nc) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) rgb[ch] += Y[j] * k[3 * j + ch];
    }
  }
  for (int ch = 0; ch < 3; ++ch) o[ch] = fmaxf(rgb[ch], 0.f);
  for (int ch = 3; ch < out_dim; ++ch) o[ch] = 0.f;
}

__global__ void __launch_bounds__(256)
sh_to_rgb_kernel(int64_t n, int degree, const float* __restrict__ means3d,
                 const float* __restrict__ sh, int coef_stride, float cx, float cy, float cz,
                 float* __restrict__ out, int out_dim) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const float m[3] = {means3d[3 * i + 0], means3d[3 * i + 1], means3d[3 * i + 2]};
  const float* k = sh + i * coef_stride * 3;
  sh_colour(degree, m, k, cx, cy, cz, out + i * out_dim, out_dim);
}

// Up to kShViews camera centres per launch, passed by value.
constexpr int kShViews = 32;
struct ShCentres {
  float c[kShViews][3];
};

// The colours of every Gaussian for a batch of cameras. out_dim / 4 lanes
// per Gaussian, one float4 column each, so a wave's stores cover contiguous
// rows, and each store instruction writes whole rows: every lane of a
// Gaussian reads its coefficients once and evaluates the colour for every
// camera (the lanes would otherwise wait), the first writes (r, g, b, 0), the
// others zeros. View v's table is out + v * n * out_dim.
__global__ void __launch_bounds__(256)
sh_to_rgb_views_kernel(int64_t n, int degree, const float* __restrict__ means3d,
                       const float* __restrict__ sh, int coef_stride, ShCentres centres,
                       int n_views, float* __restrict__ out, int out_dim) {
  const int parts = out_dim >> 2;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t i = t / parts;
  if (i >= n) return;
  const int part = static_cast<int>(t - i * parts);
  float4* row = reinterpret_cast<float4*>(out) + i * parts + part;  // view 0
  const int64_t view_stride = n * parts;
  const float m[3] = {means3d[3 * i + 0], means3d[3 * i + 1], means3d[3 * i + 2]};
  const int nc = (degree + 1) * (degree + 1);
  float k[48];
#pragma unroll
  for (int j = 0; j < 48; ++j) k[j] = j < 3 * nc ? sh[i * coef_stride * 3 + j] : 0.f;
#pragma unroll
  for (int v = 0; v < kShViews; ++v) {  // constant indices into the argument block
    if (v >= n_views) continue;
    float o[4];
    sh_colour(degree, m, k, centres.c[v][0], centres.c[v][1], centres.c[v][2], o, 4);
    const bool c0 = part == 0;
    store_stream(row + v * view_stride, make_float4(c0 ? o[0] : 0.f, c0 ? o[1] : 0.f, c0 ? o[2] : 0.f, 0.f));
  }
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

extern "C" int qr_sh_to_rgb_views(void* stream, int64_t n, int32_t degree, const float* means3d,
                                  const float* sh, int32_t coef_stride, const qr_camera* cams,
                                  int32_t n_views, float* out, int32_t out_dim) {
  const char* name = "qr_sh_to_rgb_views";
  if (n < 0) return fail(QR_ERR_INVALID_ARG, "%s: n < 0", name);
  if (degree < 0 || degree > 3) return fail(QR_ERR_UNSUPPORTED, "%s: degree %d outside [0, 3]", name, degree);
  if (coef_stride < (degree + 1) * (degree + 1))
    return fail(QR_ERR_INVALID_ARG, "%s: coef_stride %d < (degree + 1)^2", name, coef_stride);
  if (out_dim < 4 || out_dim % 4 != 0)
    return fail(QR_ERR_UNSUPPORTED, "%s: out_dim %d not a positive multiple of 4", name, out_dim);
  if (n_views <= 0) return fail(QR_ERR_INVALID_ARG, "%s: n_views %d <= 0", name, n_views);
  if (!cams) return fail(QR_ERR_INVALID_ARG, "%s: null cameras", name);
  if (n == 0) return QR_OK;
  if (!means3d || !sh || !out) return fail(QR_ERR_INVALID_ARG, "%s: null array pointer", name);
  const int64_t threads = n * (out_dim / 4);
  if (threads >= (1ll << 31) * 256) return fail(QR_ERR_UNSUPPORTED, "%s: n too large", name);
  for (int v0 = 0; v0 < n_views; v0 += kShViews) {
    const int nv = n_views - v0 < kShViews ? n_views - v0 : kShViews;
    ShCentres c;
    for (int v = 0; v < nv; ++v) {  // camera centre -R^T t
      const float* R = cams[v0 + v].R_cw;
      const float* t = cams[v0 + v].t;
      c.c[v][0] = -(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]);
      c.c[v][1] = -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]);
      c.c[v][2] = -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]);
    }
    hipLaunchKernelGGL(sh_to_rgb_views_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0,
                       as_stream(stream), n, degree, means3d, sh, coef_stride, c, nv,
                       out + static_cast<int64_t>(v0) * n * out_dim, out_dim);
    const int rc = check_launch(name);
    if (rc != QR_OK) return rc;
  }
  return QR_OK;
}
