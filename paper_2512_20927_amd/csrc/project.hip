// EWA projection of 3D Gaussians to 2D conics and tile footprints.
//
// Sec. 3 of the paper: a Gaussian has mean mu, covariance Sigma = R S S^T R^T
// (scale s, quaternion r) and opacity alpha, and is splatted with EWA to a 2D
// Gaussian evaluated at each pixel. One thread per Gaussian; the inputs are
// structure-of-arrays columns read with unit stride, the outputs are written
// as float2 / float4 / int4 records so the renderers fetch one Gaussian with
// one or two vector loads.
#include <algorithm>

#include "common.h"

namespace qr {

// Gaussian i seen from `cam`, written to record o of the outputs.
__device__ __forceinline__ void project_one(int64_t i, int64_t o, const float* __restrict__ means3d,
                                            const float* __restrict__ scales,
                                            const float* __restrict__ quats,
                                            const float* __restrict__ opacity, const qr_camera& cam,
                                            const qr_params& prm, float2* __restrict__ means2d,
                                            float4* __restrict__ conic_opacity,
                                            float* __restrict__ depth, int4* __restrict__ rect,
                                            uint32_t* __restrict__ touched) {
  const float mx = means3d[3 * i + 0], my = means3d[3 * i + 1], mz = means3d[3 * i + 2];
  const float sx = scales[3 * i + 0], sy = scales[3 * i + 1], sz = scales[3 * i + 2];
  float qw = quats[4 * i + 0], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
  const float op = opacity[i];

  // camera space
  const float* R = cam.R_cw;
  const float px = R[0] * mx + R[1] * my + R[2] * mz + cam.t[0];
  const float py = R[3] * mx + R[4] * my + R[5] * mz + cam.t[1];
  const float pz = R[6] * mx + R[7] * my + R[8] * mz + cam.t[2];

  bool ok = pz > cam.z_near && op >= prm.alpha_min;

  const float inv_z = 1.0f / pz;
  const float u = cam.fx * px * inv_z + cam.cx;
  const float v = cam.fy * py * inv_z + cam.cy;

  // rotation from the normalised quaternion
  const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const float r00 = 1.f - 2.f * (qy * qy + qz * qz), r01 = 2.f * (qx * qy - qw * qz), r02 = 2.f * (qx * qz + qw * qy);
  const float r10 = 2.f * (qx * qy + qw * qz), r11 = 1.f - 2.f * (qx * qx + qz * qz), r12 = 2.f * (qy * qz - qw * qx);
  const float r20 = 2.f * (qx * qz - qw * qy), r21 = 2.f * (qy * qz + qw * qx), r22 = 1.f - 2.f * (qx * qx + qy * qy);
  // M = R diag(s); Sigma = M M^T
  const float m00 = r00 * sx, m01 = r01 * sy, m02 = r02 * sz;
  const float m10 = r10 * sx, m11 = r11 * sy, m12 = r12 * sz;
  const float m20 = r20 * sx, m21 = r21 * sy, m22 = r22 * sz;

  // T = J R_cw (2x3), with x/z, y/z clamped to guard x half field of view
  const float lim_x = prm.guard * (0.5f * cam.width) / cam.fx;
  const float lim_y = prm.guard * (0.5f * cam.height) / cam.fy;
  const float txz = fminf(lim_x, fmaxf(-lim_x, px * inv_z));
  const float tyz = fminf(lim_y, fmaxf(-lim_y, py * inv_z));
  const float j00 = cam.fx * inv_z, j02 = -cam.fx * txz * inv_z;
  const float j11 = cam.fy * inv_z, j12 = -cam.fy * tyz * inv_z;
  const float t00 = j00 * R[0] + j02 * R[6], t01 = j00 * R[1] + j02 * R[7], t02 = j00 * R[2] + j02 * R[8];
  const float t10 = j11 * R[3] + j12 * R[6], t11 = j11 * R[4] + j12 * R[7], t12 = j11 * R[5] + j12 * R[8];
  // A = T M (2x3); Sigma_2D = A A^T
  const float a00 = t00 * m00 + t01 * m10 + t02 * m20;
  const float a01 = t00 * m01 + t01 * m11 + t02 * m21;
  const float a02 = t00 * m02 + t01 * m12 + t02 * m22;
  const float a10 = t10 * m00 + t11 * m10 + t12 * m20;
  const float a11 = t10 * m01 + t11 * m11 + t12 * m21;
  const float a12 = t10 * m02 + t11 * m12 + t12 * m22;
  const float cxx = a00 * a00 + a01 * a01 + a02 * a02 + prm.dilation;
  const float cxy = a00 * a10 + a01 * a11 + a02 * a12;
  const float cyy = a10 * a10 + a11 * a11 + a12 * a12 + prm.dilation;
  const float det = cxx * cyy - cxy * cxy;
  ok = ok && det > 0.f;
  const float inv_det = 1.0f / det;

  // footprint: bounding box of the ellipse where alpha' >= alpha_min
  const float r2 = 2.0f * logf(op / prm.alpha_min);
  const float hx = sqrtf(fmaxf(r2 * cxx, 0.f));
  const float hy = sqrtf(fmaxf(r2 * cyy, 0.f));
  int4 rc = make_int4(0, 0, 0, 0);
  uint32_t cnt = 0;
  // NaN/Inf anywhere makes one of these comparisons false
  ok = ok && (u - hx - 0.5f) < static_cast<float>(cam.width) && (u + hx - 0.5f) >= 0.f &&
       (v - hy - 0.5f) < static_cast<float>(cam.height) && (v + hy - 0.5f) >= 0.f;
  if (ok) {
    // clamp in float before converting so that no out-of-range cast occurs
    const int x0 = static_cast<int>(fmaxf(ceilf(u - hx - 0.5f), 0.f));
    const int x1 = static_cast<int>(fminf(floorf(u + hx - 0.5f), static_cast<float>(cam.width - 1)));
    const int y0 = static_cast<int>(fmaxf(ceilf(v - hy - 0.5f), 0.f));
    const int y1 = static_cast<int>(fminf(floorf(v + hy - 0.5f), static_cast<float>(cam.height - 1)));
    if (x1 >= x0 && y1 >= y0) {
      rc = make_int4(x0 / kTile, y0 / kTile, x1 / kTile + 1, y1 / kTile + 1);
      cnt = static_cast<uint32_t>((rc.z - rc.x) * (rc.w - rc.y));
    }
  }
  means2d[o] = make_float2(u, v);
  conic_opacity[o] = make_float4(cyy * inv_det, -cxy * inv_det, cxx * inv_det, op);
  depth[o] = pz;
  rect[o] = rc;
  touched[o] = cnt;
}

// Up to kViewChunk cameras per launch, passed by value; blockIdx.y picks the
// camera, and view v's records occupy [v n, (v + 1) n) of every output. The
// single-camera entry point launches the same kernel with one camera, so one
// view projected alone or in a batch gives bit-identical records.
constexpr int kViewChunk = 32;
struct CameraChunk {
  qr_camera cam[kViewChunk];
};

__global__ void __launch_bounds__(256)
project_views_kernel(int64_t n, const float* __restrict__ means3d, const float* __restrict__ scales,
                     const float* __restrict__ quats, const float* __restrict__ opacity,
                     CameraChunk cams, int64_t first_view, qr_params prm,
                     float2* __restrict__ means2d, float4* __restrict__ conic_opacity,
                     float* __restrict__ depth, int4* __restrict__ rect,
                     uint32_t* __restrict__ touched) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int64_t o = (first_view + blockIdx.y) * n + i;
  project_one(i, o, means3d, scales, quats, opacity, cams.cam[blockIdx.y], prm, means2d,
              conic_opacity, depth, rect, touched);
}

}  // namespace qr

using namespace qr;

static int check_camera(const char* name, const qr_camera* cam) {
  if (cam->width <= 0 || cam->height <= 0)
    return fail(QR_ERR_INVALID_ARG, "%s: image size must be positive", name);
  if (!(cam->fx > 0.f) || !(cam->fy > 0.f))
    return fail(QR_ERR_INVALID_ARG, "%s: focal lengths must be positive", name);
  return QR_OK;
}

static int check_project_args(const char* name, int64_t n, const qr_params* prm,
                              const float* means3d, const float* scales, const float* quats,
                              const float* opacity, const float* means2d,
                              const float* conic_opacity, const float* depth,
                              const int32_t* tile_rect, const uint32_t* tiles_touched) {
  if (!(prm->alpha_min > 0.f) || !(prm->alpha_max >= prm->alpha_min))
    return fail(QR_ERR_INVALID_ARG, "%s: need 0 < alpha_min <= alpha_max", name);
  if (n == 0) return QR_OK;
  if (!means3d || !scales || !quats || !opacity || !means2d || !conic_opacity || !depth ||
      !tile_rect || !tiles_touched)
    return fail(QR_ERR_INVALID_ARG, "%s: null array pointer", name);
  return QR_OK;
}

extern "C" int qr_project(void* stream, int64_t n, const float* means3d, const float* scales,
                          const float* quats, const float* opacity, const qr_camera* cam,
                          const qr_params* prm, float* means2d, float* conic_opacity,
                          float* depth, int32_t* tile_rect, uint32_t* tiles_touched) {
  if (n < 0) return fail(QR_ERR_INVALID_ARG, "qr_project: n < 0");
  if (!cam || !prm) return fail(QR_ERR_INVALID_ARG, "qr_project: null camera or params");
  int rc = check_camera("qr_project", cam);
  if (rc == QR_OK)
    rc = check_project_args("qr_project", n, prm, means3d, scales, quats, opacity, means2d,
                            conic_opacity, depth, tile_rect, tiles_touched);
  if (rc != QR_OK || n == 0) return rc;
  CameraChunk chunk{};
  chunk.cam[0] = *cam;
  hipLaunchKernelGGL(project_views_kernel, dim3(static_cast<unsigned>(ceil_div(n, 256)), 1u), dim3(256),
                     0, as_stream(stream), n, means3d, scales, quats, opacity, chunk, int64_t{0},
                     *prm, reinterpret_cast<float2*>(means2d),
                     reinterpret_cast<float4*>(conic_opacity), depth,
                     reinterpret_cast<int4*>(tile_rect), tiles_touched);
  return check_launch("qr_project");
}

extern "C" int qr_project_views(void* stream, int64_t n, const float* means3d, const float* scales,
                                const float* quats, const float* opacity, int32_t n_views,
                                const qr_camera* cams, const qr_params* prm, float* means2d,
                                float* conic_opacity, float* depth, int32_t* tile_rect,
                                uint32_t* tiles_touched) {
  if (n < 0 || n_views <= 0) return fail(QR_ERR_INVALID_ARG, "qr_project_views: n < 0 or n_views <= 0");
  if (!cams || !prm) return fail(QR_ERR_INVALID_ARG, "qr_project_views: null cameras or params");
  for (int32_t v = 0; v < n_views; ++v) {
    const int rc = check_camera("qr_project_views", &cams[v]);
    if (rc != QR_OK) return rc;
    if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
      return fail(QR_ERR_INVALID_ARG, "qr_project_views: camera %d has another image size", v);
  }
  if (n * static_cast<int64_t>(n_views) >= (1ll << 40))
    return fail(QR_ERR_UNSUPPORTED, "qr_project_views: too many records");
  const int rc = check_project_args("qr_project_views", n, prm, means3d, scales, quats, opacity,
                                    means2d, conic_opacity, depth, tile_rect, tiles_touched);
  if (rc != QR_OK || n == 0) return rc;
  hipStream_t s = as_stream(stream);
  const unsigned blocks = static_cast<unsigned>(ceil_div(n, 256));
  for (int32_t v0 = 0; v0 < n_views; v0 += kViewChunk) {
    const int nv = std::min<int32_t>(kViewChunk, n_views - v0);
    CameraChunk chunk{};
    for (int k = 0; k < nv; ++k) chunk.cam[k] = cams[v0 + k];
    hipLaunchKernelGGL(project_views_kernel, dim3(blocks, static_cast<unsigned>(nv)), dim3(256), 0,
                       s, n, means3d, scales, quats, opacity, chunk, static_cast<int64_t>(v0), *prm,
                       reinterpret_cast<float2*>(means2d), reinterpret_cast<float4*>(conic_opacity),
                       depth, reinterpret_cast<int4*>(tile_rect), tiles_touched);
  }
  return check_launch("qr_project_views");
}
