"""ctypes binding of libqrender.so: argument marshalling only.

Each ``qr_*`` function here has the name and argument order of the C entry
point in ``include/qrender.h``; torch tensors are passed as device pointers
and the current torch stream is used unless ``stream`` is given. No compute
happens in Python. If the shared library has not been built the import
fails loudly; there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import torch

# the in-tree build (paper_2512_20927_amd/build.py)
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqrender.so")

QR_OK, QR_ERR_INVALID_ARG, QR_ERR_UNSUPPORTED, QR_ERR_CAPACITY, QR_ERR_HIP = 0, -1, -2, -3, -4
QR_F32, QR_BF16, QR_FP8_E4M3 = 0, 1, 2
QR_SELECT_QUANTILE, QR_SELECT_STRATIFIED, QR_SELECT_TOPK = 0, 1, 2
QR_REDUCE_MAX, QR_REDUCE_MEAN = 0, 1
QR_TILE = 16
QR_MAX_K = 64
QR_BIN_SORT_SCRATCH_BYTES = 64 * 1024 * 1024

EXPORTED = [
    "qr_version", "qr_last_error", "qr_project", "qr_count_pairs",
    "qr_bin_sort_workspace_size", "qr_bin_sort", "qr_render_dense", "qr_render_quantile",
    "qr_render_dense_backward", "qr_render_quantile_backward", "qr_quantize_features",
    "qr_render_quantile_batched", "qr_batch_schedule", "qr_project_views", "qr_bin_sort_views",
    "qr_render_quantile_batched_backward", "qr_autotune_batched", "qr_devoxelize",
    "qr_devoxelize_backward", "qr_sh_to_rgb", "qr_sh_to_rgb_views", "qr_bin_sort_noalloc",
    "qr_render_dense_batched",
]
QR_BATCH_TILE_BITS = 20


class QRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class qr_camera(ctypes.Structure):
    _fields_ = [("R_cw", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_float)]


class qr_view(ctypes.Structure):
    _fields_ = [("tile_offsets", ctypes.c_void_p), ("sorted_gid", ctypes.c_void_p),
                ("means2d", ctypes.c_void_p), ("conic_opacity", ctypes.c_void_p),
                ("features", ctypes.c_void_p), ("feature_scale", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("T_q", ctypes.c_void_p), ("n_sel", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class qr_view_grad(ctypes.Structure):
    _fields_ = [("grad_out", ctypes.c_void_p), ("grad_features", ctypes.c_void_p),
                ("grad_means2d", ctypes.c_void_p), ("grad_conic_opacity", ctypes.c_void_p)]


class qr_params(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_eps", ctypes.c_float), ("dilation", ctypes.c_float),
                ("guard", ctypes.c_float), ("out_dtype", ctypes.c_int32), ("selection", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqrender.so is not built; run `python paper_2512_20927_amd/build.py` "
                          "(expected at %s)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cam_p, prm_p = ctypes.POINTER(qr_camera), ctypes.POINTER(qr_params)
    sig = {
        "qr_version": ([], ctypes.c_char_p),
        "qr_last_error": ([], ctypes.c_char_p),
        "qr_project": ([P, i64, P, P, P, P, cam_p, prm_p, P, P, P, P, P], i32),
        "qr_count_pairs": ([P, i64, P, P, sz, ctypes.POINTER(ctypes.c_uint64)], i32),
        "qr_bin_sort_workspace_size": ([i64, i32, i32, i64, ctypes.POINTER(ctypes.c_size_t)], i32),
        "qr_bin_sort": ([P, i64, i32, i32, P, P, P, i64, P, sz, P, P, P, P], i32),
        "qr_bin_sort_noalloc": ([P, i64, i32, i32, P, P, P, i64, P, P, P, P], i32),
        "qr_project_views": ([P, i64, P, P, P, P, i32, cam_p, prm_p, P, P, P, P, P], i32),
        "qr_bin_sort_views": ([P, i32, i64, i32, i32, P, P, P, i64, P, sz, P, P, P, P], i32),
        "qr_render_dense": ([P, i32, i32, prm_p, P, P, P, P, P, i32, P, i32, P, P, P], i32),
        "qr_render_quantile": ([P, i32, i32, prm_p, i32, P, P, P, P, P, i32, P, i32, P, P, P, P, P, P, P], i32),
        "qr_render_dense_backward": ([P, i32, i32, prm_p, P, P, P, P, P, i32, P, i32, P, P, P, P, P], i32),
        "qr_render_quantile_backward": ([P, i32, i32, prm_p, i32, P, P, P, P, P, i32, P, i32, P, P, P, P], i32),
        "qr_quantize_features": ([P, i64, i32, P, i32, P, P], i32),
        "qr_render_quantile_batched": ([P, i32, P, prm_p, i32, i32, i32, P, i64, i32, P, sz], i32),
        "qr_render_dense_batched": ([P, i32, P, prm_p, i32, i32, P, i64, i32, P, sz], i32),
        "qr_batch_schedule": ([P, i32, P, P, i64, P, P, sz], i32),
        "qr_render_quantile_batched_backward": ([P, i32, P, P, prm_p, i32, i32, i32, P, i64, i32, P, sz], i32),
        "qr_sh_to_rgb": ([P, i64, i32, P, P, i32, cam_p, P, i32], i32),
        "qr_sh_to_rgb_views": ([P, i64, i32, P, P, i32, cam_p, i32, P, i32], i32),
        "qr_devoxelize": ([P, i64, i32, P, P, i64, i64, P, i32, P, P], i32),
        "qr_devoxelize_backward": ([P, i64, i32, P, P, i64, i64, i32, P, P, P], i32),
        "qr_autotune_batched": ([P, i32, P, prm_p, i32, i32, i32, ctypes.POINTER(ctypes.c_void_p), i32, i64,
                                 ctypes.POINTER(i32), i32, i32, P, sz, ctypes.POINTER(ctypes.c_float),
                                 ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_LIB = _load()


def lib():
    return _LIB


def version() -> str:
    return _LIB.qr_version().decode()


def last_error() -> str:
    return _LIB.qr_last_error().decode()


def _check(rc):
    if rc != QR_OK:
        raise QRError(rc, last_error())


_EMPTY = {}


def _ptr(t):
    """Device pointer of a tensor (None -> NULL). Checks contiguity.

    The C ABI takes no NULL for required arrays; an empty tensor (e.g. a
    scene with no Gaussians, whose lists are all empty so nothing is read)
    is passed as a valid 16-byte allocation on its device."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.numel() == 0:
        key = str(t.device)
        if key not in _EMPTY:
            _EMPTY[key] = torch.zeros(4, dtype=torch.float32, device=t.device)
        return ctypes.c_void_p(_EMPTY[key].data_ptr())
    return ctypes.c_void_p(t.data_ptr())


def _need(t, numel, dtypes, name):
    """Host-side shape/dtype/device guard so that no kernel is launched on a
    buffer smaller than the C ABI assumes."""
    if t is None:
        return
    if t.dtype not in dtypes:
        raise TypeError("%s: dtype %s not in %s" % (name, t.dtype, dtypes))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


F32 = (torch.float32,)
I32 = (torch.int32,)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def make_camera(cam) -> qr_camera:
    """qr_camera from any object with R_cw, t, fx, fy, cx, cy, width, height, z_near."""
    c = qr_camera()
    R = [float(x) for x in list(getattr(cam.R_cw, "ravel", lambda: cam.R_cw)())]
    for i in range(9):
        c.R_cw[i] = R[i]
    t = [float(x) for x in list(cam.t)]
    for i in range(3):
        c.t[i] = t[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.z_near = float(getattr(cam, "z_near", 0.2))
    return c


def make_params(alpha_min=1.0 / 255.0, alpha_max=0.99, T_eps=1e-4, dilation=0.3, guard=1.3,
                out_dtype=QR_F32, selection=0) -> qr_params:
    return qr_params(alpha_min, alpha_max, T_eps, dilation, guard, out_dtype, selection)


DTYPE_CODE = {torch.float32: QR_F32, torch.bfloat16: QR_BF16, torch.uint8: QR_FP8_E4M3}
if hasattr(torch, "float8_e4m3fn"):
    DTYPE_CODE[torch.float8_e4m3fn] = QR_FP8_E4M3


# ---- entry points ------------------------------------------------------------

def qr_project(means3d, scales, quats, opacity, camera: qr_camera, params: qr_params,
               means2d, conic_opacity, depth, tile_rect, tiles_touched, stream=None):
    n = means3d.shape[0]
    for t, k, nm in ((means3d, 3, "means3d"), (scales, 3, "scales"), (quats, 4, "quats"),
                     (opacity, 1, "opacity"), (means2d, 2, "means2d"),
                     (conic_opacity, 4, "conic_opacity"), (depth, 1, "depth")):
        _need(t, n * k, F32, nm)
    _need(tile_rect, 4 * n, I32, "tile_rect")
    _need(tiles_touched, n, I32, "tiles_touched")
    _check(_LIB.qr_project(_stream(stream), n, _ptr(means3d), _ptr(scales), _ptr(quats),
                           _ptr(opacity), ctypes.byref(camera), ctypes.byref(params),
                           _ptr(means2d), _ptr(conic_opacity), _ptr(depth), _ptr(tile_rect),
                           _ptr(tiles_touched)))


def qr_project_views(means3d, scales, quats, opacity, cameras, params: qr_params,
                     means2d, conic_opacity, depth, tile_rect, tiles_touched, stream=None):
    """cameras: a ctypes array of qr_camera (see make_cameras); outputs hold
    len(cameras) * N records, view-major."""
    n = means3d.shape[0]
    nv = len(cameras)
    for t, k, nm in ((means3d, 3, "means3d"), (scales, 3, "scales"), (quats, 4, "quats"),
                     (opacity, 1, "opacity")):
        _need(t, n * k, F32, nm)
    for t, k, nm in ((means2d, 2, "means2d"), (conic_opacity, 4, "conic_opacity"), (depth, 1, "depth")):
        _need(t, nv * n * k, F32, nm)
    _need(tile_rect, 4 * nv * n, I32, "tile_rect")
    _need(tiles_touched, nv * n, I32, "tiles_touched")
    _check(_LIB.qr_project_views(_stream(stream), n, _ptr(means3d), _ptr(scales), _ptr(quats),
                                 _ptr(opacity), nv, cameras, ctypes.byref(params), _ptr(means2d),
                                 _ptr(conic_opacity), _ptr(depth), _ptr(tile_rect),
                                 _ptr(tiles_touched)))


def make_cameras(cams):
    """ctypes array of qr_camera from camera-like objects."""
    arr = (qr_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, qr_camera) else make_camera(c)
    return arr


def qr_count_pairs(tiles_touched, workspace, stream=None) -> int:
    out = ctypes.c_uint64(0)
    _need(tiles_touched, tiles_touched.shape[0], I32, "tiles_touched")
    _check(_LIB.qr_count_pairs(_stream(stream), tiles_touched.shape[0], _ptr(tiles_touched),
                               _ptr(workspace), workspace.numel() * workspace.element_size(),
                               ctypes.byref(out)))
    return int(out.value)


def qr_bin_sort_workspace_size(n, tiles_x, tiles_y, capacity) -> int:
    out = ctypes.c_size_t(0)
    _check(_LIB.qr_bin_sort_workspace_size(n, tiles_x, tiles_y, capacity, ctypes.byref(out)))
    return int(out.value)


def qr_bin_sort(n, tiles_x, tiles_y, tile_rect, tiles_touched, depth, capacity, workspace,
                sorted_gid, sorted_keys, tile_offsets, total_pairs, stream=None):
    _need(tile_rect, 4 * n, I32, "tile_rect")
    _need(tiles_touched, n, I32, "tiles_touched")
    _need(depth, n, F32, "depth")
    _need(sorted_gid, capacity, I32, "sorted_gid")
    _need(sorted_keys, capacity, (torch.int64,), "sorted_keys")
    _need(tile_offsets, tiles_x * tiles_y + 1, I32, "tile_offsets")
    _need(total_pairs, 1, I32, "total_pairs")
    _check(_LIB.qr_bin_sort(_stream(stream), n, tiles_x, tiles_y, _ptr(tile_rect),
                            _ptr(tiles_touched), _ptr(depth), capacity, _ptr(workspace),
                            workspace.numel() * workspace.element_size(), _ptr(sorted_gid),
                            _ptr(sorted_keys), _ptr(tile_offsets), _ptr(total_pairs)))


def qr_bin_sort_noalloc(n, tiles_x, tiles_y, tile_rect, tiles_touched, depth, capacity,
                        sorted_gid, sorted_keys, tile_offsets, total_pairs, stream=None):
    """qr_bin_sort with the library's static per-GPU workspace (no workspace
    argument; calls on one GPU must not overlap)."""
    _need(tile_rect, 4 * n, I32, "tile_rect")
    _need(tiles_touched, n, I32, "tiles_touched")
    _need(depth, n, F32, "depth")
    _need(sorted_gid, capacity, I32, "sorted_gid")
    _need(sorted_keys, capacity, (torch.int64,), "sorted_keys")
    _need(tile_offsets, tiles_x * tiles_y + 1, I32, "tile_offsets")
    _need(total_pairs, 1, I32, "total_pairs")
    _check(_LIB.qr_bin_sort_noalloc(_stream(stream), n, tiles_x, tiles_y, _ptr(tile_rect),
                                    _ptr(tiles_touched), _ptr(depth), capacity, _ptr(sorted_gid),
                                    _ptr(sorted_keys), _ptr(tile_offsets), _ptr(total_pairs)))


def qr_bin_sort_views(n_views, n_per_view, tiles_x, tiles_y, tile_rect, tiles_touched, depth,
                      capacity, workspace, sorted_gid, sorted_keys, tile_offsets, total_pairs,
                      stream=None):
    n = n_views * n_per_view
    _need(tile_rect, 4 * n, I32, "tile_rect")
    _need(tiles_touched, n, I32, "tiles_touched")
    _need(depth, n, F32, "depth")
    _need(sorted_gid, capacity, I32, "sorted_gid")
    _need(sorted_keys, capacity, (torch.int64,), "sorted_keys")
    _need(tile_offsets, n_views * tiles_x * tiles_y + 1, I32, "tile_offsets")
    _need(total_pairs, 1, I32, "total_pairs")
    _check(_LIB.qr_bin_sort_views(_stream(stream), n_views, n_per_view, tiles_x, tiles_y,
                                  _ptr(tile_rect), _ptr(tiles_touched), _ptr(depth), capacity,
                                  _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _ptr(sorted_gid), _ptr(sorted_keys), _ptr(tile_offsets),
                                  _ptr(total_pairs)))


def _feat_args(features, feature_scale):
    code = DTYPE_CODE.get(features.dtype)
    if code is None:
        raise ValueError("unsupported feature dtype %s" % features.dtype)
    if features.dim() != 2 or not features.is_cuda or not features.is_contiguous():
        raise ValueError("features must be a contiguous [N, D] device tensor")
    if code == QR_FP8_E4M3:
        _need(feature_scale, features.shape[0], F32, "feature_scale")
    return _ptr(features), code, _ptr(feature_scale), features.shape[1]


def _check_render(width, height, tile_offsets, sorted_gid, means2d, conic_opacity, features, K=1):
    n = features.shape[0]
    tx, ty = (width + QR_TILE - 1) // QR_TILE, (height + QR_TILE - 1) // QR_TILE
    _need(tile_offsets, tx * ty + 1, I32, "tile_offsets")
    _need(sorted_gid, 1, I32, "sorted_gid")
    _need(means2d, 2 * n, F32, "means2d")
    _need(conic_opacity, 4 * n, F32, "conic_opacity")
    return width * height


def qr_render_dense(width, height, params, tile_offsets, sorted_gid, means2d, conic_opacity,
                    features, feature_scale, out, T_final=None, n_contrib=None, stream=None):
    fp, code, sp, dim = _feat_args(features, feature_scale)
    npx = _check_render(width, height, tile_offsets, sorted_gid, means2d, conic_opacity, features)
    _need(out, npx * dim, F32, "out")
    _need(T_final, npx, F32, "T_final")
    _need(n_contrib, npx, I32, "n_contrib")
    _check(_LIB.qr_render_dense(_stream(stream), width, height, ctypes.byref(params),
                                _ptr(tile_offsets), _ptr(sorted_gid), _ptr(means2d),
                                _ptr(conic_opacity), fp, code, sp, dim, _ptr(out), _ptr(T_final),
                                _ptr(n_contrib)))


def qr_render_quantile(width, height, params, K, tile_offsets, sorted_gid, means2d, conic_opacity,
                       features, feature_scale, out, T_q=None, n_sel=None, sel_gid=None,
                       sel_w=None, stream=None, T_final=None, last_pos=None):
    fp, code, sp, dim = _feat_args(features, feature_scale)
    npx = _check_render(width, height, tile_offsets, sorted_gid, means2d, conic_opacity, features)
    _need(out, npx * dim, (torch.bfloat16,) if params.out_dtype == QR_BF16 else F32, "out")
    _need(T_q, npx, F32, "T_q")
    _need(n_sel, npx, I32, "n_sel")
    _need(T_final, npx, F32, "T_final")
    _need(last_pos, npx, I32, "last_pos")
    _need(sel_gid, npx * K, I32, "sel_gid")
    _need(sel_w, npx * K, F32, "sel_w")
    _check(_LIB.qr_render_quantile(_stream(stream), width, height, ctypes.byref(params), K,
                                   _ptr(tile_offsets), _ptr(sorted_gid), _ptr(means2d),
                                   _ptr(conic_opacity), fp, code, sp, dim, _ptr(out), _ptr(T_q),
                                   _ptr(n_sel), _ptr(T_final), _ptr(last_pos), _ptr(sel_gid),
                                   _ptr(sel_w)))


def qr_render_dense_backward(width, height, params, tile_offsets, sorted_gid, means2d,
                             conic_opacity, features, feature_scale, out, grad_out,
                             grad_features, grad_means2d, grad_conic_opacity, stream=None):
    fp, code, sp, dim = _feat_args(features, feature_scale)
    npx = _check_render(width, height, tile_offsets, sorted_gid, means2d, conic_opacity, features)
    n = features.shape[0]
    _need(out, npx * dim, F32, "out")
    _need(grad_out, npx * dim, F32, "grad_out")
    _need(grad_features, n * dim, F32, "grad_features")
    _need(grad_means2d, n * 2, F32, "grad_means2d")
    _need(grad_conic_opacity, n * 4, F32, "grad_conic_opacity")
    _check(_LIB.qr_render_dense_backward(_stream(stream), width, height, ctypes.byref(params),
                                         _ptr(tile_offsets), _ptr(sorted_gid), _ptr(means2d),
                                         _ptr(conic_opacity), fp, code, sp, dim, _ptr(out),
                                         _ptr(grad_out), _ptr(grad_features), _ptr(grad_means2d),
                                         _ptr(grad_conic_opacity)))


def qr_render_quantile_backward(width, height, params, K, tile_offsets, sorted_gid, means2d,
                                conic_opacity, features, feature_scale, grad_out, grad_features,
                                grad_means2d, grad_conic_opacity, stream=None):
    fp, code, sp, dim = _feat_args(features, feature_scale)
    npx = _check_render(width, height, tile_offsets, sorted_gid, means2d, conic_opacity, features)
    n = features.shape[0]
    _need(grad_out, npx * dim, F32, "grad_out")
    _need(grad_features, n * dim, F32, "grad_features")
    _need(grad_means2d, n * 2, F32, "grad_means2d")
    _need(grad_conic_opacity, n * 4, F32, "grad_conic_opacity")
    _check(_LIB.qr_render_quantile_backward(_stream(stream), width, height, ctypes.byref(params),
                                            K, _ptr(tile_offsets), _ptr(sorted_gid),
                                            _ptr(means2d), _ptr(conic_opacity), fp, code, sp, dim,
                                            _ptr(grad_out), _ptr(grad_features),
                                            _ptr(grad_means2d), _ptr(grad_conic_opacity)))


def qr_quantize_features(features, dtype_code, out, scale=None, stream=None):
    n, dim = features.shape
    _need(features, n * dim, F32, "features")
    if out.numel() < n * dim or out.element_size() != (2 if dtype_code == QR_BF16 else 1):
        raise ValueError("out must hold n * dim codes of the requested width")
    if dtype_code == QR_FP8_E4M3:
        _need(scale, n, F32, "scale")
    _check(_LIB.qr_quantize_features(_stream(stream), features.shape[0], features.shape[1],
                                     _ptr(features), dtype_code, _ptr(out), _ptr(scale)))


def qr_render_quantile_batched(n_views, views_dev, params, K, dtype_code, dim, schedule, n_workgroups,
                               workspace, stream=None):
    """views_dev: uint8 device tensor holding n_views qr_view records (see
    pack_views); schedule: int32 device tensor of packed (view, tile) items;
    n_workgroups 0 = one workgroup per item (workspace may be None), > 0 =
    persistent workgroups with the work counter in `workspace`."""
    if views_dev.numel() < n_views * ctypes.sizeof(qr_view):
        raise ValueError("views_dev is smaller than n_views qr_view records")
    _need(schedule, 0, I32, "schedule")
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_LIB.qr_render_quantile_batched(_stream(stream), n_views, _ptr(views_dev),
                                           ctypes.byref(params), K, dtype_code, dim,
                                           _ptr(schedule), schedule.numel(), n_workgroups,
                                           _ptr(workspace) if workspace is not None else None,
                                           ws_bytes))


def qr_render_dense_batched(n_views, views_dev, params, dtype_code, dim, schedule, n_workgroups,
                            workspace, stream=None):
    """The dense blend over the same views table and schedule as
    qr_render_quantile_batched; each view's T_q / n_sel fields receive
    T_final / n_contrib."""
    if views_dev.numel() < n_views * ctypes.sizeof(qr_view):
        raise ValueError("views_dev is smaller than n_views qr_view records")
    _need(schedule, 0, I32, "schedule")
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_LIB.qr_render_dense_batched(_stream(stream), n_views, _ptr(views_dev),
                                        ctypes.byref(params), dtype_code, dim, _ptr(schedule),
                                        schedule.numel(), n_workgroups,
                                        _ptr(workspace) if workspace is not None else None,
                                        ws_bytes))


def qr_render_quantile_batched_backward(n_views, views_dev, grads_dev, params, K, dtype_code, dim,
                                        schedule, n_workgroups, workspace, stream=None):
    """Backward of qr_render_quantile_batched over the same views and
    schedule; grads_dev: uint8 device tensor holding n_views qr_view_grad
    records (see pack_grads)."""
    if views_dev.numel() < n_views * ctypes.sizeof(qr_view):
        raise ValueError("views_dev is smaller than n_views qr_view records")
    if grads_dev.numel() < n_views * ctypes.sizeof(qr_view_grad):
        raise ValueError("grads_dev is smaller than n_views qr_view_grad records")
    _need(schedule, 0, I32, "schedule")
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_LIB.qr_render_quantile_batched_backward(
        _stream(stream), n_views, _ptr(views_dev), _ptr(grads_dev), ctypes.byref(params), K,
        dtype_code, dim, _ptr(schedule), schedule.numel(), n_workgroups,
        _ptr(workspace) if workspace is not None else None, ws_bytes))


def qr_autotune_batched(n_views, views_dev, params, K, dtype_code, dim, schedules, wg_per_cu, reps,
                        workspace, stream=None):
    """Times qr_render_quantile_batched for every (schedule, workgroups per
    CU) pair; schedules: int32 device tensors of n_items packed items each.
    Returns (best schedule index, best workgroups per CU, timings_ms as a
    [len(schedules)][len(wg_per_cu)] list)."""
    if views_dev.numel() < n_views * ctypes.sizeof(qr_view):
        raise ValueError("views_dev is smaller than n_views qr_view records")
    n_items = schedules[0].numel()
    for sch in schedules:
        _need(sch, n_items, I32, "schedule")
        if sch.numel() != n_items:
            raise ValueError("schedules differ in length")
    ns, nw = len(schedules), len(wg_per_cu)
    sch_ptrs = (ctypes.c_void_p * ns)(*[sch.data_ptr() for sch in schedules])
    wg = (ctypes.c_int32 * nw)(*wg_per_cu)
    times = (ctypes.c_float * (ns * nw))()
    bi, bw = ctypes.c_int32(-1), ctypes.c_int32(-1)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_LIB.qr_autotune_batched(_stream(stream), n_views, _ptr(views_dev), ctypes.byref(params), K,
                                    dtype_code, dim, sch_ptrs, ns, n_items, wg, nw, reps,
                                    _ptr(workspace) if workspace is not None else None, ws_bytes,
                                    times, ctypes.byref(bi), ctypes.byref(bw)))
    return bi.value, bw.value, [[times[i * nw + j] for j in range(nw)] for i in range(ns)]


def qr_sh_to_rgb(means3d, sh, degree, camera, out, stream=None):
    """means3d f32 [N,3]; sh f32 [N, S, 3] (S >= (degree+1)^2); out f32 [N, C]
    (C >= 3): RGB in columns 0..2, zeros elsewhere."""
    n = means3d.shape[0]
    if means3d.dim() != 2 or means3d.shape[1] != 3:
        raise ValueError("means3d must be [N, 3]")
    if sh.dim() != 3 or sh.shape[0] != n or sh.shape[2] != 3:
        raise ValueError("sh must be [N, S, 3] with N = %d" % n)
    if out.dim() != 2 or out.shape[0] != n:
        raise ValueError("out must be [N, C] with N = %d" % n)
    _need(means3d, 3 * n, F32, "means3d")
    _need(sh, n * sh.shape[1] * 3, F32, "sh")
    _need(out, n * out.shape[1], F32, "out")
    cam = make_camera(camera)
    _check(_LIB.qr_sh_to_rgb(_stream(stream), n, degree, _ptr(means3d), _ptr(sh), sh.shape[1],
                             ctypes.byref(cam), _ptr(out), out.shape[1]))


def qr_sh_to_rgb_views(means3d, sh, degree, cameras, out, stream=None):
    """qr_sh_to_rgb for a list of cameras: out f32 [V, N, C] (C >= 3), view
    v's colour table in out[v]."""
    n = means3d.shape[0]
    if means3d.dim() != 2 or means3d.shape[1] != 3:
        raise ValueError("means3d must be [N, 3]")
    if sh.dim() != 3 or sh.shape[0] != n or sh.shape[2] != 3:
        raise ValueError("sh must be [N, S, 3] with N = %d" % n)
    if out.dim() != 3 or out.shape[0] != len(cameras) or out.shape[1] != n:
        raise ValueError("out must be [V, N, C] with V = %d, N = %d" % (len(cameras), n))
    _need(means3d, 3 * n, F32, "means3d")
    _need(sh, n * sh.shape[1] * 3, F32, "sh")
    _need(out, len(cameras) * n * out.shape[2], F32, "out")
    if out.data_ptr() % 16:
        raise ValueError("out must be 16-byte aligned")
    cams = make_cameras(cameras)
    _check(_LIB.qr_sh_to_rgb_views(_stream(stream), n, degree, _ptr(means3d), _ptr(sh), sh.shape[1],
                                   cams, len(cameras), _ptr(out), out.shape[2]))


def qr_devoxelize(offsets, voxel_unique, unique_pred, reduce, out, argmax=None, stream=None):
    """offsets: int64 [G+1]; voxel_unique: int32 [M]; unique_pred: f32 [U, C];
    out: f32 [G, C]; argmax: int32 [G, C] or None."""
    G = offsets.numel() - 1
    U, C = unique_pred.shape
    _need(offsets, G + 1, (torch.int64,), "offsets")
    _need(voxel_unique, voxel_unique.numel(), I32, "voxel_unique")
    _need(unique_pred, U * C, F32, "unique_pred")
    _need(out, G * C, F32, "out")
    _need(argmax, G * C, I32, "argmax")
    _check(_LIB.qr_devoxelize(_stream(stream), G, C, _ptr(offsets), _ptr(voxel_unique),
                              voxel_unique.numel(), U, _ptr(unique_pred), reduce, _ptr(out),
                              _ptr(argmax)))


def qr_devoxelize_backward(offsets, voxel_unique, n_unique, reduce, grad_out, argmax, grad_unique,
                           stream=None):
    G = offsets.numel() - 1
    C = grad_out.shape[1]
    _need(offsets, G + 1, (torch.int64,), "offsets")
    _need(voxel_unique, voxel_unique.numel(), I32, "voxel_unique")
    _need(grad_out, G * C, F32, "grad_out")
    _need(argmax, G * C, I32, "argmax")
    _need(grad_unique, n_unique * C, F32, "grad_unique")
    _check(_LIB.qr_devoxelize_backward(_stream(stream), G, C, _ptr(offsets), _ptr(voxel_unique),
                                       voxel_unique.numel(), n_unique, reduce, _ptr(grad_out),
                                       _ptr(argmax), _ptr(grad_unique)))


def pack_grads(grads) -> bytes:
    """Host bytes of a qr_view_grad array; `grads` are dicts with grad_out
    and (each optional) grad_features, grad_means2d, grad_conic_opacity."""
    arr = (qr_view_grad * len(grads))()
    for i, g in enumerate(grads):
        arr[i].grad_out = g["grad_out"].data_ptr()
        for f in ("grad_features", "grad_means2d", "grad_conic_opacity"):
            t = g.get(f)
            setattr(arr[i], f, t.data_ptr() if t is not None else None)
    return bytes(arr)


def pack_views(views) -> bytes:
    """Host bytes of a qr_view array; `views` are dicts of tensors / ints."""
    arr = (qr_view * len(views))()
    for i, v in enumerate(views):
        for f in ("tile_offsets", "sorted_gid", "means2d", "conic_opacity", "features", "out"):
            setattr(arr[i], f, v[f].data_ptr())
        for f in ("feature_scale", "T_q", "n_sel"):
            t = v.get(f)
            setattr(arr[i], f, t.data_ptr() if t is not None else None)
        arr[i].width, arr[i].height = int(v["width"]), int(v["height"])
    return bytes(arr)


def qr_batch_schedule(n_views, views_dev, view_first, schedule, workspace, stream=None):
    if views_dev.numel() < n_views * ctypes.sizeof(qr_view):
        raise ValueError("views_dev is smaller than n_views qr_view records")
    _need(view_first, n_views + 1, I32, "view_first")
    _need(schedule, 0, I32, "schedule")
    _check(_LIB.qr_batch_schedule(_stream(stream), n_views, _ptr(views_dev), _ptr(view_first),
                                  schedule.numel(), _ptr(schedule), _ptr(workspace),
                                  workspace.numel() * workspace.element_size()))
