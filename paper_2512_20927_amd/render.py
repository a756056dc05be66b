"""Frame-level runtime over the C ABI: buffers, the project -> bin_sort ->
render pipeline, and ``torch.autograd.Function`` wrappers.

Torch is used for device memory and streams only; every step of the
pipeline runs in the HIP kernels of libqrender.so.
"""

from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib as L
from ._lib import QR_TILE


@dataclasses.dataclass
class RenderParams:
    """Rasterisation constants (3D-GS conventions); see qr_params."""
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_eps: float = 1e-4
    dilation: float = 0.3
    guard: float = 1.3
    out_dtype: int = L.QR_F32  # Q-Render feature maps: L.QR_F32 or L.QR_BF16
    selection: int = L.QR_SELECT_QUANTILE  # or QR_SELECT_STRATIFIED (Stratified-K), QR_SELECT_TOPK

    def c(self) -> L.qr_params:
        return L.make_params(self.alpha_min, self.alpha_max, self.T_eps, self.dilation, self.guard,
                             self.out_dtype, self.selection)


def tiles_of(width: int, height: int):
    return (width + QR_TILE - 1) // QR_TILE, (height + QR_TILE - 1) // QR_TILE


@dataclasses.dataclass
class Projected:
    means2d: torch.Tensor        # f32 [N,2]
    conic_opacity: torch.Tensor  # f32 [N,4]
    depth: torch.Tensor          # f32 [N]
    tile_rect: torch.Tensor      # i32 [N,4]
    tiles_touched: torch.Tensor  # i32 [N] (u32 on the device side)


@dataclasses.dataclass
class Bins:
    tile_offsets: torch.Tensor   # i32 [n_tiles+1] (u32)
    sorted_gid: torch.Tensor     # i32 [capacity] (u32)
    total_pairs: torch.Tensor    # i32 [1] (u32)
    capacity: int
    sorted_keys: torch.Tensor | None = None  # i64 [capacity] (u64)


def alloc_projected(n: int, device="cuda") -> Projected:
    f = dict(dtype=torch.float32, device=device)
    return Projected(torch.empty(n, 2, **f), torch.empty(n, 4, **f), torch.empty(n, **f),
                     torch.empty(n, 4, dtype=torch.int32, device=device),
                     torch.empty(n, dtype=torch.int32, device=device))


def project(means3d, scales, quats, opacity, camera, params: RenderParams = RenderParams(),
            out: Projected | None = None, stream=None) -> Projected:
    n = means3d.shape[0]
    pr = out if out is not None else alloc_projected(n, means3d.device)
    L.qr_project(means3d, scales, quats, opacity, L.make_camera(camera), params.c(), pr.means2d,
                 pr.conic_opacity, pr.depth, pr.tile_rect, pr.tiles_touched, stream=stream)
    return pr


def project_views(means3d, scales, quats, opacity, cameras, params: RenderParams = RenderParams(),
                  out: Projected | None = None, stream=None) -> Projected:
    """Projection of the scene into every camera of a batch (one image size)
    in one launch per 32 cameras; record v*N + i is Gaussian i in view v."""
    n = means3d.shape[0]
    cams = cameras if isinstance(cameras, ctypes.Array) else L.make_cameras(cameras)
    pr = out if out is not None else alloc_projected(len(cams) * n, means3d.device)
    L.qr_project_views(means3d, scales, quats, opacity, cams, params.c(), pr.means2d,
                       pr.conic_opacity, pr.depth, pr.tile_rect, pr.tiles_touched, stream=stream)
    return pr


def count_pairs(pr: Projected, stream=None) -> int:
    ws = torch.empty(1, dtype=torch.int64, device=pr.depth.device)
    return L.qr_count_pairs(pr.tiles_touched, ws, stream=stream)


class Binner:
    """Holds the bin_sort workspace and outputs for a fixed (N, tiles, capacity)."""

    def __init__(self, n: int, width: int, height: int, capacity: int, device="cuda",
                 keep_keys: bool = False):
        self.n, self.width, self.height = n, width, height
        self.tiles_x, self.tiles_y = tiles_of(width, height)
        self.capacity = int(capacity)
        nb = L.qr_bin_sort_workspace_size(n, self.tiles_x, self.tiles_y, self.capacity)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.bins = Bins(torch.empty(self.tiles_x * self.tiles_y + 1, **i32),
                         torch.empty(max(self.capacity, 1), **i32), torch.empty(1, **i32),
                         self.capacity,
                         torch.empty(max(self.capacity, 1), dtype=torch.int64, device=device)
                         if keep_keys else None)

    def __call__(self, pr: Projected, stream=None) -> Bins:
        b = self.bins
        L.qr_bin_sort(self.n, self.tiles_x, self.tiles_y, pr.tile_rect, pr.tiles_touched, pr.depth,
                      self.capacity, self.workspace, b.sorted_gid, b.sorted_keys, b.tile_offsets,
                      b.total_pairs, stream=stream)
        return b


class ViewsBinner:
    """bin_sort_views workspace and outputs for a batch of n_views views of
    n_per_view Gaussians each: view v's tile lists are tiles
    [v*T, (v+1)*T) of one stacked grid (T tiles per view) and hold
    view-local Gaussian ids."""

    def __init__(self, n_views: int, n_per_view: int, width: int, height: int, capacity: int,
                 device="cuda", keep_keys: bool = False):
        self.n_views, self.n_per_view = n_views, n_per_view
        self.width, self.height = width, height
        self.tiles_x, self.tiles_y = tiles_of(width, height)
        self.tiles_per_view = self.tiles_x * self.tiles_y
        self.capacity = int(capacity)
        nb = L.qr_bin_sort_workspace_size(n_views * n_per_view, self.tiles_x, n_views * self.tiles_y,
                                          self.capacity)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.bins = Bins(torch.empty(n_views * self.tiles_per_view + 1, **i32),
                         torch.empty(max(self.capacity, 1), **i32), torch.empty(1, **i32),
                         self.capacity,
                         torch.empty(max(self.capacity, 1), dtype=torch.int64, device=device)
                         if keep_keys else None)

    def __call__(self, pr: Projected, stream=None) -> Bins:
        b = self.bins
        L.qr_bin_sort_views(self.n_views, self.n_per_view, self.tiles_x, self.tiles_y, pr.tile_rect,
                            pr.tiles_touched, pr.depth, self.capacity, self.workspace, b.sorted_gid,
                            b.sorted_keys, b.tile_offsets, b.total_pairs, stream=stream)
        return b

    def view(self, pr: Projected, v: int):
        """(Projected, Bins) of view v as views into the batch buffers (no
        copies), usable wherever a single view's projection and bins are."""
        n, T = self.n_per_view, self.tiles_per_view
        s = slice(v * n, (v + 1) * n)
        b = self.bins
        return (Projected(pr.means2d[s], pr.conic_opacity[s], pr.depth[s], pr.tile_rect[s],
                          pr.tiles_touched[s]),
                Bins(b.tile_offsets[v * T:(v + 1) * T + 1], b.sorted_gid, b.total_pairs,
                     b.capacity, b.sorted_keys))


def bin_sort(pr: Projected, width: int, height: int, capacity: int | None = None,
             keep_keys: bool = False, stream=None) -> Bins:
    """One-shot binning; counts the pairs (a synchronising call) when no
    capacity is given."""
    if capacity is None:
        capacity = count_pairs(pr, stream=stream)
    return Binner(pr.depth.shape[0], width, height, capacity, pr.depth.device, keep_keys)(pr, stream)


def render_quantile(pr: Projected, bins: Bins, features, width: int, height: int, K: int,
                    params: RenderParams = RenderParams(), feature_scale=None, out=None,
                    debug: bool = False, stream=None):
    """Quantile Rendering of one view. Returns dict(out, T_q, n_sel[, T_final,
    last_pos, sel_gid, sel_w]); with ``debug`` the selections and, for
    Algorithm 1's rule, T_final and last_pos are returned too."""
    dev = features.device
    dim = features.shape[1]
    if out is None:
        out_t = torch.bfloat16 if params.out_dtype == L.QR_BF16 else torch.float32
        out = torch.empty(height, width, dim, dtype=out_t, device=dev)
    T_q = torch.empty(height, width, dtype=torch.float32, device=dev)
    n_sel = torch.empty(height, width, dtype=torch.int32, device=dev)
    sel_gid = sel_w = T_final = last_pos = None
    if debug:
        sel_gid = torch.empty(height, width, K, dtype=torch.int32, device=dev)
        sel_w = torch.empty(height, width, K, dtype=torch.float32, device=dev)
        if params.selection == L.QR_SELECT_QUANTILE:
            T_final = torch.empty(height, width, dtype=torch.float32, device=dev)
            last_pos = torch.empty(height, width, dtype=torch.int32, device=dev)
    L.qr_render_quantile(width, height, params.c(), K, bins.tile_offsets, bins.sorted_gid,
                         pr.means2d, pr.conic_opacity, features, feature_scale, out, T_q, n_sel,
                         sel_gid, sel_w, stream=stream, T_final=T_final, last_pos=last_pos)
    r = dict(out=out, T_q=T_q, n_sel=n_sel)
    if debug:
        r.update(sel_gid=sel_gid, sel_w=sel_w)
        if T_final is not None:
            r.update(T_final=T_final, last_pos=last_pos)
    return r


def render_dense(pr: Projected, bins: Bins, features, width: int, height: int,
                 params: RenderParams = RenderParams(), feature_scale=None, out=None, stream=None):
    """Dense alpha blend of one view. Returns dict(out, T_final, n_contrib)."""
    dev = features.device
    dim = features.shape[1]
    if out is None:
        out = torch.empty(height, width, dim, dtype=torch.float32, device=dev)
    T_final = torch.empty(height, width, dtype=torch.float32, device=dev)
    n_contrib = torch.empty(height, width, dtype=torch.int32, device=dev)
    L.qr_render_dense(width, height, params.c(), bins.tile_offsets, bins.sorted_gid, pr.means2d,
                      pr.conic_opacity, features, feature_scale, out, T_final, n_contrib,
                      stream=stream)
    return dict(out=out, T_final=T_final, n_contrib=n_contrib)


def quantize(features, dtype: str):
    """Encode a float32 feature table for storage: 'bf16' -> (bf16 tensor, None),
    'fp8' -> (uint8 e4m3 codes, float32 per-row scale)."""
    n, dim = features.shape
    if dtype == "bf16":
        out = torch.empty(n, dim, dtype=torch.bfloat16, device=features.device)
        L.qr_quantize_features(features, L.QR_BF16, out)
        return out, None
    if dtype == "fp8":
        out = torch.empty(n, dim, dtype=torch.uint8, device=features.device)
        scale = torch.empty(n, dtype=torch.float32, device=features.device)
        L.qr_quantize_features(features, L.QR_FP8_E4M3, out, scale)
        return out, scale
    raise ValueError(dtype)


# ---- autograd -----------------------------------------------------------------

class QuantileRenderFn(torch.autograd.Function):
    """f~Q = QuantileRender(means2d, conic_opacity, features) for fixed bins.

    ``storage`` (optional) is a reduced-precision copy of ``features`` (bf16
    tensor or (uint8 e4m3 codes, scale)); the forward reads it and the
    gradient is taken with respect to the decoded values and returned for the
    float32 ``features``.
    """

    @staticmethod
    def forward(ctx, means2d, conic_opacity, features, bins, width, height, K, params, storage=None):
        feats, scale = (features, None) if storage is None else storage
        pr = Projected(means2d.contiguous(), conic_opacity.contiguous(), None, None, None)
        r = render_quantile(pr, bins, feats, width, height, K, params, scale)
        ctx.save_for_backward(pr.means2d, pr.conic_opacity)
        ctx.feats, ctx.scale = feats, scale
        ctx.bins, ctx.width, ctx.height, ctx.K, ctx.params = bins, width, height, K, params
        ctx.mark_non_differentiable(r["T_q"], r["n_sel"])
        return r["out"], r["T_q"], r["n_sel"]

    @staticmethod
    def backward(ctx, grad_out, _g_tq, _g_ns):
        means2d, conic_opacity = ctx.saved_tensors
        n, dim = ctx.feats.shape
        dev = means2d.device
        gf = torch.zeros(n, dim, dtype=torch.float32, device=dev)
        gm = torch.zeros(n, 2, dtype=torch.float32, device=dev)
        gc = torch.zeros(n, 4, dtype=torch.float32, device=dev)
        b = ctx.bins
        L.qr_render_quantile_backward(ctx.width, ctx.height, ctx.params.c(), ctx.K, b.tile_offsets,
                                      b.sorted_gid, means2d, conic_opacity, ctx.feats, ctx.scale,
                                      grad_out.contiguous(), gf, gm, gc)
        return gm, gc, gf, None, None, None, None, None, None


class DenseRenderFn(torch.autograd.Function):
    """Dense alpha blend (Eq. 1) for fixed bins; same conventions as QuantileRenderFn."""

    @staticmethod
    def forward(ctx, means2d, conic_opacity, features, bins, width, height, params, storage=None):
        feats, scale = (features, None) if storage is None else storage
        pr = Projected(means2d.contiguous(), conic_opacity.contiguous(), None, None, None)
        r = render_dense(pr, bins, feats, width, height, params, scale)
        ctx.save_for_backward(pr.means2d, pr.conic_opacity, r["out"])
        ctx.feats, ctx.scale = feats, scale
        ctx.bins, ctx.width, ctx.height, ctx.params = bins, width, height, params
        ctx.mark_non_differentiable(r["T_final"], r["n_contrib"])
        return r["out"], r["T_final"], r["n_contrib"]

    @staticmethod
    def backward(ctx, grad_out, _g_t, _g_n):
        means2d, conic_opacity, out = ctx.saved_tensors
        n, dim = ctx.feats.shape
        dev = means2d.device
        gf = torch.zeros(n, dim, dtype=torch.float32, device=dev)
        gm = torch.zeros(n, 2, dtype=torch.float32, device=dev)
        gc = torch.zeros(n, 4, dtype=torch.float32, device=dev)
        b = ctx.bins
        L.qr_render_dense_backward(ctx.width, ctx.height, ctx.params.c(), b.tile_offsets,
                                   b.sorted_gid, means2d, conic_opacity, ctx.feats, ctx.scale,
                                   out, grad_out.contiguous(), gf, gm, gc)
        return gm, gc, gf, None, None, None, None, None
