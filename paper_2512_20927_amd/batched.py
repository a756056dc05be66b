"""Batched multi-view Quantile Rendering in one launch, and the autotuner
that picks its launch shape.

A batch is any list of views (each with its own scene, bins and output
buffer). ``BatchedQuantile`` packs the views' device pointers into a device
``qr_view`` table once; ``render`` then issues a single launch over all
(view, tile) items: either one workgroup per item, or a fixed number of
persistent workgroups per CU taking items through an atomic counter. Two
schedules (item orders) are available: ``natural`` (view-major order, fixed)
and ``heavy`` (longest tile lists first, built on the device by
``qr_batch_schedule`` from the current bins, so no host round trip). The
autotuner times the candidates (schedule x workgroups per CU) with HIP events
and caches the winner as JSON keyed by device, shapes and K. ``backward``
runs the Q-Render backward of every view in one launch over the same items.
``BatchedDense`` renders the dense blend over the same items and launch
shapes.
"""

from __future__ import annotations

import json
import os

import torch

from . import _lib as L
from .render import tiles_of

SCHEDULES = ("natural", "heavy")


def _check_tensor(t, numel, dtypes, name, device):
    """Shape, dtype, layout and device of one view array (dtype and size
    first, so that the message names the mismatch that matters)."""
    if t is None:
        raise ValueError("%s is required" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s: dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.device != device:
        raise ValueError("%s is on %s, the batch on %s" % (name, t.device, device))


def validate_views(views, K: int, dim: int, dtype_code: int, params, dense: bool = False):
    """Host-side checks of every view record before its pointers are packed
    into the device table: the batched kernels read sizes from the records
    and cannot check the buffers behind them, so a mismatch here would be an
    out-of-bounds access there. Raises TypeError / ValueError naming the view
    and field."""
    if not views:
        raise ValueError("a batch needs at least one view")
    if not dense and not 1 <= K <= L.QR_MAX_K:
        raise ValueError("K = %d outside [1, %d]" % (K, L.QR_MAX_K))
    out_dt = (torch.bfloat16,) if params.out_dtype == L.QR_BF16 else L.F32
    feat_dt = tuple(t for t, c in L.DTYPE_CODE.items() if c == dtype_code)
    dev = views[0]["out"].device
    for i, v in enumerate(views):
        W, H = int(v["width"]), int(v["height"])
        if W <= 0 or H <= 0:
            raise ValueError("view %d: image size %dx%d" % (i, W, H))
        tx, ty = tiles_of(W, H)
        f = v["features"]
        name = lambda k: "view %d: %s" % (i, k)
        if f.dim() != 2 or f.shape[1] != dim:
            raise ValueError("%s must be [N, %d], got %s" % (name("features"), dim, tuple(f.shape)))
        n = f.shape[0]
        _check_tensor(f, n * dim, feat_dt, name("features"), dev)
        if dtype_code == L.QR_FP8_E4M3:
            _check_tensor(v.get("feature_scale"), n, L.F32, name("feature_scale"), dev)
        _check_tensor(v["tile_offsets"], tx * ty + 1, L.I32, name("tile_offsets"), dev)
        _check_tensor(v["sorted_gid"], 1, L.I32, name("sorted_gid"), dev)
        _check_tensor(v["means2d"], 2 * n, L.F32, name("means2d"), dev)
        _check_tensor(v["conic_opacity"], 4 * n, L.F32, name("conic_opacity"), dev)
        _check_tensor(v["out"], W * H * dim, out_dt, name("out"), dev)
        if v.get("T_q") is not None:
            _check_tensor(v["T_q"], W * H, L.F32, name("T_q"), dev)
        if v.get("n_sel") is not None:
            _check_tensor(v["n_sel"], W * H, L.I32, name("n_sel"), dev)


class BatchedQuantile:
    def __init__(self, views, K: int, dim: int, dtype_code: int, params, _dense: bool = False):
        """views: list of dicts with tile_offsets, sorted_gid, means2d,
        conic_opacity, features, feature_scale (or None), out, T_q, n_sel (or
        None), width, height (all tensors on one device); checked by
        validate_views before anything is packed."""
        validate_views(views, K, dim, dtype_code, params, dense=_dense)
        self.n_views = len(views)
        self.K, self.dim, self.dtype_code, self.params = K, dim, dtype_code, params
        dev = views[0]["out"].device
        self._views = views  # keeps the tensors alive
        raw = L.pack_views(views)
        self.views_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        counts = [tiles_of(v["width"], v["height"])[0] * tiles_of(v["width"], v["height"])[1] for v in views]
        first = [0]
        for c in counts:
            first.append(first[-1] + c)
        self.n_items = first[-1]
        self.view_first = torch.tensor(first, dtype=torch.int32, device=dev)
        nat = [(v << L.QR_BATCH_TILE_BITS) | t for v, c in enumerate(counts) for t in range(c)]
        self.natural = torch.tensor(nat, dtype=torch.int64, device=dev).to(torch.int32)
        self.heavy = torch.empty(self.n_items, dtype=torch.int32, device=dev)
        self.sched_ws = torch.empty(64, dtype=torch.int32, device=dev)
        self.counter = torch.empty(8, dtype=torch.int32, device=dev)  # one work counter per XCD
        props = torch.cuda.get_device_properties(dev)
        self.n_cu = props.multi_processor_count
        self.device_name = props.name

    def schedule(self, kind: str):
        if kind == "natural":
            return self.natural
        if kind == "heavy":
            L.qr_batch_schedule(self.n_views, self.views_dev, self.view_first, self.heavy, self.sched_ws)
            return self.heavy
        raise ValueError(kind)

    def render(self, kind: str = "natural", wg_per_cu: int = 0, start_event=None):
        """wg_per_cu 0: one workgroup per (view, tile) item; > 0: that many
        persistent workgroups per CU taking items through per-XCD work
        counters. start_event (optional) is recorded on the current stream
        after the schedule is built, right before the render launch."""
        sched = self.schedule(kind)
        if start_event is not None:
            start_event.record()
        L.qr_render_quantile_batched(self.n_views, self.views_dev, self.params, self.K,
                                     self.dtype_code, self.dim, sched, self.n_cu * wg_per_cu,
                                     self.counter if wg_per_cu > 0 else None)

    def set_grads(self, grads):
        """grads: one dict per view (same order as the views) with grad_out
        f32[H, W, dim] and the accumulated gradient tensors grad_features,
        grad_means2d, grad_conic_opacity (each may be None; views of one scene
        may share them). Validated against the views' shapes."""
        if len(grads) != self.n_views:
            raise ValueError("need one gradient record per view")
        for v, g in zip(self._views, grads):
            n, dim = v["features"].shape[0], self.dim
            L._need(g["grad_out"], v["width"] * v["height"] * dim, L.F32, "grad_out")
            for f, per in (("grad_features", dim), ("grad_means2d", 2), ("grad_conic_opacity", 4)):
                if g.get(f) is not None:
                    L._need(g[f], n * per, L.F32, f)
        self._grads = grads  # keeps the tensors alive
        raw = L.pack_grads(grads)
        self.grads_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.views_dev.device)

    def backward(self, kind: str = "natural", wg_per_cu: int = 0):
        """Accumulates the Q-Render gradients of every view (set_grads) in
        one launch; same launch shapes as render."""
        if getattr(self, "grads_dev", None) is None:
            raise RuntimeError("set_grads() first")
        sched = self.schedule(kind)
        L.qr_render_quantile_batched_backward(self.n_views, self.views_dev, self.grads_dev,
                                              self.params, self.K, self.dtype_code, self.dim,
                                              sched, self.n_cu * wg_per_cu,
                                              self.counter if wg_per_cu > 0 else None)

    def key(self) -> str:
        shapes = sorted({(v["width"], v["height"]) for v in self._views})
        return "%s|views=%d|%s|D=%d|K=%d|dtype=%d" % (self.device_name, self.n_views, shapes,
                                                      self.dim, self.K, self.dtype_code)


class BatchedDense(BatchedQuantile):
    """The dense blend (Eq. 1) over the same view table, items, schedules and
    launch shapes as BatchedQuantile: the two renderers then differ only in
    which Gaussians of each ray they blend. Each view's ``T_q`` / ``n_sel``
    tensors receive T_final / n_contrib. ``autotune`` works on it unchanged
    (K = 0 selects the dense launch in the library's autotuner)."""

    def __init__(self, views, dim: int, dtype_code: int, params):
        if params.out_dtype != L.QR_F32:
            raise ValueError("the dense blend writes float32 maps only")
        # K = 0 marks the dense launch (the library's autotuner times it)
        super().__init__(views, 0, dim, dtype_code, params, _dense=True)

    def render(self, kind: str = "natural", wg_per_cu: int = 0, start_event=None):
        sched = self.schedule(kind)
        if start_event is not None:
            start_event.record()
        L.qr_render_dense_batched(self.n_views, self.views_dev, self.params, self.dtype_code,
                                  self.dim, sched, self.n_cu * wg_per_cu,
                                  self.counter if wg_per_cu > 0 else None)

    def set_grads(self, grads):
        raise NotImplementedError("the batched launch has no dense backward; use "
                                  "qr_render_dense_backward per view")

    def backward(self, kind: str = "natural", wg_per_cu: int = 0):
        raise NotImplementedError("the batched launch has no dense backward")


def default_cache_path() -> str:
    return os.environ.get("QRENDER_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "qrender", "autotune.json"))


def autotune(bq: BatchedQuantile, wg_per_cu=(0, 2, 4, 8), schedules=SCHEDULES, reps: int = 3,
             cache_path: str | None = None, use_cache: bool = True):
    """Times every (schedule, workgroups per CU) candidate (0 workgroups per
    CU = one workgroup per item) through qr_autotune_batched and returns
    (best_config, timings_ms). The best is cached under bq.key()."""
    cache_path = cache_path or default_cache_path()
    cache = {}
    if use_cache and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if bq.key() in cache:
            return cache[bq.key()], {}
    # the timing loop runs in the library (qr_autotune_batched, HIP events)
    scheds = [bq.schedule(kind) for kind in schedules]  # builds the device-side schedules
    bi, bw, ms = L.qr_autotune_batched(bq.n_views, bq.views_dev, bq.params, bq.K, bq.dtype_code,
                                       bq.dim, scheds, list(wg_per_cu), reps, bq.counter)
    timings = {"%s/%d" % (kind, w): ms[i][j] for i, kind in enumerate(schedules)
               for j, w in enumerate(wg_per_cu)}
    kind, w = schedules[bi], bw
    cfg = {"schedule": kind, "wg_per_cu": int(w), "ms": timings["%s/%d" % (kind, w)]}
    cache[bq.key()] = cfg
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return cfg, timings
