"""Quantile Rendering of high-dimensional Gaussian features on AMD MI355X.

The compute path is libqrender.so (hand-written HIP for gfx950) behind the C
ABI of include/qrender.h; this package binds it with ctypes and adds a thin
frame-level runtime and autograd wrappers. Importing the package loads the
library and fails loudly if it has not been built.
"""

from . import _lib  # noqa: F401  (loads libqrender.so or raises ImportError)
from ._lib import QRError, version  # noqa: F401
from .render import (  # noqa: F401
    RenderParams,
    Projected,
    Bins,
    Binner,
    ViewsBinner,
    project,
    project_views,
    count_pairs,
    bin_sort,
    render_quantile,
    render_dense,
    quantize,
    QuantileRenderFn,
    DenseRenderFn,
    tiles_of,
)
