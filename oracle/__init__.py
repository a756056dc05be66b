"""FP64 CPU oracle for Quantile Rendering of Gaussian feature maps.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library
(no kernels, headers, helpers or constant tables); the only thing both sides
use is the seeded input generator in ``synth``.

Every function is a plain, slow, obviously-correct float64 restatement of the
paper's definitions:

* ``project``   - EWA splatting of 3D Gaussians to 2D conics and tile
                  footprints (Sec. 3, the 3D-GS preliminaries).
* ``binning``   - (tile, depth, id) pairs sorted with Python's ``sorted``.
* ``render``    - dense alpha-blending (Eq. 1, "V-Render") and Quantile
                  Rendering (Algorithm 1) per tile, one list entry at a time.
* ``brute``     - per-pixel evaluation of every Gaussian in the scene, no tiles.
* ``selection`` - the closed "interval" form of the quantile selection.
* ``stratified`` - the Stratified-K variant (Appendix): per-ray thresholds
                  from the ray's transmittance statistics.
* ``topk``      - the Top-K sampler the paper compares with (the K largest
                  dense weights per ray, normalised by their sum).
* ``devoxelize`` - per-Gaussian features as the max (or mean) of the
                  predictions of the voxels each Gaussian covers.
* ``sh``        - view-dependent RGB from spherical-harmonic coefficients.
* ``backward``  - analytic gradients of both renderers.
* ``quant``     - bfloat16 / OCP e4m3 storage codes for the feature table.

Where the paper is silent, each module states the reading it takes.
Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or hand-worked examples.
"""

from .params import RenderParams  # noqa: F401
from .project import project, quat_to_rot  # noqa: F401
from .binning import bin_sort  # noqa: F401
from .render import render_dense, render_quantile, quantile_thresholds  # noqa: F401
from .brute import brute_force_render  # noqa: F401
from .selection import interval_selection  # noqa: F401
from .sh import sh_basis, sh_to_rgb  # noqa: F401
from .topk import render_topk  # noqa: F401
from .devoxelize import devoxelize, devoxelize_backward  # noqa: F401
from .stratified import render_stratified, stratified_thresholds, transmittance_stats  # noqa: F401
from .backward import dense_backward, quantile_backward  # noqa: F401
from . import quant  # noqa: F401
