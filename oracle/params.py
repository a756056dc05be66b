"""Render parameters of the oracle.

The paper fixes none of these numerically; it renders "following 3D-GS"
(Sec. 4.2). The values are the 3D-GS rasteriser conventions:

* alpha_min = 1/255 - a Gaussian whose alpha' at a pixel is below this is not
  part of that pixel's ray list I (it is not "rasterized" there).
* alpha_max = 0.99  - alpha' is clamped from above.
* T_eps = 1e-4      - the dense blend stops before transmittance drops below
  this (Eq. 1 itself has no stop; T_eps = 0 means every Gaussian on the ray).
* dilation = 0.3    - EWA low-pass filter added to the 2D covariance (px^2).
* guard = 1.3       - the projection Jacobian is evaluated with x/z, y/z
  clamped to 1.3 x the half field of view.
* tile = 16         - screen tiles are 16 x 16 pixels.
"""

import dataclasses


@dataclasses.dataclass(frozen=True)
class RenderParams:
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_eps: float = 1e-4
    dilation: float = 0.3
    guard: float = 1.3
    tile: int = 16
