"""Seeded synthetic scenes and cameras.

This module only draws random numbers and builds camera poses. It holds none
of the rendering arithmetic (no projection, binning, blending or quantile
selection), so both the FP64 oracle and the HIP path can take their inputs
from it without sharing any of the method's code.
"""

from .scenes import (  # noqa: F401
    Camera,
    Scene,
    look_camera,
    make_tiny,
    make_room,
    room_poses,
    tiny_camera,
    room_camera,
    make_fd_case,
    make_batched,
    sh_coefficients,
    CONFIGS,
)
