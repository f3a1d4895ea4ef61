"""MI355X (gfx950) Fuzzy Metaballs renderers: the sort-free two-parameter blend and the
zero-parameter alpha compositing.

Keselman & Hebert, "Flexible Techniques for Differentiable Rendering with 3D
Gaussians" (WACV 2024): forward (depth, alpha, normals, colour, forward and backward
flow), hand-written adjoint, and a batched form, all in HIP kernels behind the C ABI
of include/fmb.h.  Importing the package loads libfmb.so and fails if it is not built.
"""

from . import _lib
from ._lib import FmbError  # noqa: F401

_lib.load()

from .render import (Batch, Cameras, Scene, kernel_times, launch_config, loss_grad, render,  # noqa: E402,F401
                     set_launch_config, timing_enable)

__all__ = ["Batch", "Cameras", "FmbError", "Scene", "kernel_times", "launch_config", "loss_grad", "render",
           "set_launch_config", "timing_enable"]
