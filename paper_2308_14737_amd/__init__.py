"""MI355X (gfx950) sort-free two-parameter Fuzzy Metaballs renderer.

Keselman & Hebert, "Flexible Techniques for Differentiable Rendering with 3D
Gaussians" (WACV 2024): forward (depth, alpha, normals, flow), hand-written adjoint,
and a persistent batched form, all in HIP kernels behind the C ABI of
include/fmb.h.  Importing the package loads libfmb.so and fails if it is not built.
"""

from . import _lib

_lib.load()

from .render import Batch, Cameras, Scene, kernel_times, launch_config, loss_grad, render, timing_enable  # noqa: E402,F401

__all__ = ["Batch", "Cameras", "Scene", "kernel_times", "launch_config", "loss_grad", "render", "timing_enable"]
