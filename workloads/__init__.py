"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package only draws Gaussians, cameras and cotangents.  It holds none of the
renderer's arithmetic: no ray-Gaussian intersection, blending, projection or
gradient is computed here.
"""

from .synth import (  # noqa: F401
    BETA1, BETA2, ETA,
    Scene, Cameras, Workload,
    make_config, make_scene, look_at, fibonacci_sphere, perturb_means,
    pixel_indices, random_cotangents, config_names, with_backward_flow,
)
