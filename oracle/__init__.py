"""FP64 CPU oracle for the sort-free two-parameter Fuzzy-Metaballs renderer.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark import this package; the GPU library never does.
"""

from .oracle import (  # noqa: F401
    build, lib_path, load, OracleScene, pixel_rays, dir_rays, project,
    render, backward, ray_terms, max_weight, blend_weights, MODELS, split_statistic,
    prune_mask, split_mask, split_gaussians, render_workload_view, loss_grad,
)
