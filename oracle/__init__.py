"""FP64 CPU oracle for the NeDF composition hot path (test infrastructure).

This package is a plain, slow, obviously correct NumPy float64 statement of
what the GPU path computes, written from the paper (Gao et al., "A General
Implicit Framework for Fast NeRF Composition and Rendering", AAAI 2024,
arXiv 2308.04669).  Each function cites the section, equation or algorithm
it follows.  It is test infrastructure only: the tests, the smoke entry point
and the benchmark's CPU-baseline leg may import it; the product path never
does, and this package imports nothing from the product package.  The only
code shared with the GPU side is the seeded input generator in ``synthetic``,
which holds none of the method's arithmetic.

Where the paper is silent or ambiguous the oracle takes a stated reading
(listed in the design notes); library primitives (matmul, cumsum, exp) serve
as steps, with no blocking or reordering beyond the stated definitions.

Parity pins: every function here is checked by the CPU test-suite against a
closed form, an invariant, a brute-force evaluation or a library routine,
except the random-MLP density values and trained NeDF weights themselves,
which are "parity unpinned" beyond being the stated definition (the MLP
forward pass itself is pinned on hand-set weights).
"""
from .geometry import (camera_rays, to_local, pluecker, encode, sphere_chord,
                       inverse_transform, f32_record, RecordInstance)
from .rounding import round_bf16, round_e4m3, bf16_rounding_margin, e4m3_rounding_margin
from .fields import mlp_forward, density, nerf_eval, nedf_eval, sdf, surface_value, fp8_calibrate
from .render import (march, march_compose, nedf_pair, nedf_compose, secant_refine, depth_lower_bound,
                     compose_pruned, march_compose_pruned, nedf_compose_pruned,
                     shade_deferred, shadow_factor, composite)
from .train import nedf_loss_and_grads, adam_step
from .classifier import (line_points, encode_points, segment, segment_inverse, classifier_forward,
                         classifier_decode, classifier_eval, classifier_loss_and_grads)

__all__ = [
    "camera_rays", "to_local", "pluecker", "encode", "sphere_chord", "inverse_transform", "f32_record",
    "RecordInstance",
    "round_bf16", "round_e4m3", "bf16_rounding_margin", "e4m3_rounding_margin", "fp8_calibrate", "mlp_forward", "density", "nerf_eval", "nedf_eval", "sdf",
    "march", "march_compose", "nedf_pair", "nedf_compose", "secant_refine", "depth_lower_bound",
    "compose_pruned", "march_compose_pruned", "nedf_compose_pruned",
    "shade_deferred", "shadow_factor", "composite", "nedf_loss_and_grads", "adam_step",
    "line_points", "encode_points", "segment", "segment_inverse", "classifier_forward", "classifier_decode",
    "classifier_eval", "classifier_loss_and_grads",
]
