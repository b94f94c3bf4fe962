"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This package is the only code that both the GPU path's callers and the FP64
oracle use.  It draws scenes and environment maps and ray-casts them into
G-buffers; it holds none of the shading method's arithmetic (no BRDF, no
environment filtering, no ray marching against the depth buffer).

The paper's own data (garage and campus sequences, trained Gaussian scenes)
is not public, so analytic scenes of a ground plane, spheres and boxes stand
in for the rasterised G-buffers of Eq. (g-buffer) in Sec. 3.2.
"""

from .generate import (  # noqa: F401
    CONFIGS,
    SERVE,
    Scene,
    bf16_round,
    f16_round,
    look_at_camera,
    make_env,
    make_scene,
    quantise_gbuffer,
    serving_requests,
    serving_scene,
)
