"""FP64 CPU oracle for screen-space GGX shading of a G-buffer.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
It shares no code with the HIP library: the two sides meet only in the seeded
input generator (``scenes``), which holds none of the method's arithmetic.

What it computes is the per-pixel estimator of the paper (3D Gaussian Inverse
Rendering with Approximated Global Illumination): a direct diffuse term read
from an environment map (Sec. 3.2, "Shading") plus a Monte-Carlo estimate of
the specular integral whose rays are marched in screen space against the
depth buffer (Sec. 3.3, the estimator below Fig. 3, and Appendix D,
Algorithm 1), with the microfacet terms of Appendix B.  Everything is float64
NumPy, vectorised over rays.  Places where the paper is silent or garbled
follow the readings documented with the design (camera conventions,
slab hit test, VNDF sampling, textbook Schlick, env-at-miss, ...); each
function names the reading it takes.

Modules:
  philox  - Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  camera  - pinhole projection and pixel-centre unprojection
  env     - equirect lookup, box mip chain, bilinear/trilinear filtering
  brdf    - GGX D, Schlick F, Smith G1, VNDF sampling, sample weights
  march   - min-max depth pyramids, linear march (Algorithm 1), the
            hierarchical march (the build's own traversal), brute-force checker
  shade   - the whole per-pixel estimator (optionally with given hit codes)
  grad    - derivatives of the estimator with the hit codes held fixed,
            by finite differences of the forward
"""

from . import brdf, camera, env, grad, march, philox, shade  # noqa: F401
from .shade import shade_frame, shade_pixels  # noqa: F401
