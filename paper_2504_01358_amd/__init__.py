"""Screen-space GGX shading of a G-buffer on AMD Instinct MI355X (gfx950).

The hot path of "3D Gaussian Inverse Rendering with Approximated Global
Illumination": deferred shading of a G-buffer with environment-lit diffuse
light plus one-bounce specular light estimated by Monte-Carlo rays marched in
screen space against the depth buffer.  The work runs in hand-written HIP
kernels behind the C-ABI of ``include/ssr.h``; ``ssr`` is the Python binding.

The binding (and with it ``libssr.so``) loads on first use of any public
name, so ``paper_2504_01358_amd.build`` can run before the library exists;
using the API without the library raises ImportError.
"""

_PUBLIC = (
    "BF16", "F16", "F32", "HIT_BACKGROUND", "HIT_CAP", "HIT_INVALID", "HIT_OFFSCREEN",
    "HIT_SKIPPED", "MARCH_HIZ", "MARCH_LINEAR", "NO_DIRECT", "NO_SPECULAR", "Context",
    "SSRError", "env_build_mips", "env_mips_floats", "hiz_build", "hiz_floats",
    "philox4x32_10", "status_string",
)

__all__ = list(_PUBLIC)


def __getattr__(name):
    if name in _PUBLIC:
        from . import ssr
        return getattr(ssr, name)
    raise AttributeError(name)
