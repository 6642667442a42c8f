"""MI355X (gfx950) Holographic Radiance Cascades.

Per-pixel fluence of a 2-D scene of emission and attenuation (Algorithm 1 of
the paper, without the blur), its vector-Jacobian product, and a batched
forward + backward over many scenes, all computed by the HIP library
``libhrc.so`` behind the C ABI of ``include/hrc.h``.  PyTorch supplies device
memory and streams only.

    from paper_2505_02041_amd import fluence, Context, Batch
"""
from .hrc import (Batch, Context, HRCFunction, MultibounceFunction, RGBFunction,  # noqa: F401
                  default_context, fluence, fluence_multibounce, fluence_rgb)
from ._lib import HRCError  # noqa: F401

__all__ = ["fluence", "fluence_multibounce", "fluence_rgb", "Context", "Batch", "HRCFunction",
           "MultibounceFunction", "RGBFunction", "default_context", "HRCError"]
