"""MI355X-native anchor-Gaussian render hot path (decode, project, bin/sort,
blend, and their backward) behind the libasgs C ABI (include/asgs.h).

Importing this package loads libasgs.so and fails loudly if it is not built.
"""
from . import _lib  # noqa: F401  (raises ImportError when the library is missing)
from .core import RenderContext, Decoder, pack_params, unpack_params, gaussians_to_device  # noqa: F401

__all__ = ["RenderContext", "Decoder", "pack_params", "unpack_params", "gaussians_to_device"]
