"""MI355X-native 3D Gaussian Splatting rasterizer with exact ellipse/tile
intersection (FlashGS, arXiv 2408.07967), built on hand-written HIP kernels
for gfx950 behind a small C ABI.

Submodules load lazily so that the input generators (``scenes``) import
without the GPU library.
"""
import importlib

__all__ = ["scenes", "binding", "render"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
