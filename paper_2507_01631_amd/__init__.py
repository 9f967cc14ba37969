"""MI355X-native tile-NeRF training step (Snake-NeRF, arXiv 2507.01631).

``libsnake.so`` (HIP, gfx950) holds every kernel; ``_lib`` is its ctypes
binding under the C names and ``pipeline`` composes one training step.
"""
from . import _lib
from ._lib import SnakeError, grid_desc, mlp_desc
from .pipeline import SnakeTileStep, TileNeRF, level_resolutions

__all__ = ["_lib", "SnakeError", "grid_desc", "mlp_desc", "SnakeTileStep", "TileNeRF",
           "level_resolutions"]
