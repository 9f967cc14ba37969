"""MI355X-native tile-NeRF training step (Snake-NeRF, arXiv 2507.01631).

``libsnake.so`` (HIP, gfx950) holds every kernel; ``_lib`` is its ctypes
binding under the C names, ``pipeline`` composes one training step of a
tile and ``window`` the step of a 2x2 window of tiles with their own
networks, capturable in one HIP graph.
"""
from . import _lib
from ._lib import SnakeError, grid_desc, mlp_desc
from .pipeline import SnakeTileStep, TileNeRF, level_resolutions
from .window import WindowNeRF

__all__ = ["_lib", "SnakeError", "grid_desc", "mlp_desc", "SnakeTileStep", "TileNeRF",
           "WindowNeRF", "level_resolutions"]
