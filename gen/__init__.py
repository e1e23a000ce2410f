"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Only input manufacture lives here; see ``gen.scene``, ``gen.sequence``, ``gen.keypoints`` and ``gen.color``.
"""
from .scene import SPECS, SceneSpec, batch_spec, make_scene, plane_scene  # noqa: F401
from .keypoints import keypoints  # noqa: F401
from .color import color_image, point_colors  # noqa: F401
