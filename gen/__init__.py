"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Only input manufacture lives here; see ``gen.scene``, ``gen.sequence`` and ``gen.keypoints``.
"""
from .scene import SPECS, SceneSpec, batch_spec, make_scene, plane_scene  # noqa: F401
from .keypoints import keypoints  # noqa: F401
