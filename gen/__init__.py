"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Only input manufacture lives here; see ``gen.scene``.
"""
from .scene import SPECS, SceneSpec, batch_spec, make_scene, plane_scene  # noqa: F401
