"""MI355X-native (gfx950) library for MIS-SLAM's per-frame deformable registration.

The compute lives in libmisslam.so (C ABI in include/misslam.h); ``misslam``
is its tensor-level Python binding.
"""
