"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmarks.

This module only draws random numbers and lays them out as float32 arrays. It
holds none of the rendering or decoding arithmetic: every quantity the method
computes is computed elsewhere (the oracle and the HIP library, independently).
"""
from .scenes import (  # noqa: F401
    Camera,
    PlainScene,
    AnchorScene,
    HEADS,
    look_at,
    camera_c1,
    camera_c2,
    camera_half,
    plain_scene,
    tiny_scene,
    anchor_scene,
    tiny_anchor_scene,
    anchor_weights,
    room_cells,
    targets,
    perturb_pose,
    trajectory,
    c1,
    c2,
    c3,
    c4,
    c5,
)
from .maps import residual_maps, feature_inputs, mapping_maps, uncertainty_inputs  # noqa: F401,E402
