"""Seeded synthetic inputs (scenes, depth frames, trajectories) and trajectory
metrics.  Shared by the tests, the smoke check and the benchmark; holds none
of the pose-search or fusion arithmetic."""
from .camera import Intrinsics, Pose, axis_angle, look_rotation, mat_to_quat, quat_to_mat, render_depth
from .configs import Sequence, SmallFrame, fast_trajectory, room_sequence, small_frame
from .metrics import ate, horn_align, translation_error
from .scene import Box, Cylinder, Scene, Sphere, analytic_tsdf, procedural_room, unit_box_room

__all__ = [
    "Intrinsics", "Pose", "axis_angle", "look_rotation", "mat_to_quat", "quat_to_mat", "render_depth",
    "Sequence", "SmallFrame", "fast_trajectory", "room_sequence", "small_frame", "ate", "horn_align",
    "translation_error", "Box", "Cylinder", "Scene", "Sphere", "analytic_tsdf", "procedural_room",
    "unit_box_room",
]
