"""Seeded synthetic scenes for geometry-aware guided matching.

This package only produces inputs: camera poses, 3D points, keypoints,
uint8 descriptors and per-pair fundamental matrices.  It holds none of the
matching arithmetic, so both the CPU oracle and the GPU library consume the
same bytes from it.
"""
from .generator import (  # noqa: F401
    IMG_W, IMG_H, FOCAL, Camera, Image, PairScene, MultiViewScene,
    look_at_camera, fundamental_from_poses, make_pair_scene, make_two_view_2k,
    make_two_view_16k, make_multiview_scene, make_arc_batch, make_three_rings,
    make_ten_rings, sample_pairs_by_angle, covisible_pairs, poisson_arrivals,
    materialize, stress_requests, visibility_lists, visibility_csr, by_scale,
)
