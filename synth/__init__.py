"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates scenes only (trajectories, map points, observation lists,
noise, outliers, initial-state perturbations).  It holds none of the bundle
adjustment arithmetic: no residual, Jacobian, loss, normal equation or solver.
"""
from .scenes import (  # noqa: F401
    Scene, PoseRequest, make_config0, make_config1, make_config2, make_arc_scene,
    make_config3_sizes, make_config3_problem, make_config4_requests, make_small_drive,
    save_scene, load_scene, IMG_W, IMG_H, FX, FY, CX, CY,
    PoseGraph, make_pose_graph, EDGE_SEQUENTIAL, EDGE_LOOP, EDGE_EXTRINSIC, RigScene, make_rig_drive,
)
