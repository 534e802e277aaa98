"""Seeded synthetic inputs for the swept-contact docking search.

This package only *makes inputs*: meshes, probe trajectories, SO(3) sample
sets and grid specs with the shapes, sizes and structure of the workloads the
paper evaluates (Sec. VI-A: free-form meshes of 5-8 mm scanned by a cylindrical
probe along sweeping contact trajectories).  It holds none of the method's
arithmetic (no signed distances, no grids, no correlation, no refinement), so
it can feed both the FP64 oracle and the HIP path without coupling them.
"""
from .gen import (  # noqa: F401
    SEED, rng, icosphere, perturbed_sphere, touchable_mask, quat_to_mat,
    mat_to_quat, quat_mul, haar_quaternion, sobol_hopf_so3, hemisphere_directions,
    min_rotation_to, footprint_top, make_trajectory, Problem, make_problem,
    CONFIGS, config_problem, grid_edge_m, BATCH_N, BATCH_M, SERVE_MESHES, SERVE_RATE, batch_spec,
    batch_problem, serve_mesh, serve_spec, serve_problem, serve_arrivals, serve_picks,
)
