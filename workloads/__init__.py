"""Seeded synthetic inputs for the volumetric-ray-casting (VRC) estimator.

This package only produces data: meshes, material maps, tabulated total cross
sections, ray batches and energy-bin edges.  It holds none of the estimator's
arithmetic, so both the GPU library's tests and the CPU oracle may take their
inputs from here without sharing any of the method's code.
"""

from .gen import (  # noqa: F401
    Mesh,
    RectMesh,
    rect_mesh,
    RZMesh,
    rz_mesh,
    rays_in_rz,
    XSTables,
    Mixtures,
    random_mixtures,
    density_field,
    Rays,
    Workload,
    E_MIN_MEV,
    E_MAX_MEV,
    isotropic_directions,
    log_uniform_energies,
    synthetic_sigma_table,
    constant_sigma_table,
    rays_in_box,
    rays_in_cylinder,
    rays_near_faces,
    slab_mesh,
    cylinder_spheres_mesh,
    sphere_mesh,
    log_bin_edges,
    config1_tiny,
    config2_multimaterial,
    config3_precision,
    config4_batches,
    config4_batches_device,
    config5_serving_geometry,
    rays_to_f32,
)
