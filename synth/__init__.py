"""Seeded synthetic inputs for the normal bake.

This package only produces inputs (meshes, per-corner UVs, vertex normals of the
high-poly surface, target maps are NOT made here).  It holds none of the bake's
own arithmetic: no rasterisation, ray query, tangent frame or encoding.  Both
the FP64 oracle and the GPU path consume what it returns.
"""
from .meshes import (  # noqa: F401
    icosphere,
    unit_directions,
    analytic_radius,
    analytic_normal,
    gradient_noise,
    noise_radius,
    bump_radius,
    displace,
    vertex_normals,
    face_grid_atlas,
    decimate,
    Asset,
    make_config,
    make_batch_assets,
    batch_asset_specs,
    make_batch_asset,
    CONFIGS,
)
