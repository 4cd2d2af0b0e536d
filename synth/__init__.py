"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds geometry, camera, cache, emission and material generators
only.  It performs none of the method's arithmetic (no sampling, no ray
casting, no shading, no loss): every array it returns is an *input* to the
bake or to the factored render.
"""
from .scenes import (  # noqa: F401
    Scene,
    Camera,
    tiny_box,
    room,
    serving_rooms,
    large_room,
    material_grid,
    random_shading,
    random_materials,
    random_observations,
    observation_noise,
    serving_trace,
    emitter_observations,
    emission_mask,
    hashgrid_params,
    emitter_schedule,
    icosphere,
    SERVING_TRIANGLES,
    SIGMA_GRID,
)
