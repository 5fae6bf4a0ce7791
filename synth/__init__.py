"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only *generates inputs*: voxel tet meshes, material and
contact-geometry descriptors, external forces, initial velocities and loss
vectors, all from seeded NumPy generators.  It holds none of the method's
arithmetic (no masses, no element operators, no contact laws): each side
derives those from these inputs on its own.
"""

from .mesh import VoxelMesh, box_mesh, voxel_mesh, quadruped_mesh  # noqa: F401
from .configs import (  # noqa: F401
    SceneSpec,
    tiny_scene,
    beam_scene,
    slab_scene,
    quadruped_scene,
    batched_scenes,
    beam_push_force,
    loss_vector,
    slope_scene,
)
