"""Seeded synthetic inputs for the V-FPI contact solve.

This package is the only code shared by the CPU oracle (``oracle/``) and the
HIP path (``paper_2201_09212_amd``).  It builds the data of one time step of
the linear contact problem  A v = b + J_c^T lambda  (paper Sec. II-A, eq. lindyn;
Sec. III-A, eq. jcnode): a block-sparse SPD matrix A, the right-hand side b, a
warm-start velocity, and nodal contacts (node index, SO(3) contact frame R,
phi, mu).  It holds none of the solver's arithmetic: no W, no projection, no
iteration.  Scenes are described in ``scenes.cloth``, ``scenes.fem`` and
``scenes.random``.
"""
from .problem import Problem, concat_problems, rng
from .geometry import onb_duff, contacts_from_gaps
from .cloth import (ClothScene, cloth_cfg1, cloth_cfg2, cloth_cfg2_drop, cloth_cfg4_envs, cloth_cfg5_scene, cloth_drape,
                    cloth_pair_collision)
from .fem import FemScene, fem_block, fem_cfg3, fem_ctx
from .random import random_problem, inclined_plane_particles, two_level_diagonal, colliding_particle_pairs

__all__ = [
    "Problem", "concat_problems", "rng", "onb_duff", "contacts_from_gaps",
    "ClothScene", "cloth_cfg1", "cloth_cfg2", "cloth_cfg2_drop", "cloth_cfg4_envs", "cloth_cfg5_scene",
    "FemScene", "fem_block", "fem_cfg3", "fem_ctx", "cloth_drape", "random_problem", "inclined_plane_particles",
]
from .vnode import VirtualScene, rigid_box_on_floor, particles_on_cloth
