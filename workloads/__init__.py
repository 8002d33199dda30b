"""Seeded synthetic inputs for the multibody MFS scattering path.

This package produces geometry only: point sets on each scatterer's shape,
body centres, incident directions and field targets.  It holds none of the
method's arithmetic (no fundamental solution, no matrices, no solves), so that
the CPU oracle and the HIP path can both draw the exact same inputs from it
while sharing no computational code.
"""

from .shapes import (  # noqa: F401
    ShapeDiscretisation,
    disk2d,
    starfish2d,
    ellipse2d,
    teardrop2d,
    cshape2d,
    rod2d,
    kite2d,
    sphere3d,
    ellipsoid3d,
    bumpy_sphere3d,
    torus3d,
    fibonacci_sphere,
    circle_points,
)
from .scenes import (  # noqa: F401
    Scene,
    grid_centres_2d,
    random_centres,
    random_rotations,
    plane_wave_directions_2d,
    far_targets,
)
from . import serving  # noqa: F401
from .configs import (  # noqa: F401
    BASE_SEED,
    WorkloadConfig,
    c1_disks16,
    c2_starfish2000,
    c3_spheres1000,
    c4_mixed_multi_incidence,
    c4_shapes,
    CONFIGS,
    make_scene,
)
