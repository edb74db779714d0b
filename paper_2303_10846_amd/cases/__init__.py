"""Seeded synthetic inputs (meshes, velocity sets, case constants) shared by the solver and its tests."""
from . import configs, dvs, mesh  # noqa: F401
from .configs import (capsule_case, cavity_case, freestream_box_case, rest_state,  # noqa: F401
                      small_sphere_case, sphere_case)
