"""Seeded synthetic inputs (media, sources, solver settings) shared by the tests,
the benchmark and the oracle checks.

This package holds none of the solver's arithmetic: it only draws random media
fields, converts velocities to Lame parameters, places point sources and names
the workload configurations.  Both the HIP path and the CPU oracle receive the
arrays it produces as plain inputs.
"""
from .media import (gaussian_random_field, lame_from_velocities, gardner_density,
                    homogeneous_media, heterogeneous_2d_media, layered_3d_media,
                    shear_frequency)
from .configs import CONFIGS, get_config, Workload

__all__ = ["gaussian_random_field", "lame_from_velocities", "gardner_density",
           "homogeneous_media", "heterogeneous_2d_media", "layered_3d_media",
           "shear_frequency", "CONFIGS", "get_config", "Workload"]
