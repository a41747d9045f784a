"""Seeded synthetic inputs shared by the oracle and the device path.

This module only produces geometry (points, panel areas) and seeded random
vectors.  It holds none of the H-LU arithmetic: no kernel entries, no trees,
no factorisation.  Both sides of every parity test read their inputs from
here and nothing else.
"""
from .geometry import (icosphere, ellipsoid_surface, segment, circle, config_inputs,
                       rhs_uniform, rhs_normal, ellipsoid_batch_spec,
                       serving_trace)

__all__ = ["icosphere", "ellipsoid_surface", "segment", "circle", "config_inputs", "rhs_uniform",
           "rhs_normal", "ellipsoid_batch_spec", "serving_trace"]
