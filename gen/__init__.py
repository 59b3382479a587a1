"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only draws random numbers and lays them out; it holds none of the
rendering arithmetic.  Every array is in the boundary's SoA layout:

  mu [3,N], scale [3,N], rot [4,N] (w,x,y,z), sh [K,3,N] with K=(D+1)^2,
  opacity [N], vel [3,N], period [N], tau [N], beta [N]      (all float32)

Draws are made in float64 with numpy's PCG64 (``default_rng(seed)``) and cast
to float32, in the fixed order mu, log-scale, rotation, opacity, velocity,
period, tau, beta, sh; cameras and request traces come after.
"""
from .scenes import (  # noqa: F401
    CONFIGS,
    FIELDS,
    make_scene,
    make_camera,
    yaw_camera,
    make_config,
    make_trace,
    make_target,
    subset_scene,
)
