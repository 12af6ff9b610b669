"""Seeded synthetic inputs shared by the FP64 CPU oracle and the GPU path.

This package only *generates inputs*: mesh vertex coordinates and tetrahedra,
periodic vertex identification, boundary tags, per-element material arrays,
initial-condition functions, time-step size, point sources and receiver
positions.  It holds none of the method's arithmetic (no basis, quadrature,
flux, constitutive law or time stepping); both the oracle and the GPU library
derive everything else from these arrays on their own.
"""
from .mesh import cube_mesh, kuhn_inradius
from .configs import (Workload, make_workload, plane_wave_ic, CONFIGS,
                      table1_material)

__all__ = ["cube_mesh", "kuhn_inradius", "Workload", "make_workload",
           "plane_wave_ic", "CONFIGS", "table1_material"]
