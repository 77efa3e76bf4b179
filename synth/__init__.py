"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and evaluates analytic initial fields on the
staggered grid.  It holds none of the solver's arithmetic (no divergence,
gradient, Poisson solve or projection): both the CPU oracle and the GPU path
receive exactly the arrays produced here.

Array convention (shared by every consumer): fields are float64 arrays of
shape (nz + 2, ny, nx), index [k, j, i], x fastest.  Planes k = 0 and
k = nz + 1 are ghost planes; this module leaves them at zero.  A square duct (walls
in y as well) adds two ghost rows after the interior ones, (nz + 2, ny + 2, nx).
  u[k, j, i]  at x = (i + 1) dx, y = (j + 1/2) dy, z = zc[k]
  v[k, j, i]  at x = (i + 1/2) dx, y = (j + 1) dy, z = zc[k]
  w[k, j, i]  at x = (i + 1/2) dx, y = (j + 1/2) dy, z = zf[k]
  p, nu_t     at cell centres (i + 1/2, j + 1/2, zc[k])
"""
from .fields import (isotropic_field, channel_field, duct_field, uniform_shear_field,
                     taylor_green_field, random_state, box_ensemble)

__all__ = ["isotropic_field", "channel_field", "duct_field", "uniform_shear_field",
           "taylor_green_field", "random_state", "box_ensemble"]
