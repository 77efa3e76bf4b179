"""Plain, slow FP64 CPU oracle of one CaLES substep (test infrastructure only).

This package exists to check the HIP library.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the library and its
Python binding never do, and it shares no code with them.  Every function
cites the passage of the paper (Xiao et al., "CaLES: A GPU-accelerated solver
for large-eddy simulation of wall-bounded flows", arXiv 2411.09364) that it
follows.  Where the paper is silent the reading taken is named R1..R40 in the
docstring of the function that uses it.

Modules
  grid      staggered grid, tanh stretching (R1)
  ops       divergence, gradient, Laplacian, advection, strain, SGS flux divergence
  bc        ghost planes and the log-law wall model (Alg. 2, Sec. 2.2 wall model)
  sgs       Smagorinsky / van Driest and dynamic Smagorinsky (Sec. 2.1, Eqs. smag..mij)
  poisson   eigenfunction-expansion Poisson solve (Sec. 2.2, Eq. poi)
  substep   RK3 predictor, CN-z, projection, pressure update, bulk forcing, dt (Alg. 1)
  mlp       learned Smagorinsky-coefficient closure (forward, backward, Adam, BF16 rounding)
  stats     long-run channel statistics, C_f and Re_tau, batch means, Eqs. eps_f and error

The square duct of Sec. 4.4 (walls in y and z, periodic x) runs through the same
modules: two ghost rows in y (grid.py), the y-wall rules and wall model (bc.py, R35),
the four-wall van Driest factor (sgs.py, R36), the cosine expansion in y (poisson.py,
R37), the dynamic model's y filter rules and x-line averages (sgs.py, R38) and the
learned closure's four-wall y+ input (mlp.py, R40); tests/test_oracle_duct.py pins them
(dense Poisson solve, laminar fixed point, exchange of y and z, closed-form shear inputs).

Parity unpinned (no paper value or closed form fixes them; listed also in the
design notes): the tanh map (R1), arithmetic two-point averages on the
stretched grid (R3), the filter width definition used by the static model
(R5), the edge eddy viscosity as a four-point mean (R18).
"""
from .case import Case
from .grid import Grid
from . import ops, bc, sgs, poisson, substep, mlp, stats

__all__ = ["Case", "Grid", "ops", "bc", "sgs", "poisson", "substep", "mlp", "stats"]
