"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds only input generators (random gauge links, random spinor
fields, random gauge transformations).  It contains none of the trace
estimation method's arithmetic: no Dirac operator, no noise, no solver, no
estimator.  Both the CPU oracle and the GPU library receive the arrays it
produces through their canonical layouts:

* gauge:  complex128, shape (4, V, 3, 3) -- [mu][site][row][col]
* spinor: complex128, shape (V, 4, 3)    -- [site][spin][colour]

with site = x + Lx*(y + Ly*(z + Lz*t)) and mu = 0..3 the x, y, z, t axes.
"""

from .inputs import (  # noqa: F401
    gell_mann,
    su3_exp_field,
    gauge_field,
    random_spinor,
    gauge_transform,
    volume,
)
