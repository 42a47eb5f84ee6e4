"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method itself (no Dirac operator, no
alpha ratios, no solver, no correlator).  It only draws the inputs the method
is applied to:

* gauge fields: unit links (free field) or ``U = exp(i eps H)`` with ``H``
  traceless Hermitian and Gaussian per link, projected back to SU(3);
* distance profiles ``alpha(x0)`` as plain tables of ``T`` positive numbers
  (the caller of the library passes such a table; how it is used is the
  method's business);
* point sources and random spinor fields;
* random gauge transformations (for covariance tests).

Host layout of every field (complex128, x0 slowest, x3 fastest):

* links   ``U[x0][x1][x2][x3][mu][a][b]``, mu = 0 (time), 1, 2, 3;
* spinors ``psi[x0][x1][x2][x3][spin][colour]``.

The paper's physics runs use CLS gauge ensembles (introduction and Table 1);
these synthetic fields stand in for them at the same lattice shapes.
"""
from .fields import (  # noqa: F401
    GELL_MANN,
    free_gauge,
    gauge_su3,
    project_su3,
    random_su3,
    random_spinor,
    point_source,
    point_sources_12,
    gauge_transform,
    volume,
    sf_boundary_link,
    gauge_su3_sf,
)
from .profiles import alpha_exp, alpha_exp_sym, alpha_cosh_paper, alpha_table, beta_cosh_paper  # noqa: F401
from .configs import CONFIGS, config  # noqa: F401
