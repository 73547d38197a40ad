"""Seeded synthetic inputs for the DOPE binary pairwise energy (shared by the oracle and the GPU path).

This module only *defines inputs*: integer unaries u, integer pairwise weights w on a half-stencil, the
regularisation weight lambda (quantised), the block partition parameters and the ADMM schedule parameters.
It contains none of the method's arithmetic (no block decomposition, no solver, no ADMM step).

Energy being sampled (paper Eq. 1 with the neighbourhood of Sec. 1 and the log-posterior unary of Eq. 2):
    E(y) = sum_i u_i y_i + lambda * sum_{edges (i,j)} w_ij |y_i - y_j|,   y in {0,1}^n

Layout: raster order, x fastest: i = x + W*(y + H*z).  w has shape (h, n): w[o, i] is the weight of the edge
i <-> i + offset[o] for the half-stencil offsets returned by :func:`half_stencil`; it is 0 where i + offset[o]
falls outside the grid.

Rounding of generated real values is floor(x + 0.5) in float64 (host only; it defines the input).
"""
from .configs import (  # noqa: F401
    half_stencil,
    Problem,
    config1,
    config2,
    config2_even,
    config2_sized,
    config3_sized,
    config3,
    config4,
    config4_lsatr,
    config5_request,
    config5_image,
    config5_trace,
    config_kernel,
    config3_kernel5,
    random_problem,
    lambda_q8,
    DEFAULT_MU0_2D,
    DEFAULT_MU0_3D,
    DEFAULT_EPS_Q16,
)
from .multilabel import MultiLabelProblem, multilabel_image  # noqa: F401,E402
