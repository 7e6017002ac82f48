"""Seeded synthetic inputs for multimode-fiber propagation runs.

This package only draws inputs: launch fields, per-mode propagation
constants, Kerr coupling tensors and request streams.  It contains none of the
propagation method's arithmetic (no dispersion operator, no Kerr evaluation,
no Runge-Kutta step), so that both the FP64 reference implementation and the
GPU library can consume the same bytes without sharing any code.
"""

from .fiber import (  # noqa: F401
    CONFIG_NAMES,
    Problem,
    make_problem,
    soliton_problem,
    symmetric_gaussian_tensor,
    pair_exchange_tensor,
    mode_group_mask,
    mode_groups,
    shaped_field,
    serving_stream,
    request_problem,
    RequestSpec,
    table3_beta,
    manakov_problem,
    xpm_matrix,
)
