"""FP64 CPU reference of the RK4IP step for coupled multimode NLSEs.

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library, and
only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU path: it reads plain
numpy arrays and uses numpy's FFT and matrix products in float64/complex128.

Pins (tests that tie it to the paper and to mathematics, not to itself) are
listed in the header of ``oracle/rk4ip.py``.
"""

from .rk4ip import (  # noqa: F401
    amplifier_gain,
    angular_frequencies,
    apply_linear,
    half_step_propagator,
    kerr_term,
    KerrGeneric,
    KerrManakov,
    KerrPacked,
    linear_operator,
    power,
    propagate,
    propagate_adaptive,
    propagate_steps,
    StepControlError,
    rk4ip_step,
    ssfm_agrawal_step,
    ssfm_rk4_step,
    step_doubling_estimate,
    time_grid,
)
