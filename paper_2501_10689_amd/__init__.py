"""MI355X-native VR-banded Kaczmarz RZF precoding (libvrk.so + thin binding)."""
from .vrk import (  # noqa: F401
    F_CONVERGED,
    F_MAXITER,
    F_NONFINITE,
    Plan,
    ProblemSpec,
    VrkError,
    autotune,
    host_plan,
    lib,
    options,
    precode,
)
