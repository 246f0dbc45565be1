"""MI355X-native grouped full-spectrum fitting (LASP-Adam-GPU hot path).

The HIP library ``_lib/liblasp.so`` (sources in ``csrc/``, ABI in
``include/lasp.h``) does all arithmetic; ``lasp`` is its ctypes binding.
"""

from .lasp import (  # noqa: F401
    Arms,
    DEFAULT_BOX,
    FitResult,
    KERNELS,
    LaspError,
    Pool,
    ST_CONT_NONPOS,
    ST_NO_DATA,
    ST_NONFINITE_INPUT,
    ST_NOT_CONVERGED,
    ST_OUT_OF_BOX,
    ST_POLISH_LIMIT,
    ST_SIGMA_FLOOR,
    ST_SINGULAR,
    ST_STOP_FLAT,
    ST_STOP_RISING,
    clean_mask,
    fit_group,
    forward,
    library_path,
    load,
    profile_enable,
    profile_read,
    release,
    resample,
)
