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
    fit_group,
    forward,
    library_path,
    load,
    profile_enable,
    profile_read,
    release,
)
