"""MI355X (gfx950) implementation of the fully algebraic multilevel overlapping
Schwarz preconditioner of Al Daas & Jolivet (arXiv 2109.05908).

The compute path lives in ``libdd.so`` (HIP kernels behind the C-ABI declared
in ``include/dd.h``).  This package only marshals arguments: device buffers
and streams come from PyTorch.  Importing it does not load the library;
the first call does, and fails loudly if it has not been built.
"""
from .binding import (  # noqa: F401
    DD_EIG_DENSE, DD_EIG_LOBPCG, DD_EIG_LOBPCG_MATFREE, DD_FP32, DD_FP64, DD_SCHWARZ_ADDITIVE, DD_SCHWARZ_DEFLATED,
    DD_SEL_THRESHOLD, DD_SEL_THRESHOLD_CAP, DD_START_MODEL, DD_START_RANDOM, DD_START_RANGE, DDError,
    DeviceCSR, Preconditioner, WarmStartModel,
    autotune_report, extract_local, lib, library_path, meter_read, meter_start, partition_ggg, trim_device_cache,
)
