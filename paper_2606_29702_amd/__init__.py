"""MI355X (gfx950) residual-specific partial-jet PINN library.

The arithmetic lives in the HIP library libpinnjet.so (C ABI in
include/pinn_jet.h); this package only marshals torch tensors into it.
"""
from ._lib import PinnError, KINDS, PRECISIONS  # noqa: F401  (raises if the library is missing)
from .jet import CHANNELS, RESIDUALS, DEFAULT_COEF, ModifiedPlan, PinnPlan, PinnGraph, JetResidual, jet_residual, jet_step_noalloc  # noqa: F401
from .batch import BatchAdam, PinnBatch  # noqa: F401
from .jet import tuning_cache_clear, tuning_cache_load, tuning_cache_save, tuning_cache_size  # noqa: F401
from .optim import AdamState  # noqa: F401
