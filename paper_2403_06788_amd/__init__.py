"""MI355X-native dual-scale GRFT (DS-GRFT) coherent-integration search.

The computation lives in libdsgrft.so (hand-written HIP for gfx950, C ABI in
include/dsgrft.h); this package is its thin Python binding.  Importing a
GPU entry point without the built library raises ImportError.
"""
from ._lib import DsgrftError, FORMS, PEAK_DTYPE, exported_symbols  # noqa: F401


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    if name in ("DSGRFTObjective", "objective"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
