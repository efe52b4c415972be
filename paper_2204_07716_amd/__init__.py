"""MI355X-native fast multivariate kernel regression (type-1 NUFFT moments,
FP64 local-polynomial solves, Monte-Carlo DF, GCV, conditional variance).

The compute path is the HIP library ``libfkr.so`` (C ABI in include/fkr.h);
this package is its thin Python binding.  Importing it does not load the
library; the first ``Plan`` does, and fails loudly if it was not built.
"""
from .fkreg import Batch, GCVFullH, GCVLogH, Plan, get_hlist, select_bandwidth  # noqa: F401

__all__ = ["Batch", "GCVFullH", "GCVLogH", "Plan", "get_hlist", "select_bandwidth"]
