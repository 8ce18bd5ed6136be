"""Sliced co-execution engine for MI355X (gfx950): the hot path of Kernelet
(Zhong & He) -- slicer, occupancy control, Markov-chain performance model,
PUR/MUR pruning and greedy pair scheduling -- in libkernelet.so, with eight
hand-written HIP workload kernels.  This package is the thin Python face of
that library (see include/kernelet.h)."""
from ._lib import KerneletError, lib  # noqa: F401
from .runtime import (Runtime, best_ratio, builtin_desc, builtin_grid,  # noqa: F401
                      default_config, make_profile, predict, predict_group,
                      profile_from_counters, simulate)
