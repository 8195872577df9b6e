"""HJ-Gauss Monte-Carlo Picard sweep on AMD Instinct MI355X (gfx950).

The work runs in libhjg.so (HIP kernels behind the C interface of
include/hjg.h); this package is its thin Python binding.
"""
from .api import (BatchOut, Context, PicardOut, ProblemSpec, Surrogate, TrainConfig, autotune_batched, avoid_project,  # noqa: F401
                  autotune_sweep, certify, error_budget, isocontour, knn_grid, mc_margin, philox_words, picard_sweep, picard_sweep_batched, probe_valu_rate, sample_table, smooth_slices, surrogate_sweep,
                  surrogate_tube_step, topology, topology_events, value_grad, value_grad_noalloc)

__all__ = ["Context", "ProblemSpec", "PicardOut", "philox_words", "sample_table", "value_grad", "value_grad_noalloc",
           "picard_sweep",
           "Surrogate", "TrainConfig", "surrogate_sweep", "picard_sweep_batched", "BatchOut", "autotune_sweep",
           "autotune_batched", "knn_grid", "surrogate_tube_step", "certify", "mc_margin", "error_budget", "topology",
           "topology_events", "isocontour", "smooth_slices", "avoid_project", "probe_valu_rate"]
