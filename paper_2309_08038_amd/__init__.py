"""MI355X (gfx950) rotating-SAR imaging: range compression, sparse-aperture azimuth filtering,
full back-projection (on range-compressed data and in the time domain) and the sparse filter's
adjoints as hand-written HIP kernels behind the C ABI of librosar.so (include/rosar.h)."""
from ._lib import RosarError, LIB_PATH, lib
from .api import (BatchPlan, RangeCompressed, Rotation, SasDesign, SparseFilterBandFn, SparseFilterFn, SparsePlan,
                  autotune_cache, autotune_lookup, autotune_store, autotune_sparse_filter, beampattern, backward_workspace_bytes, batch_autotune, bp_cartesian, bp_full, bp_time_domain,
                  bp_full_noalloc, bp_workspace_bytes, delta_r, empty_rc, range_compress, sas_design, sas_params,
                  sas_time_domain, sparse_filter,
                  sparse_filter_adjoint_band, sparse_filter_backward, sparse_filter_band_diff, sparse_filter_cartesian, sparse_filter_polar,
                  sparse_filter_diff, sparse_plan_autotune, weights_f16)

__all__ = [
    "RosarError", "LIB_PATH", "lib",
    "BatchPlan", "RangeCompressed", "Rotation", "SasDesign", "SparseFilterBandFn", "SparseFilterFn", "SparsePlan",
    "autotune_cache", "autotune_lookup", "autotune_store", "autotune_sparse_filter",
    "backward_workspace_bytes", "beampattern", "batch_autotune", "bp_cartesian", "bp_full", "bp_time_domain",
    "bp_full_noalloc", "bp_workspace_bytes", "delta_r", "empty_rc", "range_compress", "sas_design", "sas_params",
    "sas_time_domain", "sparse_filter",
    "sparse_filter_adjoint_band", "sparse_filter_backward", "sparse_filter_band_diff", "sparse_filter_cartesian", "sparse_filter_polar",
    "sparse_filter_diff",
    "sparse_plan_autotune", "weights_f16",
]
