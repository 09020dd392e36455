"""FP64 CPU oracle of the imaging path (test infrastructure only; see rosar_oracle)."""
from .rosar_oracle import (beampattern, bins_per_metre, bp_cartesian_at, bp_full, robust_summary, delta_r, delta_r_samples, bp_full_at, bp_terms, bp_time_domain_at, range_compress,
                           range_compress_direct, sample, sas_time_domain_at, slant_range, sparse_filter,
                           sparse_filter_adjoint_band, sparse_filter_at, sparse_filter_cartesian, sparse_filter_grad, visible_index_range,
                           wavenumber)
from . import metrics
