"""Seeded synthetic inputs shared by the oracle and the HIP path (no imaging arithmetic here)."""
from .configs import (Geometry, PolarGrid, SceneSpec, SparseSpec, Workload, WORKLOADS, band_for,
                      bin_size_m, calib, precision, radar, rotation, scaled, small)
from .scene import (Inputs, Scene, hann, jitter_draws, make_angles, make_inputs, make_scene, make_support,
                    nominal_angles, phase_matched_weights, random_complex, rng_for, simulate_raw,
                    taylor_taper)
from .batch import batch_workloads, make_batch_inputs, scaled_batch
