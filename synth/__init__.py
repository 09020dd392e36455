"""Seeded synthetic inputs shared by the oracle and the HIP path (no imaging arithmetic here)."""
from .configs import (PAPER_SIGMA_RAD, CartLattice, Geometry, PolarGrid, SceneSpec, SparseSpec, Workload, WORKLOADS,
                      band_for, bin_size_m, calib, paper_lattice, paper_radar, precision, radar, rotation, scaled,
                      small, testbed)
from .scene import (Inputs, Scene, hann, jitter_draws, make_angles, make_inputs, make_scene, make_support,
                    nominal_angles, phase_matched_weights, random_complex, rng_for, simulate_raw,
                    taylor_taper)
from .batch import batch_workloads, make_batch_inputs, scaled_batch
