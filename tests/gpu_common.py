"""Shared helpers of the GPU parity tests (inputs on the device, oracle references)."""
from __future__ import annotations

import dataclasses
import functools
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08038_amd as rs
    rs.lib()
    return rs


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


@functools.lru_cache(maxsize=8)
def inputs(name: str):
    w = {"small": synth.small, "rotation": synth.rotation, "calib": synth.calib, "testbed": synth.testbed}[name]()
    return w, synth.make_inputs(w)


@functools.lru_cache(maxsize=8)
def oracle_band(name: str):
    w, x = inputs(name)
    y = oracle.range_compress(x.raw, x.window, w.geometry.n_fft)
    return y[:, x.l_lo:x.l_lo + x.l_count]


def custom_workload(name, cfg_id, n, m, rg, r0, r1, k, win, radius=0.25, shared=False):
    g = synth.radar(n, m, radius)
    grid = synth.PolarGrid(rg, n, r0, (r1 - r0) / max(rg - 1, 1))
    return synth.Workload(name, cfg_id, g, grid, synth.SceneSpec(5, "rayleigh", r0, r1, noise_power=1e-2),
                          synth.SparseSpec(k, win, shared))


def rel_l2(a, b):
    return oracle.metrics.rel_l2(np.asarray(a), np.asarray(b))


def assert_image(got, ref, tol, what=""):
    """Relative L2 <= tol over the image, and no pixel off by more than tol times the image's
    largest magnitude: a handful of wrong pixels (a wrong bin, a wrong pulse) fails the second
    bar even where it hides under the first."""
    got, ref = np.asarray(got), np.asarray(ref)
    e = rel_l2(got, ref)
    assert e <= tol, (what, "relative L2", e)
    scale = np.abs(ref).max()
    worst = np.abs(got - ref).max()
    assert worst <= tol * scale, (what, "largest pixel error", worst, "of max", scale,
                                  "at", np.unravel_index(np.argmax(np.abs(got - ref)), ref.shape))
