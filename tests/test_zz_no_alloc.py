"""GPU test of the allocation-free back-projection entry point (rosar_bp_full_noalloc), called
through the C ABI: it equals rosar_bp_full with a caller workspace bit for bit, on two calls in
a row, the second with fewer pulses (so the second call runs on a table the first one left
behind in the library's device array)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_common import custom_workload, dev, log, need_gpu, to_dev, torch

pytestmark = pytest.mark.gpu


def _call_pair(rs, w, x, angles):
    """The same back-projection through rosar_bp_full (workspace) and rosar_bp_full_noalloc."""
    from paper_2309_08038_amd import _lib as L
    g, grid = w.geometry, w.grid
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=0)
    ang = None if angles is None else to_dev(angles)
    ref = torch.empty((grid.n_range, grid.n_az), dtype=torch.complex64, device=dev())
    got = torch.full_like(ref, complex(float("nan"), float("nan")))
    ws = torch.empty(rs.bp_workspace_bytes(g), dtype=torch.uint8, device=dev())
    gg, pg, v = L.geometry(g), L.polar_grid(grid), rc.view()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    aptr = None if ang is None else C.c_void_p(ang.data_ptr())
    L.check(L.lib().rosar_bp_full(C.byref(gg), C.byref(pg), C.byref(v), aptr, L.NEAREST, C.c_void_p(ref.data_ptr()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), stream), "rosar_bp_full")
    L.check(L.lib().rosar_bp_full_noalloc(C.byref(gg), C.byref(pg), C.byref(v), aptr, L.NEAREST,
                                          C.c_void_p(got.data_ptr()), stream), "rosar_bp_full_noalloc")
    torch.cuda.synchronize()
    return got.cpu(), ref.cpu(), oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]


def test_bp_full_noalloc_equals_workspace_entry_point():
    rs = need_gpu()
    # first call: 720 pulses with jittered angles
    w1 = custom_workload("noalloc_a", 91, 720, 128, 12, 0.6, 3.0, 8, 16)
    x1 = synth.make_inputs(w1)
    ang1 = synth.nominal_angles(w1.geometry) + np.random.default_rng(3).normal(0, 2e-3, 720)
    log("bp_full_noalloc call 1: N=720, jittered angles")
    got1, ref1, yb1 = _call_pair(rs, w1, x1, ang1)
    assert torch.equal(got1, ref1)
    want1 = oracle.bp_full(yb1, x1.l_lo, w1.geometry, w1.grid, pulse_angles=ang1)
    assert oracle.metrics.rel_l2(got1.numpy(), want1) <= 1e-4
    # second call: fewer pulses, nominal angles; the array still holds the first call's table
    w2 = custom_workload("noalloc_b", 92, 300, 64, 5, 0.5, 1.8, 8, 16)
    x2 = synth.make_inputs(w2)
    log("bp_full_noalloc call 2: N=300, nominal angles")
    got2, ref2, yb2 = _call_pair(rs, w2, x2, None)
    assert torch.equal(got2, ref2)
    want2 = oracle.bp_full(yb2, x2.l_lo, w2.geometry, w2.grid)
    assert oracle.metrics.rel_l2(got2.numpy(), want2) <= 1e-4
