"""GPU tests of batched rotations: persistent launches equal the single-rotation path bit for
bit (same block functions, same launch shape), agree with the FP64 oracle on sampled pixels,
and replay correctly from a captured HIP graph."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import dev, log, need_gpu, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu


def rotations(rs, ws, xs):
    out = []
    for w, x in zip(ws, xs):
        g = w.geometry
        rc = rs.empty_rc(g.n_pulses, x.l_lo, x.l_count, halo=w.sparse.window // 2, device=dev())
        img = torch.zeros((w.grid.n_range, w.grid.n_az), dtype=torch.complex64, device=dev())
        out.append(rs.Rotation(g, w.grid, to_dev(x.raw), to_dev(x.window), rc, to_dev(x.offsets),
                               to_dev(x.weights.astype(np.complex64)), w.sparse.window, img))
    return out


def single(rs, r, shape):
    rc = rs.range_compress(r.geom, r.raw, r.window, r.rc.l_lo, r.rc.l_count, halo=r.rc.halo)
    img = rs.sparse_filter(r.geom, r.grid, rc, r.offsets, r.weights, r.sparse_window, tile=(2, shape[0], shape[1]))
    return rc, img


def oracle_sampled(w, x, img, n=40, seed=0):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, w.grid.n_range, n)
    azs = rng.integers(0, w.grid.n_az, n)
    yb = oracle.range_compress(x.raw, x.window, w.geometry.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.sparse_filter_at(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, rows, azs)
    return rel_l2(img[rows, azs], ref)


@pytest.mark.parametrize("shape", [(4, 4), (8, 4), (2, 2), (1, 4), (4, 8)])
def test_batch_small_matches_single_and_oracle(shape):
    rs = need_gpu()
    ws = synth.scaled_batch(6)
    xs = [synth.make_inputs(w) for w in ws]
    rots = rotations(rs, ws, xs)
    log(f"batch small shape={shape}")
    plan = rs.BatchPlan(rots, tile=shape)
    px, rc_tiles, sf_tiles = plan.info()
    assert px == sum(w.grid.n_range * w.grid.n_az for w in ws)
    plan.run()
    torch.cuda.synchronize()
    for w, x, r in zip(ws, xs, rots):
        rc1, img1 = single(rs, r, shape)
        torch.cuda.synchronize()
        n = w.geometry.n_pulses
        assert torch.equal(r.rc.data, rc1.data), w.name
        assert torch.equal(r.image, img1), w.name
        assert oracle_sampled(w, x, r.image.cpu().numpy()) <= 1e-4, w.name
    plan.close()


def test_batch_graph_replay():
    rs = need_gpu()
    ws = synth.scaled_batch(6, seed=42)
    xs = [synth.make_inputs(w) for w in ws]
    rots = rotations(rs, ws, xs)
    plan = rs.BatchPlan(rots, tile=(4, 4))
    log("batch graph: eager reference")
    plan.run()
    torch.cuda.synchronize()
    ref = [r.image.clone() for r in rots]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.run()                        # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            plan.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        log(f"batch graph: replay {rep}")
        for r in rots:
            r.image.zero_()
            r.rc.data.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for r, e in zip(rots, ref):
            assert torch.equal(r.image, e), rep
        # eager work between replays
        plan.run()
        torch.cuda.synchronize()
    plan.close()


def test_batch_full_stream_autotuned():
    """The 64-rotation stream (uneven pulses, samples, rows and K): autotuned shape, checked
    against the single-rotation path on every rotation and against the oracle on a sample."""
    rs = need_gpu()
    ws = synth.batch_workloads(64)
    xs = synth.make_batch_inputs(ws)
    rots = rotations(rs, ws, xs)
    log("batch full: autotune")
    shape, us = rs.batch_autotune(rots, reps=2)
    log(f"batch full: best shape {shape}, {us:.1f} us")
    plan = rs.BatchPlan(rots, tile=shape)
    plan.run()
    torch.cuda.synchronize()
    for i, (w, x, r) in enumerate(zip(ws, xs, rots)):
        _, img1 = single(rs, r, shape)
        torch.cuda.synchronize()
        assert torch.equal(r.image, img1), w.name
        if i % 16 == 0:
            assert oracle_sampled(w, x, r.image.cpu().numpy(), n=20, seed=i) <= 1e-4, w.name
    plan.close()


def test_batch_autotune_refused_under_capture():
    """The batch autotuner allocates, synchronises and times: on a capturing stream it returns an
    error before touching the capture, which then ends normally and replays a batch run."""
    rs = need_gpu()
    ws = synth.scaled_batch(3, seed=7)
    xs = [synth.make_inputs(w) for w in ws]
    rots = rotations(rs, ws, xs)
    plan = rs.BatchPlan(rots, tile=(4, 4))
    plan.run()
    torch.cuda.synchronize()
    ref = [r.image.clone() for r in rots]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    log("batch autotune under capture")
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            with pytest.raises(rs.RosarError, match="capture"):
                rs.batch_autotune(rots, reps=1)
            plan.run()
    torch.cuda.current_stream().wait_stream(s)
    for r in rots:
        r.image.zero_()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    assert all(torch.equal(r.image, e) for r, e in zip(rots, ref))
