"""GPU tests of sparse-filter plans (one filter design, tap tables built once per range row):
a plan's run equals rosar_sparse_filter_tiled with the same launch shape bit for bit, for every
planned shape, both interpolations and all storage types; it follows the oracle; it is reusable
across rotations and replays correctly from a captured HIP graph."""
import json

import numpy as np
import pytest

import oracle
import synth
from gpu_common import custom_workload, inputs, log, need_gpu, oracle_band, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu

TOL = 1e-4
PLAN_SHAPES = [(4, 8), (8, 4), (4, 4), (2, 8), (2, 4), (8, 2)]


def upload(rs, w, x, dtype="c64", scale=1.0):
    g = w.geometry
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2,
                           dtype=dtype, scale=scale)
    return rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_plan_shapes_bit_identical_to_single_call(interp):
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    ref = oracle.sparse_filter(oracle_band("small"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                               interp=interp)
    for shape in PLAN_SHAPES + [None]:
        log(f"plan small shape={shape} interp={interp}")
        plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp, tile=shape)
        img = plan.run(rc).cpu()
        t = (2,) + (shape if shape is not None else (2, 4))
        single = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp, tile=t).cpu()
        assert torch.equal(img, single), shape
        assert rel_l2(img.numpy(), ref) <= TOL, shape
        plan.close()


def test_plan_reused_across_rotations():
    """One plan, two rotations' data: the second image is the first rotated by one azimuth bin."""
    rs = need_gpu()
    w, x = inputs("small")
    rc0, off, wts = upload(rs, w, x)
    x1 = synth.Inputs(**{**x.__dict__, "raw": np.roll(x.raw, 1, axis=0)})
    rc1, _, _ = upload(rs, w, x1)
    log("plan reused across rotations")
    plan = rs.SparsePlan(w.geometry, w.grid, rc0, off, wts, w.sparse.window)
    i0 = plan.run(rc0).cpu()
    out = torch.empty_like(i0, device=rc1.data.device)
    i1 = plan.run(rc1, out=out).cpu()
    assert torch.equal(i1, torch.roll(i0, 1, dims=1))
    plan.close()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_plan_reduced_precision(dtype):
    rs = need_gpu()
    w, x = inputs("small")
    scale = 2.0 ** -4 if dtype == "f16" else 1.0
    rc, off, wts = upload(rs, w, x, dtype=dtype, scale=scale)
    ref = oracle.sparse_filter(oracle_band("small"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights)
    for shape in ((8, 4), (4, 4), (8, 2)):
        for wt in (wts, rs.weights_f16(wts)):
            log(f"plan {dtype} shape={shape} weights={wt.dtype}")
            plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wt, w.sparse.window, tile=shape)
            img = plan.run(rc).cpu()
            single = rs.sparse_filter(w.geometry, w.grid, rc, off, wt, w.sparse.window, tile=(2,) + shape).cpu()
            assert torch.equal(img, single), (shape, wt.dtype)
            assert rel_l2(img.numpy(), ref) <= 1e-2, (shape, wt.dtype)
            plan.close()


EDGE = [
    # name, N, M, rows, r0, r1, K, W
    ("ragged_n_k5", 100, 128, 9, 0.6, 2.5, 5, 16),
    ("k100_gt_wave", 300, 256, 6, 0.8, 4.0, 100, 128),
    ("k1", 64, 64, 3, 0.5, 1.2, 1, 2),
    ("w_equals_n", 96, 64, 4, 0.5, 1.0, 40, 96),
    ("many_rows", 128, 64, 300, 0.4, 1.4, 12, 32),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_plan_edge_cases(case, interp):
    rs = need_gpu()
    name, n, m, rg, r0, r1, k, win = case
    w = custom_workload(name, 60 + len(name), n, m, rg, r0, r1, k, win)
    x = synth.make_inputs(w)
    log(f"plan edge {name} interp={interp}")
    yb = oracle.range_compress(x.raw, x.window, m)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, interp=interp)
    rc, off, wts = upload(rs, w, x)
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, win, interp=interp)
    img = plan.run(rc).cpu()
    single = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, win, interp=interp, tile=(2, 2, 4)).cpu()
    assert torch.equal(img, single)
    assert rel_l2(img.numpy(), ref) <= TOL
    plan.close()


def test_plan_rotation_size():
    """Rotation workload (1024 x 3600, K = 64 of 256): bit-identical to the default single call,
    oracle parity on sampled pixels."""
    rs = need_gpu()
    w, x = inputs("rotation")
    rc, off, wts = upload(rs, w, x)
    log("plan rotation size")
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window)
    img = plan.run(rc).cpu()
    single = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window).cpu()
    assert torch.equal(img, single)
    rng = np.random.default_rng(7)
    rows = rng.integers(0, w.grid.n_range, 300)
    azs = rng.integers(0, w.grid.n_az, 300)
    ref = oracle.sparse_filter_at(oracle_band("rotation"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                                  rows, azs)
    assert rel_l2(img.numpy()[rows, azs], ref) <= TOL
    plan.close()


@pytest.mark.parametrize("dtype", ["c64", "bf16"])
def test_plan_autotune(dtype):
    """The autotuner returns a plan shape; a plan of that shape equals the single call."""
    rs = need_gpu()
    w, x = inputs("rotation")
    rc, off, wts = upload(rs, w, x, dtype=dtype)
    log(f"plan autotune {dtype}")
    shape, us = rs.sparse_plan_autotune(w.geometry, w.grid, rc, off, wts, w.sparse.window, reps=3)
    log(f"plan autotune {dtype}: {shape} {us:.1f} us")
    assert (shape in PLAN_SHAPES or shape == "fastconv") and 0.0 < us < 1e5
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, tile=shape)
    img = plan.run(rc).cpu()
    if shape == "fastconv":
        single = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window).cpu()
        assert rel_l2(img.numpy(), single.numpy()) <= 1e-5
    else:
        single = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, tile=(2,) + shape).cpu()
        assert torch.equal(img, single)
    plan.close()


def test_plan_autotune_cache(tmp_path):
    """With a cache file the first autotune stores its result under the GPU's architecture and
    shape class (in the library, which writes the file); an entry found there is returned
    without timing (an edited entry comes back, also after the file is reloaded)."""
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    path = str(tmp_path / "tune.json")
    log("plan autotune cache")
    try:
        first = rs.sparse_plan_autotune(w.geometry, w.grid, rc, off, wts, w.sparse.window, reps=2, cache=path)
        d = json.loads(open(path).read())
        (key, entry), = d.items()
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        assert key.startswith(arch + "|plan|"), key
        tile = "fastconv" if entry["variant"] == 3 else (entry["pixels_per_lane"], entry["waves"])
        assert (tile, pytest.approx(entry["us"], rel=1e-6)) == first
        d[key] = {"variant": 2, "pixels_per_lane": 2, "waves": 4, "us": 1.25}
        open(path, "w").write(json.dumps(d))
        rs.autotune_cache(path)     # reload the edited file
        assert rs.sparse_plan_autotune(w.geometry, w.grid, rc, off, wts, w.sparse.window, reps=2) == ((2, 4), 1.25)
        # the single-call autotuner caches under its own key
        t1 = rs.autotune_sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, reps=2)
        keys = json.loads(open(path).read()).keys()
        assert len(keys) == 2 and any("|single|" in k for k in keys)
        assert rs.autotune_sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, reps=2) == t1
    finally:
        rs.autotune_cache(None)


def test_plan_layout_mismatch_rejected():
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window)
    other = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count,
                              halo=w.sparse.window // 2 + 2)
    log("plan layout mismatch")
    with pytest.raises(rs.RosarError) as ei:
        plan.run(other)
    assert "layout" in str(ei.value)
    plan.close()


def test_plan_graph_replay():
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, tile=(4, 4))
    log("plan graph: eager reference")
    img = plan.run(rc)
    torch.cuda.synchronize()
    ref = img.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.run(rc, out=img)             # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            plan.run(rc, out=img)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        log(f"plan graph: replay {rep}")
        img.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, ref), rep
        plan.run(rc, out=img)             # eager work between replays
        torch.cuda.synchronize()
    plan.close()


# ------------------------------------------------------------------ azimuth fast convolution
# Same sum as the direct filter, evaluated with FFTs along azimuth: equal to the oracle within
# the float32 bar (1e-4 relative L2), and to the direct filter within 1e-5.

@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_fastconv_small(interp):
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    ref = oracle.sparse_filter(oracle_band("small"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                               interp=interp)
    log(f"fastconv small interp={interp}")
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp, tile="fastconv")
    img = plan.run(rc).cpu().numpy()
    assert rel_l2(img, ref) <= TOL
    direct = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp).cpu().numpy()
    assert rel_l2(img, direct) <= 1e-5
    plan.close()


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_fastconv_edge_cases(case, interp):
    rs = need_gpu()
    name, n, m, rg, r0, r1, k, win = case
    w = custom_workload(name, 60 + len(name), n, m, rg, r0, r1, k, win)
    x = synth.make_inputs(w)
    log(f"fastconv edge {name} interp={interp}")
    yb = oracle.range_compress(x.raw, x.window, m)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, interp=interp)
    rc, off, wts = upload(rs, w, x)
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, win, interp=interp, tile="fastconv")
    img = plan.run(rc).cpu().numpy()
    assert rel_l2(img, ref) <= TOL
    plan.close()


def test_fastconv_rotation_size():
    """Rotation workload (N = 3600 = 2^4 3^2 5^2): oracle parity on sampled pixels and the whole
    image against the direct filter."""
    rs = need_gpu()
    w, x = inputs("rotation")
    rc, off, wts = upload(rs, w, x)
    log("fastconv rotation size")
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, tile="fastconv")
    img = plan.run(rc).cpu().numpy()
    direct = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window).cpu().numpy()
    assert rel_l2(img, direct) <= 1e-5
    rng = np.random.default_rng(11)
    rows = rng.integers(0, w.grid.n_range, 300)
    azs = rng.integers(0, w.grid.n_az, 300)
    ref = oracle.sparse_filter_at(oracle_band("rotation"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                                  rows, azs)
    assert rel_l2(img[rows, azs], ref) <= TOL
    plan.close()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_fastconv_reduced_precision(dtype):
    rs = need_gpu()
    w, x = inputs("small")
    scale = 2.0 ** -4 if dtype == "f16" else 1.0
    rc, off, wts = upload(rs, w, x, dtype=dtype, scale=scale)
    ref = oracle.sparse_filter(oracle_band("small"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights)
    for wt in (wts, rs.weights_f16(wts)):
        log(f"fastconv {dtype} weights={wt.dtype}")
        plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wt, w.sparse.window, tile="fastconv")
        img = plan.run(rc).cpu().numpy()
        assert rel_l2(img, ref) <= 1e-2, wt.dtype
        # the direct 16-bit path also rounds the weights to the storage type (v_dot2 operands);
        # the fast convolution applies them in float32, so it is at least as close to the oracle
        direct = rs.sparse_filter(w.geometry, w.grid, rc, off, wt, w.sparse.window).cpu().numpy()
        assert rel_l2(img, ref) <= rel_l2(direct, ref) + 1e-5, wt.dtype
        plan.close()


def test_fastconv_graph_replay():
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, tile="fastconv")
    log("fastconv graph: eager reference")
    img = plan.run(rc)
    torch.cuda.synchronize()
    ref = img.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.run(rc, out=img)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            plan.run(rc, out=img)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        log(f"fastconv graph: replay {rep}")
        img.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, ref), rep
        plan.run(rc, out=img)
        torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_fastconv_parallel_runs_own_workspaces(interp):
    """Rotation size: two runs of one fast-convolution plan on two different rotations, captured
    on two streams as parallel branches of one graph, each with its own spectrum workspace: every
    replay equals the eager images bit for bit (the runs share only what a run reads)."""
    rs = need_gpu()
    w, x = inputs("rotation")
    rc1, off, wts = upload(rs, w, x)
    x2 = synth.Inputs(**{**x.__dict__, "raw": np.roll(x.raw, 7, axis=0) * np.complex64(0.5 - 0.25j)})
    rc2, _, _ = upload(rs, w, x2)
    plan = rs.SparsePlan(w.geometry, w.grid, rc1, off, wts, w.sparse.window, interp=interp, tile="fastconv")
    nbytes = plan.workspace_bytes()
    assert nbytes == x.l_count * w.geometry.n_pulses * 8
    ws = [torch.empty(nbytes, dtype=torch.uint8, device=rc1.data.device) for _ in range(2)]
    log(f"fastconv parallel runs {interp}: eager references")
    ref1, ref2 = plan.run(rc1), plan.run(rc2)
    torch.cuda.synchronize()
    ref1, ref2 = ref1.clone(), ref2.clone()
    assert not torch.equal(ref1, ref2)
    img1, img2 = torch.empty_like(ref1), torch.empty_like(ref2)
    s, sa, sb = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            sa.wait_stream(s)
            sb.wait_stream(s)
            with torch.cuda.stream(sa):
                plan.run(rc1, out=img1, workspace=ws[0])
            with torch.cuda.stream(sb):
                plan.run(rc2, out=img2, workspace=ws[1])
            s.wait_stream(sa)
            s.wait_stream(sb)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        log(f"fastconv parallel runs {interp}: replay {rep}")
        img1.zero_()
        img2.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img1, ref1), ("first branch", rep)
        assert torch.equal(img2, ref2), ("second branch", rep)
        plan.run(rc2, out=img1)          # eager work between replays, on the plan's own buffer
        torch.cuda.synchronize()
    plan.close()


def test_fastconv_plan_builds_identical():
    """Two builds of the same fast-convolution plan give the same image bits (the kernel spectra
    are accumulated in a fixed order)."""
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    imgs = []
    for i in range(2):
        log(f"fastconv plan build {i}")
        plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp="linear", tile="fastconv")
        imgs.append(plan.run(rc).cpu())
        plan.close()
    assert torch.equal(imgs[0], imgs[1])


@pytest.mark.parametrize("variant", ["fastconv-nearest", "fastconv-linear", "direct-linear", "direct-nearest"])
def test_plan_runs_deterministic(variant):
    """Rotation size: repeated eager runs and graph replays of one plan give identical bits."""
    rs = need_gpu()
    w, x = inputs("rotation")
    rc, off, wts = upload(rs, w, x)
    method, interp = variant.split("-")
    tile = "fastconv" if method == "fastconv" else (4, 4)
    plan = rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp, tile=tile)
    log(f"plan determinism {variant}: eager runs")
    img = plan.run(rc)
    torch.cuda.synchronize()
    ref = img.clone()
    for i in range(5):
        plan.run(rc, out=img)
        torch.cuda.synchronize()
        assert torch.equal(img, ref), ("eager", i)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            for _ in range(4):
                plan.run(rc, out=img)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        log(f"plan determinism {variant}: replay {rep}")
        img.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, ref), ("replay", rep)
    plan.close()


def test_plan_create_refused_under_capture():
    """Plan creation and the plan autotuner allocate and synchronise: on a capturing stream they
    return an error before touching the capture, which stays valid; a capturable call in the
    same capture replays to the eager result."""
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts = upload(rs, w, x)
    eager = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window)
    torch.cuda.synchronize()
    img = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    log("plan create under capture")
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            with pytest.raises(rs.RosarError, match="capture"):
                rs.SparsePlan(w.geometry, w.grid, rc, off, wts, w.sparse.window)
            with pytest.raises(rs.RosarError, match="capture"):
                rs.sparse_plan_autotune(w.geometry, w.grid, rc, off, wts, w.sparse.window, reps=1)
            rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, out=img)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(2):
        img.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, eager)
