"""GPU tests of the adjoint of the sparse filter with respect to the range-compressed band
(A^H g for the linear map Y -> I of Algorithm 2 / eq. 43): against the FP64 oracle adjoint at the
gradient bar (relative L2 <= 1e-3), the adjoint identity with the GPU forward filter, and
reproducibility."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import custom_workload, inputs, log, need_gpu, oracle_band, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-3


def setup(rs, w, x):
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    gimg = synth.random_complex((w.grid.n_range, w.grid.n_az), 77).astype(np.complex64)
    return rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)), gimg


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_adjoint_band_small(interp):
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts, gimg = setup(rs, w, x)
    log(f"adjoint band small {interp}")
    got = rs.sparse_filter_adjoint_band(w.geometry, w.grid, rc, off, wts, w.sparse.window, to_dev(gimg),
                                        interp=interp).cpu().numpy()
    want = oracle.sparse_filter_adjoint_band(x.l_count, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, gimg,
                                             interp=interp)
    assert got.shape == (x.l_count, w.geometry.n_pulses)
    assert rel_l2(got, want.T) <= TOL_GRAD


EDGE = [
    # name, N, M, rows, r0, r1, K, W
    ("ragged_n_k5", 100, 128, 9, 0.6, 2.5, 5, 16),
    ("k100_gt_wave", 300, 256, 6, 0.8, 4.0, 100, 128),
    ("k1", 64, 64, 3, 0.5, 1.2, 1, 2),
    ("w_equals_n", 96, 64, 4, 0.5, 1.0, 40, 96),
    ("many_rows", 128, 64, 300, 0.4, 1.4, 12, 32),
    # more than 2048 range rows: the staged form's row list takes 32-bit entries
    ("rows_over_2048", 64, 64, 2100, 0.4, 1.4, 8, 16),
    # a window of the whole rotation: one staged gradient row would not fit the LDS budget, so
    # the global-gather form runs
    ("wide_window_gather", 4096, 64, 3, 0.6, 1.0, 50, 4096),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_adjoint_band_edge_cases(case, interp):
    rs = need_gpu()
    name, n, m, rg, r0, r1, k, win = case
    w = custom_workload(name, 60 + len(name), n, m, rg, r0, r1, k, win)
    x = synth.make_inputs(w)
    rc, off, wts, gimg = setup(rs, w, x)
    log(f"adjoint band edge {name} {interp}")
    got = rs.sparse_filter_adjoint_band(w.geometry, w.grid, rc, off, wts, win, to_dev(gimg),
                                        interp=interp).cpu().numpy()
    want = oracle.sparse_filter_adjoint_band(x.l_count, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, gimg,
                                             interp=interp)
    assert rel_l2(got, want.T) <= TOL_GRAD


def test_adjoint_band_rotation_size():
    """Rotation workload (1024 x 3600, K = 64 of 256, 399 band rows): the whole gradient."""
    rs = need_gpu()
    w, x = inputs("rotation")
    rc, off, wts, gimg = setup(rs, w, x)
    log("adjoint band rotation size")
    got = rs.sparse_filter_adjoint_band(w.geometry, w.grid, rc, off, wts, w.sparse.window, to_dev(gimg))
    again = rs.sparse_filter_adjoint_band(w.geometry, w.grid, rc, off, wts, w.sparse.window, to_dev(gimg))
    torch.cuda.synchronize()
    assert torch.equal(got, again)              # fixed summation order
    want = oracle.sparse_filter_adjoint_band(x.l_count, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, gimg)
    assert rel_l2(got.cpu().numpy(), want.T) <= TOL_GRAD


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_adjoint_band_identity_with_gpu_forward(interp):
    """<g, A Y> = <A^H g, Y> with both maps evaluated on the GPU (sums in float64 on the host)."""
    rs = need_gpu()
    w, x = inputs("small")
    rc, off, wts, gimg = setup(rs, w, x)
    log(f"adjoint band identity {interp}")
    img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp).cpu().numpy()
    gy = rs.sparse_filter_adjoint_band(w.geometry, w.grid, rc, off, wts, w.sparse.window, to_dev(gimg),
                                       interp=interp).cpu().numpy().astype(np.complex128)
    band = rc.pulses(w.geometry.n_pulses).cpu().numpy().astype(np.complex128)   # [l_count, N] as read
    lhs = np.sum(np.conj(gimg.astype(np.complex128)) * img.astype(np.complex128))
    rhs = np.sum(np.conj(gy) * band)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_band_autograd(interp):
    """torch.autograd through the plain filter with respect to the band: for
    L = Re(sum conj(c) I), dL/dRe(I) + j dL/dIm(I) = c, so band.grad = A^H c (oracle)."""
    rs = need_gpu()
    w, x = inputs("small")
    yb = oracle_band("small")
    band = to_dev(yb.T.astype(np.complex64)).requires_grad_(True)        # [l_count, N]
    c = synth.random_complex((w.grid.n_range, w.grid.n_az), 78).astype(np.complex64)
    log(f"band autograd {interp}")
    img = rs.sparse_filter_band_diff(w.geometry, w.grid, band, x.l_lo, to_dev(x.offsets),
                                     to_dev(x.weights.astype(np.complex64)), w.sparse.window, interp=interp)
    ref_img = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, interp=interp)
    assert rel_l2(img.detach().cpu().numpy(), ref_img) <= 1e-4
    loss = torch.real(torch.sum(torch.conj(to_dev(c)) * img))
    loss.backward()
    want = oracle.sparse_filter_adjoint_band(x.l_count, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, c,
                                             interp=interp)
    assert rel_l2(band.grad.cpu().numpy(), want.T) <= TOL_GRAD
