"""C-ABI checks that need no GPU: exported symbols, struct layouts, argument validation.

Every call here fails validation (or hits the fault-injection hook) before any device work,
so nothing is launched."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rosar.h")

rs = pytest.importorskip("paper_2309_08038_amd")
from paper_2309_08038_amd import _lib as L  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("librosar.so not built")
    return L.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rosar_[a-z_0-9]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(n for n, _, _ in L.PROTOTYPES)


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\s[TW]\s(rosar_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_struct_layouts_match_c(tmp_path):
    """sizeof/offsetof of the C structs (gcc on the public header) equal the ctypes mirrors."""
    structs = {"rosar_geometry": L.Geometry, "rosar_polar_grid": L.PolarGrid, "rosar_rc_view": L.RcView,
               "rosar_sparse_set": L.SparseSet, "rosar_tile": L.Tile, "rosar_rotation_desc": L.RotationDesc,
               "rosar_cart_grid": L.CartGrid}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(c), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"


def geom(**kw):
    d = dict(n_pulses=360, n_fast=256, n_fft=256, reserved=0, radius_m=0.25, fc_hz=77e9, slope_hz_s=1.5625e14,
             fs_hz=1e7, t_start_s=0.0, c_m_s=299792458.0, phi0_rad=0.0)
    d.update(kw)
    return L.Geometry(**d)


FAKE = C.c_void_p(0x10000)      # aligned, never dereferenced (validation fails before use)


def rc_call(lib, g, **kw):
    a = dict(raw=FAKE, window=None, l_lo=0, l_count=16, halo=0, dt=L.C64, scale=1.0, out=FAKE, ld=360)
    a.update(kw)
    return lib.rosar_range_compress(C.byref(g) if g is not None else None, a["raw"], a["window"], a["l_lo"],
                                    a["l_count"], a["halo"], a["dt"], a["scale"], a["out"], a["ld"], None)


@pytest.mark.parametrize("kw,status", [
    (dict(n_pulses=1), L.ROSAR_ERR_INVALID_ARG),
    (dict(n_fft=98, n_fast=98), L.ROSAR_ERR_UNSUPPORTED),      # 2 x 7^2: no mixed-radix path
    (dict(n_fft=9000, n_fast=9000), L.ROSAR_ERR_UNSUPPORTED),  # over the 8192-point workgroup FFT
    (dict(n_fft=128, n_fast=256), L.ROSAR_ERR_INVALID_ARG),
    (dict(radius_m=float("nan")), L.ROSAR_ERR_INVALID_ARG),
    (dict(radius_m=-1.0), L.ROSAR_ERR_INVALID_ARG),
    (dict(slope_hz_s=0.0), L.ROSAR_ERR_INVALID_ARG),
    (dict(fs_hz=float("inf")), L.ROSAR_ERR_INVALID_ARG),
    (dict(c_m_s=0.0), L.ROSAR_ERR_INVALID_ARG),
    (dict(reserved=1), L.ROSAR_ERR_INVALID_ARG),
])
def test_range_compress_geometry_validation(lib, kw, status):
    assert rc_call(lib, geom(**kw)) == status
    assert lib.rosar_last_error().decode()


@pytest.mark.parametrize("kw,status", [
    (dict(raw=None), L.ROSAR_ERR_INVALID_ARG),
    (dict(raw=C.c_void_p(0x10004)), L.ROSAR_ERR_INVALID_ARG),
    (dict(out=None), L.ROSAR_ERR_INVALID_ARG),
    (dict(window=C.c_void_p(0x10002)), L.ROSAR_ERR_INVALID_ARG),
    (dict(l_lo=-1), L.ROSAR_ERR_INVALID_ARG),
    (dict(l_count=0), L.ROSAR_ERR_INVALID_ARG),
    (dict(l_lo=250, l_count=16), L.ROSAR_ERR_INVALID_ARG),
    (dict(halo=-1), L.ROSAR_ERR_INVALID_ARG),
    (dict(halo=10, ld=370), L.ROSAR_ERR_INVALID_ARG),
    (dict(ld=359), L.ROSAR_ERR_INVALID_ARG),
    (dict(dt=7), L.ROSAR_ERR_INVALID_ARG),
    (dict(scale=0.0), L.ROSAR_ERR_INVALID_ARG),
    (dict(scale=float("nan")), L.ROSAR_ERR_INVALID_ARG),
])
def test_range_compress_argument_validation(lib, kw, status):
    assert rc_call(lib, geom(), **kw) == status
    assert rc_call(lib, None) == L.ROSAR_ERR_INVALID_ARG


def sf_call(lib, g=None, grid=None, view=None, sset=None, interp=L.NEAREST, image=FAKE, dphi=None):
    g = g or geom()
    grid = grid or L.PolarGrid(8, 360, 1.0, 0.05)
    view = view or L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = sset or L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    return lib.rosar_sparse_filter(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset), dphi, None, interp,
                                   image, None)


@pytest.mark.parametrize("field,value,status", [
    ("grid.n_az", 180, L.ROSAR_ERR_UNSUPPORTED),
    ("grid.n_range", 0, L.ROSAR_ERR_INVALID_ARG),
    ("grid.r0_m", 0.0, L.ROSAR_ERR_INVALID_ARG),
    ("grid.dr_m", -0.1, L.ROSAR_ERR_INVALID_ARG),
    ("view.data", None, L.ROSAR_ERR_INVALID_ARG),
    ("view.dtype", 5, L.ROSAR_ERR_INVALID_ARG),
    ("view.ld", 400, L.ROSAR_ERR_INVALID_ARG),
    ("view.scale", -1.0, L.ROSAR_ERR_INVALID_ARG),
    ("view.l_count", 300, L.ROSAR_ERR_INVALID_ARG),
    ("view.reserved", 3, L.ROSAR_ERR_INVALID_ARG),
    ("set.k", 0, L.ROSAR_ERR_INVALID_ARG),
    ("set.k", 2000, L.ROSAR_ERR_INVALID_ARG),
    ("set.k", 65, L.ROSAR_ERR_INVALID_ARG),           # k > window
    ("set.window", 63, L.ROSAR_ERR_INVALID_ARG),      # odd
    ("set.window", 400, L.ROSAR_ERR_INVALID_ARG),     # > N
    ("set.offsets", None, L.ROSAR_ERR_INVALID_ARG),
    ("set.weights", 0x40004, L.ROSAR_ERR_INVALID_ARG),  # misaligned c64
    ("set.w_dtype", L.C16_BF16, L.ROSAR_ERR_INVALID_ARG),
])
def test_sparse_filter_validation(lib, field, value, status):
    g = geom()
    grid = L.PolarGrid(8, 360, 1.0, 0.05)
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    obj, name = field.split(".")
    setattr({"grid": grid, "view": view, "set": sset}[obj], name, value)
    assert sf_call(lib, g, grid, view, sset) == status
    assert lib.rosar_last_error().decode() != ""     # every rejection says why


def test_sparse_filter_other_validation(lib):
    assert sf_call(lib, interp=7) == L.ROSAR_ERR_INVALID_ARG
    assert sf_call(lib, image=None) == L.ROSAR_ERR_INVALID_ARG
    assert sf_call(lib, image=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert sf_call(lib, dphi=C.c_void_p(0x10002)) == L.ROSAR_ERR_INVALID_ARG
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    # unsupported launch shapes: 3 pixels per lane, variants outside 0..2, 8 x 8
    for t in (L.Tile(1, 3, 4, 0), L.Tile(3, 4, 4, 0), L.Tile(-1, 4, 4, 0), L.Tile(2, 8, 8, 0)):
        assert lib.rosar_sparse_filter_tiled(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset), None, None,
                                             L.NEAREST, FAKE, C.byref(t), None) == L.ROSAR_ERR_UNSUPPORTED, \
            (t.variant, t.pixels_per_lane, t.waves)


def test_bp_and_backward_workspace_checks(lib):
    g = geom()
    n = C.c_size_t(0)
    assert lib.rosar_bp_full_workspace_size(C.byref(g), C.byref(n)) == L.ROSAR_OK
    assert n.value >= 256 + 360 * 8   # header + (sin, cos) of half the angle error per pulse, float32
    grid = L.PolarGrid(8, 360, 1.0, 0.05)
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    # NULL / misaligned / short workspace
    for ws, nb in [(None, n.value), (C.c_void_p(0x10010), n.value), (FAKE, n.value - 1)]:
        assert lib.rosar_bp_full(C.byref(g), C.byref(grid), C.byref(view), None, L.NEAREST, FAKE, ws, nb,
                                 None) == L.ROSAR_ERR_WORKSPACE
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    m = C.c_size_t(0)
    assert lib.rosar_sparse_filter_backward_workspace_size(C.byref(g), C.byref(grid), C.byref(sset),
                                                           C.byref(m)) == L.ROSAR_OK
    assert m.value >= 2 * 8 * 360 * 4
    assert lib.rosar_sparse_filter_backward(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset), None, None,
                                            L.LINEAR, FAKE, FAKE, None, None, FAKE, m.value - 4,
                                            None) == L.ROSAR_ERR_WORKSPACE
    sset16 = L.SparseSet(32, 64, 0x30000, 0x40000, L.C16_F16, 0)
    assert lib.rosar_sparse_filter_backward(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset16), None,
                                            None, L.LINEAR, FAKE, FAKE, None, None, FAKE, m.value,
                                            None) == L.ROSAR_ERR_UNSUPPORTED


def test_status_strings(lib):
    for s in range(6):
        assert lib.rosar_status_str(s).decode().startswith("ROSAR_")
    assert lib.rosar_version().decode().startswith("rosar")


def test_fault_injection_propagates_to_python(lib, monkeypatch):
    """A launch failure reported by the library surfaces as RosarError with the message."""
    monkeypatch.setenv("ROSAR_FAULT_INJECT", "launch")
    assert rc_call(lib, geom()) == L.ROSAR_ERR_HIP
    assert "injected" in lib.rosar_last_error().decode()
    with pytest.raises(L.RosarError) as ei:
        L.check(rc_call(lib, geom()), "rosar_range_compress")
    assert ei.value.status == L.ROSAR_ERR_HIP and "injected" in str(ei.value)
    monkeypatch.delenv("ROSAR_FAULT_INJECT")


def test_python_front_end_rejects_cpu_tensors():
    import torch
    import synth
    w = synth.small()
    with pytest.raises(ValueError):
        rs.range_compress(w.geometry, torch.zeros((360, 256), dtype=torch.complex64), None, 0, 16)


def test_torch_complex_gradient_convention():
    """torch's .grad of a complex leaf is dL/dRe + j dL/dIm, the convention of the adjoint."""
    import torch
    z = torch.tensor([1.0 + 2.0j, -0.5 + 0.25j], dtype=torch.complex128, requires_grad=True)
    loss = (z.abs() ** 2).sum() + (3.0 * z.real - 2.0 * z.imag).sum()
    loss.backward()
    ref = 2 * z.detach() + (3.0 - 2.0j)
    assert torch.allclose(z.grad, ref)


def plan_create(lib, g=None, grid=None, view=None, sset=None, interp=L.NEAREST, tile=None, out=True):
    g = g or geom()
    grid = grid or L.PolarGrid(8, 360, 1.0, 0.05)
    view = view or L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = sset or L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    h = C.c_void_p(0x1234)
    st = lib.rosar_sparse_plan_create(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset), interp,
                                      C.byref(tile) if tile is not None else None, None,
                                      C.byref(h) if out else None)
    return st, h


def test_sparse_plan_validation(lib):
    st, _ = plan_create(lib, out=False)
    assert st == L.ROSAR_ERR_INVALID_ARG
    # the single-call checks apply unchanged (here: k > window), and *out is cleared on failure
    st, h = plan_create(lib, sset=L.SparseSet(65, 64, 0x30000, 0x40000, L.C64, 0))
    assert st == L.ROSAR_ERR_INVALID_ARG and h.value is None
    # band data must be 16-byte aligned for the direct-to-LDS staging
    st, _ = plan_create(lib, view=L.RcView(0x20008, L.C64, 0, 64, 32, 424, 1.0, 0))
    assert st == L.ROSAR_ERR_INVALID_ARG and "16-byte" in lib.rosar_last_error().decode()
    # a plan runs the staged kernel only: variant 1 and shapes outside the instantiated set are refused
    for t in (L.Tile(1, 4, 8, 0), L.Tile(2, 1, 1, 0), L.Tile(2, 8, 8, 0), L.Tile(2, 3, 4, 0)):
        st, _ = plan_create(lib, tile=t)
        assert st == L.ROSAR_ERR_UNSUPPORTED, (t.variant, t.pixels_per_lane, t.waves)
        assert lib.rosar_last_error().decode() != ""
    # halo below W/2: the staged kernel would need the guard loop for every edge column
    st, _ = plan_create(lib, view=L.RcView(0x20000, L.C64, 0, 64, 16, 392, 1.0, 0))
    assert st == L.ROSAR_ERR_UNSUPPORTED and "halo" in lib.rosar_last_error().decode()
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    assert lib.rosar_sparse_plan_run(None, C.byref(view), FAKE, None) == L.ROSAR_ERR_INVALID_ARG
    lib.rosar_sparse_plan_destroy(None)   # no-op


def test_sparse_plan_autotune_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    best, us = L.Tile(), C.c_float(0)

    def call(view=None, reps=5, b=True, u=True, image=FAKE, variants=0):
        view = view or L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
        return lib.rosar_sparse_plan_autotune(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset), L.NEAREST,
                                              image, variants, reps, C.byref(best) if b else None,
                                              C.byref(us) if u else None, None)

    assert call(b=False) == L.ROSAR_ERR_INVALID_ARG
    assert call(u=False) == L.ROSAR_ERR_INVALID_ARG
    assert call(reps=0) == L.ROSAR_ERR_INVALID_ARG
    assert call(reps=10001) == L.ROSAR_ERR_INVALID_ARG
    assert call(image=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(view=L.RcView(0x20008, L.C64, 0, 64, 32, 424, 1.0, 0)) == L.ROSAR_ERR_INVALID_ARG
    assert call(variants=4) == L.ROSAR_ERR_INVALID_ARG
    # halo < W/2 rules out the direct shapes; the fast convolution (N = 360) is still a candidate
    # unless excluded
    assert call(view=L.RcView(0x20000, L.C64, 0, 64, 16, 392, 1.0, 0), variants=L.PLAN_DIRECT) == \
        L.ROSAR_ERR_UNSUPPORTED
    assert lib.rosar_last_error().decode() != ""


def test_fastconv_plan_rejections(lib):
    """The azimuth fast convolution needs N = 2^a 3^b 5^c <= 8192 (checked before any device work)."""
    for n in (98, 9000, 7 * 64):
        g = geom(n_pulses=n)
        grid = L.PolarGrid(8, n, 1.0, 0.05)
        view = L.RcView(0x20000, L.C64, 0, 64, 32, n + 64, 1.0, 0)
        st, _ = plan_create(lib, g=g, grid=grid, view=view, tile=L.Tile(3, 0, 0, 0))
        assert st == L.ROSAR_ERR_UNSUPPORTED, n
        assert "2^a 3^b 5^c" in lib.rosar_last_error().decode()


def test_adjoint_band_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)
    n = C.c_size_t(0)
    assert lib.rosar_sparse_filter_adjoint_band_workspace_size(C.byref(g), C.byref(grid), C.byref(view),
                                                               C.byref(sset), L.NEAREST, C.byref(n)) == L.ROSAR_OK
    assert n.value >= 8 * (16 + 32 * 16)      # one tap list per range row
    m = C.c_size_t(0)
    assert lib.rosar_sparse_filter_adjoint_band_workspace_size(C.byref(g), C.byref(grid), C.byref(view),
                                                               C.byref(sset), L.LINEAR, C.byref(m)) == L.ROSAR_OK
    assert m.value > n.value                  # LINEAR taps touch two bins
    assert lib.rosar_sparse_filter_adjoint_band_workspace_size(C.byref(g), C.byref(grid), C.byref(view),
                                                               C.byref(sset), L.NEAREST, None) == L.ROSAR_ERR_INVALID_ARG

    def call(gimg=FAKE, gband=FAKE, ws=FAKE, nb=None, interp=L.NEAREST):
        return lib.rosar_sparse_filter_adjoint_band(C.byref(g), C.byref(grid), C.byref(view), C.byref(sset), interp,
                                                    gimg, gband, ws, n.value if nb is None else nb, None)

    assert call(gimg=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(gband=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(gband=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(interp=9) == L.ROSAR_ERR_INVALID_ARG
    for ws, nb in [(None, n.value), (C.c_void_p(0x10010), n.value), (FAKE, n.value - 1)]:
        assert call(ws=ws, nb=nb) == L.ROSAR_ERR_WORKSPACE
        assert lib.rosar_last_error().decode() != ""


def test_bp_time_domain_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)

    def call(raw=FAKE, window=None, angles=None, first=0, count=8, image=FAKE, gg=None):
        return lib.rosar_bp_time_domain(C.byref(gg or g), C.byref(grid), raw, window, angles, first, count, image,
                                        None)

    assert call(raw=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(raw=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(window=C.c_void_p(0x10002)) == L.ROSAR_ERR_INVALID_ARG
    assert call(angles=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    for first, count in ((-1, 2), (0, 0), (5, 4), (8, 1)):
        assert call(first=first, count=count) == L.ROSAR_ERR_INVALID_ARG, (first, count)
    assert call(image=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(gg=geom(n_fast=4096, n_fft=4096)) == L.ROSAR_ERR_UNSUPPORTED
    assert lib.rosar_last_error().decode() != ""


def test_delta_r_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)

    def call(window=64, deltas=FAKE, n_s=100, q=0.99, samples=FAKE, out=FAKE, gr=None):
        return lib.rosar_delta_r(C.byref(g), C.byref(gr or grid), window, deltas, n_s, q, samples, out, None)

    for window in (0, 1, 63, 362):
        assert call(window=window) == L.ROSAR_ERR_INVALID_ARG, window
    for n_s in (0, -1, (1 << 24) + 1):
        assert call(n_s=n_s) == L.ROSAR_ERR_INVALID_ARG, n_s
    for q in (0.0, -0.5, 1.0000001, float("nan"), float("inf")):
        assert call(q=q) == L.ROSAR_ERR_INVALID_ARG, q
    assert call(deltas=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(deltas=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(samples=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(out=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(gr=L.PolarGrid(600000, 360, 1.0, 0.05)) == L.ROSAR_ERR_UNSUPPORTED
    assert "n_range" in lib.rosar_last_error().decode()


def test_sas_time_domain_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)

    def call(raw=FAKE, first=0, count=8, image=FAKE, s=None, gg=None):
        return lib.rosar_sas_time_domain(C.byref(gg or g), C.byref(grid), raw, None, C.byref(s or sset), first,
                                         count, image, None)

    assert call(raw=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(first=7, count=2) == L.ROSAR_ERR_INVALID_ARG
    assert call(image=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(s=L.SparseSet(65, 64, 0x30000, 0x40000, L.C64, 0)) == L.ROSAR_ERR_INVALID_ARG
    assert call(s=L.SparseSet(32, 64, 0x30000, 0x40000, L.C16_F16, 0)) == L.ROSAR_ERR_UNSUPPORTED
    assert call(gg=geom(n_fast=4096, n_fft=4096)) == L.ROSAR_ERR_UNSUPPORTED


def test_beampattern_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)

    def call(s=None, angles=FAKE, n=100, dr=None, pattern=FAKE, summary=FAKE, gr=None):
        return lib.rosar_beampattern(C.byref(g), C.byref(gr or grid), C.byref(s or sset), angles, n, dr, pattern,
                                     summary, None)

    assert call(s=L.SparseSet(32, 64, 0x30000, 0x40000, L.C16_F16, 0)) == L.ROSAR_ERR_UNSUPPORTED
    assert call(s=L.SparseSet(32, 63, 0x30000, 0x40000, L.C64, 0)) == L.ROSAR_ERR_INVALID_ARG
    for n in (0, -3, (1 << 24) + 1):
        assert call(n=n) == L.ROSAR_ERR_INVALID_ARG, n
    assert call(angles=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(angles=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(dr=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(pattern=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(summary=C.c_void_p(0x10002)) == L.ROSAR_ERR_INVALID_ARG
    assert call(gr=L.PolarGrid(70000, 360, 1.0, 0.05)) == L.ROSAR_ERR_UNSUPPORTED
    assert lib.rosar_last_error().decode() != ""


def test_polar_validation(lib):
    g = geom()
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)

    def call(grid, image=FAKE):
        return lib.rosar_sparse_filter_polar(C.byref(g), C.byref(grid) if grid else None, C.byref(view),
                                             C.byref(sset), L.NEAREST, image, None)

    assert call(None) == L.ROSAR_ERR_INVALID_ARG
    assert call(L.PolarGrid(8, 500, 1.0, 0.05), image=None) == L.ROSAR_ERR_INVALID_ARG
    for bad in (L.PolarGrid(8, 0, 1.0, 0.05), L.PolarGrid(8, (1 << 24) + 1, 1.0, 0.05),
                L.PolarGrid(0, 500, 1.0, 0.05), L.PolarGrid(8, 500, -1.0, 0.05)):
        assert call(bad) == L.ROSAR_ERR_INVALID_ARG, (bad.n_range, bad.n_az, bad.r0_m)
    assert call(L.PolarGrid(70000, 500, 1.0, 0.05)) == L.ROSAR_ERR_UNSUPPORTED
    assert call(L.PolarGrid(40000, 60000, 1.0, 0.0001)) == L.ROSAR_ERR_UNSUPPORTED
    assert lib.rosar_last_error().decode() != ""


def test_bp_cartesian_validation(lib):
    g = geom()
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    good = L.CartGrid(16, 16, -1.0, -1.0, 0.1, 0.1)

    def call(cart=good, angles=None, interp=L.NEAREST, image=FAKE, v=None):
        return lib.rosar_bp_cartesian(C.byref(g), C.byref(cart) if cart else None, C.byref(v or view), angles,
                                      interp, image, None)

    assert call(cart=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(cart=L.CartGrid(16, 0, 0, 0, 0.1, 0.1)) == L.ROSAR_ERR_INVALID_ARG
    assert call(cart=L.CartGrid(16, 16, 0, 0, float("inf"), 0.1)) == L.ROSAR_ERR_INVALID_ARG
    assert call(angles=C.c_void_p(0x10004)) == L.ROSAR_ERR_INVALID_ARG
    assert call(interp=7) == L.ROSAR_ERR_INVALID_ARG
    assert call(image=None) == L.ROSAR_ERR_INVALID_ARG
    assert call(v=L.RcView(0x20000, L.C64, 0, 64, 32, 100, 1.0, 0)) == L.ROSAR_ERR_INVALID_ARG   # ld too small
    assert lib.rosar_last_error().decode() != ""


def test_cartesian_validation(lib):
    g, grid = geom(), L.PolarGrid(8, 360, 1.0, 0.05)
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    sset = L.SparseSet(32, 64, 0x30000, 0x40000, L.C64, 0)

    def call(cart, image=FAKE):
        return lib.rosar_sparse_filter_cartesian(C.byref(g), C.byref(grid), C.byref(cart) if cart else None,
                                                 C.byref(view), C.byref(sset), L.NEAREST, image, None)

    good = L.CartGrid(16, 16, -1.0, -1.0, 0.1, 0.1)
    assert call(None) == L.ROSAR_ERR_INVALID_ARG
    assert call(good, image=None) == L.ROSAR_ERR_INVALID_ARG
    for bad in (L.CartGrid(0, 16, 0, 0, 0.1, 0.1), L.CartGrid(16, 70000, 0, 0, 0.1, 0.1),
                L.CartGrid(16, 16, float("nan"), 0, 0.1, 0.1), L.CartGrid(16, 16, 0, 0, 0.0, 0.1),
                L.CartGrid(16, 16, 0, 0, 0.1, -1.0)):
        assert call(bad) == L.ROSAR_ERR_INVALID_ARG, (bad.nx, bad.ny, bad.x0_m, bad.dx_m, bad.dy_m)
        assert lib.rosar_last_error().decode() != ""


def test_autotune_cache_in_library(tmp_path, lib):
    """The library's autotune cache: entries round-trip through its JSON file (stores merge with
    what the file holds, reloads see them), a missing or corrupt file reads as empty, NULL
    arguments are rejected, and no file keeps entries in memory only."""
    import json
    import paper_2309_08038_amd as rs
    path = str(tmp_path / "tune.json")
    try:
        rs.autotune_cache(path)
        assert rs.autotune_lookup("gfx950|plan|k1") is None
        rs.autotune_store("gfx950|plan|k1", 2, 4, 8, 35.5)
        rs.autotune_store('gfx950|odd "key" \\ |k2', 3, 0, 0, 57.0)
        assert rs.autotune_lookup("gfx950|plan|k1") == (2, 4, 8, 35.5)
        d = json.loads(open(path).read())
        assert d["gfx950|plan|k1"] == {"variant": 2, "pixels_per_lane": 4, "waves": 8, "us": 35.5}
        assert d['gfx950|odd "key" \\ |k2']["variant"] == 3
        # another writer adds an entry to the file; the next store keeps it
        d["other|k3"] = {"variant": 1, "pixels_per_lane": 2, "waves": 2, "us": 3.0}
        open(path, "w").write(json.dumps(d))
        rs.autotune_store("gfx950|plan|k4", 2, 8, 4, 10.0)
        assert set(json.loads(open(path).read())) == {"gfx950|plan|k1", 'gfx950|odd "key" \\ |k2', "other|k3",
                                                      "gfx950|plan|k4"}
        rs.autotune_cache(path)   # reload
        assert rs.autotune_lookup("other|k3") == (1, 2, 2, 3.0)
        bad = tmp_path / "bad.json"
        bad.write_text("{not json")
        rs.autotune_cache(str(bad))
        assert rs.autotune_lookup("gfx950|plan|k1") is None
        rs.autotune_store("gfx950|plan|k1", 2, 2, 4, 1.0)
        assert json.loads(bad.read_text()) == {"gfx950|plan|k1": {"variant": 2, "pixels_per_lane": 2, "waves": 4,
                                                                  "us": 1.0}}
        rs.autotune_cache(str(tmp_path / "missing.json"))
        assert rs.autotune_lookup("gfx950|plan|k1") is None
        rs.autotune_cache(None)
        rs.autotune_store("mem|only", 2, 2, 2, 2.0)
        assert rs.autotune_lookup("mem|only") == (2, 2, 2, 2.0)
        assert not (tmp_path / "mem").exists()
        t, us, found = L.Tile(), C.c_float(0), C.c_int32(0)
        assert lib.rosar_autotune_lookup(None, C.byref(t), C.byref(us), C.byref(found)) == L.ROSAR_ERR_INVALID_ARG
        assert lib.rosar_autotune_store(b"", C.byref(t), 1.0) == L.ROSAR_ERR_INVALID_ARG
        assert lib.rosar_autotune_store(b"k", C.byref(t), -1.0) == L.ROSAR_ERR_INVALID_ARG
    finally:
        rs.autotune_cache(None)


def test_output_buffer_checks():
    """A caller's output buffer must match what the kernel writes; None allocates one."""
    import torch
    from paper_2309_08038_amd.api import _out
    t = torch.empty((4, 6), dtype=torch.complex64)
    assert _out(t, (4, 6), torch.complex64, "cpu") is t
    assert tuple(_out(None, 5, torch.float64, "cpu").shape) == (5,)
    for bad in (torch.empty((4, 7), dtype=torch.complex64), torch.empty((4, 6), dtype=torch.complex128),
                torch.empty((6, 4), dtype=torch.complex64).t()):
        with pytest.raises(ValueError):
            _out(bad, (4, 6), torch.complex64, "cpu")


# ----------------------------------------------------------------- binding argument checks
def test_arg_checks():
    """_arg: element type (TypeError), shape, device and contiguity (ValueError); None passes."""
    import torch
    from paper_2309_08038_amd.api import _arg
    assert _arg(None, "x", torch.float32, (3,)) is None
    with pytest.raises(TypeError):
        _arg(torch.zeros(3, dtype=torch.float64), "x", torch.float32, (3,))
    with pytest.raises(ValueError, match="shape"):
        _arg(torch.zeros(4, dtype=torch.float32), "x", torch.float32, (3,))
    with pytest.raises(ValueError, match="GPU"):
        _arg(torch.zeros(3, dtype=torch.float32), "x", torch.float32, (3,))
    with pytest.raises(TypeError):
        _arg([0.0, 1.0], "x", torch.float32)


class _Case:
    """Host tensors of the small workload's shapes, standing in for device tensors."""

    def __init__(self):
        import torch
        import synth
        import paper_2309_08038_amd as rs
        w = synth.small()
        self.g, self.grid, self.win = w.geometry, w.grid, w.sparse.window
        n, m, rows, k = self.g.n_pulses, self.g.n_fast, self.grid.n_range, w.sparse.k
        self.raw = torch.zeros((n, m), dtype=torch.complex64)
        self.window = torch.ones(m, dtype=torch.float32)
        self.rc = rs.RangeCompressed(torch.zeros((16, n + self.win), dtype=torch.complex64), "c64", 10, 16,
                                     self.win // 2, n + self.win)
        self.offsets = torch.zeros((rows, k), dtype=torch.int32)
        self.weights = torch.zeros((rows, k), dtype=torch.complex64)
        self.pulse_f32 = torch.zeros(n, dtype=torch.float32)
        self.pulse_f64 = torch.zeros(n, dtype=torch.float64)
        self.image = torch.zeros((rows, self.grid.n_az), dtype=torch.complex64)


def _no_launch(monkeypatch, host=()):
    """Every tensor counts as a device tensor except those in `host`, and any library call fails
    the test: each rejection must come from the binding, before a launch."""
    from paper_2309_08038_amd import api
    ids = {id(t) for t in host}
    monkeypatch.setattr(api, "_is_gpu", lambda t: id(t) not in ids)

    def launched():
        raise AssertionError("the library was called")
    monkeypatch.setattr(L, "lib", launched)


def test_binding_rejects_wrong_dtypes_before_launch(monkeypatch):
    """Per-pulse arrays, gradient images and raw cubes of the wrong element type raise TypeError
    (a float64 dphi would be read as float32 pairs; a float32 gradient image is half the bytes
    the kernel reads)."""
    import torch
    import paper_2309_08038_amd as rs
    c = _Case()
    _no_launch(monkeypatch)
    n = c.g.n_pulses
    with pytest.raises(TypeError, match="dphi"):
        rs.sparse_filter(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, dphi=c.pulse_f64)
    with pytest.raises(TypeError, match="dpsi"):
        rs.sparse_filter(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, dpsi=torch.zeros(n, dtype=torch.float16))
    with pytest.raises(TypeError, match="grad_image"):
        rs.sparse_filter_backward(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, c.image.real.contiguous())
    with pytest.raises(TypeError, match="dphi"):
        rs.sparse_filter_backward(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, c.image, dphi=c.pulse_f64)
    with pytest.raises(TypeError, match="grad_image"):
        rs.sparse_filter_adjoint_band(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, c.image.real.contiguous())
    with pytest.raises(TypeError, match="raw"):
        rs.bp_time_domain(c.g, c.grid, c.raw.to(torch.complex128))
    with pytest.raises(TypeError, match="raw"):
        rs.sas_time_domain(c.g, c.grid, torch.zeros(c.raw.shape, dtype=torch.float32), c.offsets, c.weights, c.win)
    with pytest.raises(TypeError, match="raw"):
        rs.range_compress(c.g, c.raw.to(torch.complex128), c.window, 10, 16)
    with pytest.raises(TypeError, match="angles"):
        rs.bp_full(c.g, c.grid, c.rc, angles=c.pulse_f32)
    with pytest.raises(TypeError, match="angles"):
        rs.bp_time_domain(c.g, c.grid, c.raw, angles=c.pulse_f32)
    with pytest.raises(TypeError, match="delta_r"):
        rs.beampattern(c.g, c.grid, c.offsets, c.weights, c.win, torch.zeros(5, dtype=torch.float64),
                       delta_r=torch.zeros(c.grid.n_range, dtype=torch.float32))
    with pytest.raises(TypeError, match="band"):
        bad = rs.RangeCompressed(c.rc.data.real.contiguous(), "c64", 10, 16, c.rc.halo, c.rc.ld)
        rs.sparse_filter(c.g, c.grid, bad, c.offsets, c.weights, c.win)
    with pytest.raises(TypeError, match="offsets"):
        rs.sparse_filter(c.g, c.grid, c.rc, c.offsets.long(), c.weights, c.win)
    with pytest.raises(TypeError, match="weights"):
        rs.sparse_filter(c.g, c.grid, c.rc, c.offsets, c.weights.to(torch.complex128), c.win)


def test_binding_rejects_wrong_shapes_before_launch(monkeypatch):
    import torch
    import paper_2309_08038_amd as rs
    c = _Case()
    _no_launch(monkeypatch)
    n = c.g.n_pulses
    with pytest.raises(ValueError, match="dphi"):
        rs.sparse_filter(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, dphi=torch.zeros(n - 1))
    with pytest.raises(ValueError, match="grad_image"):
        rs.sparse_filter_backward(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, c.image[:-1].contiguous())
    with pytest.raises(ValueError, match="raw"):
        rs.range_compress(c.g, c.raw[:-1].contiguous(), c.window, 10, 16)
    with pytest.raises(ValueError, match="window"):
        rs.range_compress(c.g, c.raw, c.window[:-1].contiguous(), 10, 16)
    with pytest.raises(ValueError, match="angles"):
        rs.bp_cartesian(c.g, rs_cart(), c.rc, angles=torch.zeros(n + 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="one row per range row"):
        rs.sparse_filter(c.g, c.grid, c.rc, c.offsets[:-1].contiguous(), c.weights[:-1].contiguous(), c.win)


def rs_cart():
    from types import SimpleNamespace
    return SimpleNamespace(nx=8, ny=8, x0_m=0.0, y0_m=0.0, dx_m=0.1, dy_m=0.1)


@pytest.mark.parametrize("entry", ["bp_full", "bp_cartesian", "bp_time_domain", "sparse_filter",
                                   "sparse_filter_backward", "beampattern"])
def test_binding_rejects_host_per_pulse_arrays(monkeypatch, entry):
    """A per-pulse (or per-row) array left in host memory raises ValueError in the binding, every
    other argument being a device tensor; nothing is launched."""
    import torch
    import paper_2309_08038_amd as rs
    c = _Case()
    host = {"bp_full": c.pulse_f64, "bp_cartesian": c.pulse_f64, "bp_time_domain": c.pulse_f64,
            "sparse_filter": c.pulse_f32, "sparse_filter_backward": c.pulse_f32,
            "beampattern": torch.zeros(c.grid.n_range, dtype=torch.float64)}[entry]
    _no_launch(monkeypatch, host=[host])
    call = {
        "bp_full": lambda: rs.bp_full(c.g, c.grid, c.rc, angles=host),
        "bp_cartesian": lambda: rs.bp_cartesian(c.g, rs_cart(), c.rc, angles=host),
        "bp_time_domain": lambda: rs.bp_time_domain(c.g, c.grid, c.raw, angles=host),
        "sparse_filter": lambda: rs.sparse_filter(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, dphi=host),
        "sparse_filter_backward": lambda: rs.sparse_filter_backward(c.g, c.grid, c.rc, c.offsets, c.weights, c.win,
                                                                    c.image, dpsi=host),
        "beampattern": lambda: rs.beampattern(c.g, c.grid, c.offsets, c.weights, c.win,
                                              torch.zeros(5, dtype=torch.float64), delta_r=host),
    }[entry]
    with pytest.raises(ValueError, match="GPU"):
        call()


def test_binding_reaches_the_library_with_valid_arguments(monkeypatch):
    """The same calls with every argument valid get past the binding's checks (to the patched
    library), so the rejections above are the checks under test, not some other failure."""
    import torch
    import paper_2309_08038_amd as rs
    c = _Case()
    _no_launch(monkeypatch)
    for call in (lambda: rs.sparse_filter(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, dphi=c.pulse_f32),
                 lambda: rs.bp_full(c.g, c.grid, c.rc, angles=c.pulse_f64),
                 lambda: rs.bp_time_domain(c.g, c.grid, c.raw, angles=c.pulse_f64),
                 lambda: rs.sparse_filter_adjoint_band(c.g, c.grid, c.rc, c.offsets, c.weights, c.win, c.image),
                 lambda: rs.beampattern(c.g, c.grid, c.offsets, c.weights, c.win, torch.zeros(5, dtype=torch.float64),
                                        delta_r=torch.zeros(c.grid.n_range, dtype=torch.float64))):
        with pytest.raises(AssertionError, match="library was called"):
            call()


def test_plan_workspace_entry_points_validate(lib):
    """The workspace queries and runs of a plan reject NULL arguments before any device work."""
    n = C.c_size_t(7)
    assert lib.rosar_sparse_plan_workspace_size(None, C.byref(n)) == L.ROSAR_ERR_INVALID_ARG
    v = L.RcView(0x10000, L.C64, 0, 16, 0, 360, 1.0, 0)
    assert lib.rosar_sparse_plan_run_workspace(None, C.byref(v), FAKE, FAKE, 1 << 20, None) == L.ROSAR_ERR_INVALID_ARG
    assert "NULL" in lib.rosar_last_error().decode()


def test_sas_design_validation(lib):
    """Design parameters, window and workspace are checked before any device work."""
    g = geom(n_pulses=160, n_fast=225, n_fft=225, radius_m=0.145, fc_hz=60e9, slope_hz_s=6.8e13, fs_hz=4.5e6,
             t_start_s=7e-6)
    grid = L.PolarGrid(3, 160, 1.2, 0.3)
    import paper_2309_08038_amd as rs
    from oracle import fppsca as F
    p = rs.sas_params(iters=5)
    nb, nc = C.c_size_t(0), C.c_int32(0)
    assert lib.rosar_sas_design_workspace_size(C.byref(g), C.byref(grid), C.byref(p), C.byref(nb),
                                               C.byref(nc)) == L.ROSAR_OK
    assert nc.value == len(F.candidates(g, 1.8)) and nb.value > 0      # the farthest row sees the most
    call = lambda pp, window=nc.value, ws=FAKE, wsb=nb.value: lib.rosar_sas_design(
        C.byref(g), C.byref(grid), C.byref(pp), FAKE, window, FAKE, FAKE, FAKE, None, ws, wsb, None)
    for bad in (dict(iters=0), dict(mu=1.0), dict(eta=0.0), dict(ls_alpha=0.6), dict(tau0=-1.0), dict(d_angle=0.0)):
        assert call(rs.sas_params(**{"iters": 5, **bad})) == L.ROSAR_ERR_INVALID_ARG, bad
    assert call(p, window=nc.value - 1) == L.ROSAR_ERR_INVALID_ARG
    assert call(p, wsb=nb.value - 1) == L.ROSAR_ERR_WORKSPACE
    assert call(p, ws=C.c_void_p(0x10010)) == L.ROSAR_ERR_WORKSPACE


def test_bp_full_noalloc_validation(lib):
    """The allocation-free back-projection rejects more pulses than its device array holds, and
    bad views or angles, before any device work."""
    grid = L.PolarGrid(8, 360, 1.0, 0.05)
    view = L.RcView(0x20000, L.C64, 0, 64, 32, 424, 1.0, 0)
    g = geom()
    assert lib.rosar_bp_full_noalloc(C.byref(g), C.byref(grid), C.byref(view), C.c_void_p(0x10004), L.NEAREST,
                                     FAKE, None) == L.ROSAR_ERR_INVALID_ARG
    big = geom(n_pulses=65537)
    bgrid = L.PolarGrid(8, 65537, 1.0, 0.05)
    bview = L.RcView(0x20000, L.C64, 0, 64, 0, 65537, 1.0, 0)
    assert lib.rosar_bp_full_noalloc(C.byref(big), C.byref(bgrid), C.byref(bview), None, L.NEAREST, FAKE,
                                     None) == L.ROSAR_ERR_INVALID_ARG
    assert "65536" in lib.rosar_last_error().decode()
