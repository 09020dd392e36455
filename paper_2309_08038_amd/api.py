"""Torch-tensor front end of librosar: device memory and streams come from PyTorch, every step
of the imaging path runs in the HIP kernels behind the C ABI.

Tensors must live on a ROCm GPU.  Complex C64 data are torch.complex64; 16-bit complex data
are float16 / bfloat16 tensors with a trailing dimension of 2 (re, im).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

from . import _lib as L

_TORCH_16 = {"f16": torch.float16, "bf16": torch.bfloat16}


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> C.c_void_p | None:
    return None if t is None else C.c_void_p(t.data_ptr())


def _out(t, shape, dtype, device):
    """The caller's output buffer, checked against what the kernel writes (device, dtype, shape,
    contiguity), or a new one."""
    shape = tuple(shape) if isinstance(shape, (tuple, list)) else (shape,)
    if t is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if (t.device != torch.device(device) or t.dtype != dtype or tuple(t.shape) != shape
            or not t.is_contiguous()):
        raise ValueError(f"output buffer must be a contiguous {dtype} tensor of shape {shape} on {device} "
                         f"(got {t.dtype} {tuple(t.shape)} on {t.device}, contiguous={t.is_contiguous()})")
    return t


def _is_gpu(t) -> bool:
    return t.is_cuda


def _need_gpu(*tensors):
    for t in tensors:
        if t is not None and not _is_gpu(t):
            raise ValueError("librosar operates on GPU tensors only (got a CPU tensor)")
        if t is not None and not t.is_contiguous():
            raise ValueError("librosar needs contiguous tensors")


def _arg(t, name, dtype, shape=None, copy=False):
    """Checks an input tensor before any launch, since the C ABI sees only its pointer: element
    type and shape as the kernel reads them, then that it lives on a GPU (a host pointer would
    fault the kernel), then contiguity (copy=True makes a contiguous copy instead).  None passes
    through."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor (got {type(t).__name__})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not _is_gpu(t):
        raise ValueError(f"{name} must be a GPU tensor (got one on {t.device})")
    if copy:
        return t.contiguous()
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


@dataclass
class RangeCompressed:
    """Range-compressed band Y_T[l_count][ld] as written by range_compress."""
    data: torch.Tensor
    dtype: str
    l_lo: int
    l_count: int
    halo: int
    ld: int
    scale: float = 1.0

    def view(self) -> L.RcView:
        want = {"c64": torch.complex64, "f16": torch.float16, "bf16": torch.bfloat16}.get(self.dtype)
        if want is None:
            raise ValueError(f"unknown band storage type {self.dtype!r}")
        if self.data.dtype != want or (self.dtype != "c64" and self.data.shape[-1] != 2):
            raise TypeError(f"a {self.dtype} band needs a {want} tensor"
                            f"{'' if self.dtype == 'c64' else ' with a trailing (re, im) dimension'}"
                            f" (got {self.data.dtype} {tuple(self.data.shape)})")
        _need_gpu(self.data)
        need = self.l_count * self.ld * (8 if self.dtype == "c64" else 4)
        if self.data.numel() * self.data.element_size() < need:
            raise ValueError(f"band tensor holds {self.data.numel() * self.data.element_size()} bytes, "
                             f"its layout ({self.l_count} rows x ld {self.ld}) needs {need}")
        return L.RcView(self.data.data_ptr(), L.DTYPE_CODES[self.dtype], self.l_lo, self.l_count, self.halo,
                        self.ld, float(self.scale), 0)

    def pulses(self, n_pulses: int) -> torch.Tensor:
        """[l_count, N] complex view of the stored band without the halo columns (unscaled)."""
        d = self.data
        if self.dtype != "c64":
            d = torch.view_as_complex(d.float().contiguous())
        return d[:, self.halo:self.halo + n_pulses] / self.scale


def empty_rc(n_pulses: int, l_lo: int, l_count: int, halo: int = 0, dtype: str = "c64", scale: float = 1.0,
             device="cuda") -> RangeCompressed:
    ld = n_pulses + 2 * halo
    if dtype == "c64":
        t = torch.empty((l_count, ld), dtype=torch.complex64, device=device)
    else:
        t = torch.empty((l_count, ld, 2), dtype=_TORCH_16[dtype], device=device)
    return RangeCompressed(t, dtype, l_lo, l_count, halo, ld, scale)


def range_compress(geom, raw: torch.Tensor, window: torch.Tensor | None, l_lo: int, l_count: int,
                   halo: int = 0, dtype: str = "c64", scale: float = 1.0,
                   out: RangeCompressed | None = None) -> RangeCompressed:
    """Windowed range FFT of every pulse (eq. 38), band [l_lo, l_lo+l_count) stored transposed."""
    _arg(raw, "raw", torch.complex64, (geom.n_pulses, geom.n_fast))
    _arg(window, "window", torch.float32, (geom.n_fast,))
    if out is None:
        out = empty_rc(geom.n_pulses, l_lo, l_count, halo, dtype, scale, raw.device)
    elif out.l_lo != l_lo or out.l_count != l_count:
        raise ValueError("out's band (l_lo, l_count) differs from the requested one")
    g = L.geometry(geom)
    out.view()   # size check of the band tensor against its layout
    L.check(L.lib().rosar_range_compress(C.byref(g), _ptr(raw), _ptr(window), l_lo, l_count, out.halo,
                                         L.DTYPE_CODES[out.dtype], float(out.scale), _ptr(out.data), out.ld,
                                         _stream(raw.device)), "rosar_range_compress")
    return out


def _set(offsets: torch.Tensor, weights: torch.Tensor, window: int, rows: int | None = None) -> L.SparseSet:
    if offsets.dtype != torch.int32 or offsets.dim() != 2:
        raise TypeError("offsets must be int32 [n_range, K]")
    if rows is not None and offsets.shape[0] != rows:
        raise ValueError(f"offsets and weights need one row per range row ({rows}, got {offsets.shape[0]})")
    if weights.dtype == torch.complex64 and weights.dim() == 2:
        wdt = L.C64
    elif weights.dtype == torch.float16 and weights.dim() == 3 and weights.shape[-1] == 2:
        wdt = L.C16_F16
    else:
        raise TypeError("weights must be complex64 [n_range, K] or float16 [n_range, K, 2]")
    if tuple(weights.shape[:2]) != tuple(offsets.shape):
        raise ValueError("weights and offsets shapes differ")
    _need_gpu(offsets, weights)
    return L.SparseSet(int(offsets.shape[1]), int(window), offsets.data_ptr(), weights.data_ptr(), wdt, 0)


def weights_f16(w: torch.Tensor) -> torch.Tensor:
    """complex64 [.., K] -> float16 [.., K, 2] (round to nearest)."""
    return torch.view_as_real(w).to(torch.float16).contiguous()


def sparse_filter(geom, grid, rc: RangeCompressed, offsets: torch.Tensor, weights: torch.Tensor, window: int,
                  dphi: torch.Tensor | None = None, dpsi: torch.Tensor | None = None, interp: str = "nearest",
                  out: torch.Tensor | None = None, tile: tuple[int, int, int] | None = None) -> torch.Tensor:
    """Sparse-aperture azimuth filter (Algorithm 2 / eq. 43) -> complex64 image [n_range, n_az]."""
    s = _set(offsets, weights, window, grid.n_range)
    _arg(dphi, "dphi", torch.float32, (geom.n_pulses,))
    _arg(dpsi, "dpsi", torch.float32, (geom.n_pulses,))
    _need_gpu(rc.data)
    out = _out(out, (grid.n_range, grid.n_az), torch.complex64, rc.data.device)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    t = None if tile is None else L.Tile(tile[0], tile[1], tile[2], 0)
    L.check(L.lib().rosar_sparse_filter_tiled(C.byref(g), C.byref(p), C.byref(v), C.byref(s), _ptr(dphi), _ptr(dpsi),
                                              L.INTERP_CODES[interp], _ptr(out), None if t is None else C.byref(t),
                                              _stream(out.device)), "rosar_sparse_filter")
    return out


def bp_workspace_bytes(geom) -> int:
    g = L.geometry(geom)
    n = C.c_size_t(0)
    L.check(L.lib().rosar_bp_full_workspace_size(C.byref(g), C.byref(n)), "rosar_bp_full_workspace_size")
    return int(n.value)


def bp_full(geom, grid, rc: RangeCompressed, angles: torch.Tensor | None = None, interp: str = "nearest",
            out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Full-aperture back-projection (FFT+BPA) -> complex64 image [n_range, n_az]."""
    _arg(angles, "angles", torch.float64, (geom.n_pulses,))
    _need_gpu(rc.data)
    dev = rc.data.device
    out = _out(out, (grid.n_range, grid.n_az), torch.complex64, dev)
    nbytes = bp_workspace_bytes(geom)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    _need_gpu(workspace)   # its size is checked by the library
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    L.check(L.lib().rosar_bp_full(C.byref(g), C.byref(p), C.byref(v), _ptr(angles), L.INTERP_CODES[interp],
                                  _ptr(out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream(dev)), "rosar_bp_full")
    return out


def bp_full_noalloc(geom, grid, rc: RangeCompressed, angles: torch.Tensor | None = None, interp: str = "nearest",
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """bp_full without a workspace: the per-pulse table lives in the library's device array (at
    most 65536 pulses); calls that overlap on one GPU must not be issued."""
    _arg(angles, "angles", torch.float64, (geom.n_pulses,))
    _need_gpu(rc.data)
    dev = rc.data.device
    out = _out(out, (grid.n_range, grid.n_az), torch.complex64, dev)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    L.check(L.lib().rosar_bp_full_noalloc(C.byref(g), C.byref(p), C.byref(v), _ptr(angles), L.INTERP_CODES[interp],
                                          _ptr(out), _stream(dev)), "rosar_bp_full_noalloc")
    return out


@dataclass
class SasDesign:
    """Result of the robust sparse-array synthesis (Algorithm 1) for every row of a polar grid:
    offsets [rows, window] int32 and weights [rows, window] complex64 with each row's nonzero
    taps first, count [rows] int32 of nonzero taps, history [rows, iters, 6] float64 (J, U',
    b, b1, b2, Newton steps per iteration)."""
    offsets: torch.Tensor
    weights: torch.Tensor
    count: torch.Tensor
    history: torch.Tensor

    def sparse_set(self):
        """(offsets, weights) cut to the largest nonzero count K of any row (zero-weight
        padding beyond a row's own count), contiguous, for sparse_filter / SparsePlan."""
        k = max(int(self.count.max().item()), 1)
        return self.offsets[:, :k].contiguous(), self.weights[:, :k].contiguous()


def sas_params(iters=50, max_newton=50, th=1e-3, phi_mw=0.017453292519943295, d_angle=0.008726646259971648,
               lam_b=50.0, eta=0.0005, u_min=5.0, b_min=1e-5, eps=1e-6, mu=8.0, tau0=1.0, newton_tol=1e-8,
               ls_alpha=0.01, ls_beta=0.5, ls_min=1e-10) -> L.SasParams:
    """Design parameters (defaults: the paper's Table V; barrier-method settings)."""
    return L.SasParams(int(iters), int(max_newton), th, phi_mw, d_angle, lam_b, eta, u_min, b_min, eps, mu, tau0,
                       newton_tol, ls_alpha, ls_beta, ls_min)


def sas_design(geom, grid, delta_r: torch.Tensor, params: L.SasParams | None = None,
               window: int | None = None) -> SasDesign:
    """Robust sparse-array synthesis of every row of `grid` on the GPU (Algorithm 1 with eq. 36);
    delta_r [rows] float64 on the device (rosar_delta_r)."""
    params = sas_params() if params is None else params
    _arg(delta_r, "delta_r", torch.float64, (grid.n_range,))
    dev = delta_r.device
    g, p = L.geometry(geom), L.polar_grid(grid)
    nbytes, ncand = C.c_size_t(0), C.c_int32(0)
    L.check(L.lib().rosar_sas_design_workspace_size(C.byref(g), C.byref(p), C.byref(params), C.byref(nbytes),
                                                    C.byref(ncand)), "rosar_sas_design_workspace_size")
    window = max(int(ncand.value), 1) if window is None else int(window)
    offsets = torch.empty((grid.n_range, window), dtype=torch.int32, device=dev)
    weights = torch.empty((grid.n_range, window), dtype=torch.complex64, device=dev)
    count = torch.empty(grid.n_range, dtype=torch.int32, device=dev)
    hist = torch.empty((grid.n_range, params.iters, 6), dtype=torch.float64, device=dev)
    ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
    L.check(L.lib().rosar_sas_design(C.byref(g), C.byref(p), C.byref(params), _ptr(delta_r), window, _ptr(offsets),
                                     _ptr(weights), _ptr(count), _ptr(hist), _ptr(ws), ws.numel(), _stream(dev)),
            "rosar_sas_design")
    return SasDesign(offsets, weights, count, hist)


def backward_workspace_bytes(geom, grid, offsets, weights, window) -> int:
    g, p, s = L.geometry(geom), L.polar_grid(grid), _set(offsets, weights, window, grid.n_range)
    n = C.c_size_t(0)
    L.check(L.lib().rosar_sparse_filter_backward_workspace_size(C.byref(g), C.byref(p), C.byref(s), C.byref(n)),
            "rosar_sparse_filter_backward_workspace_size")
    return int(n.value)


def sparse_filter_backward(geom, grid, rc: RangeCompressed, offsets, weights, window, grad_image,
                           dphi=None, dpsi=None, interp: str = "linear", need_w=True, need_phi=True, need_psi=True,
                           workspace: torch.Tensor | None = None, out=None):
    """Adjoint of sparse_filter -> (grad_weights c64 [n_range, K] | None, grad_dphi f32 [N] | None,
    grad_dpsi f32 [N] | None) for grad_image = dL/dRe(I) + j dL/dIm(I).  `out` may supply the three
    output tensors (entries None for gradients not wanted)."""
    s = _set(offsets, weights, window, grid.n_range)
    _arg(grad_image, "grad_image", torch.complex64, (grid.n_range, grid.n_az))
    _arg(dphi, "dphi", torch.float32, (geom.n_pulses,))
    _arg(dpsi, "dpsi", torch.float32, (geom.n_pulses,))
    _need_gpu(rc.data)
    dev = grad_image.device
    if out is not None:
        gw, gd, gp = out
        for t, shape, dt in ((gw, tuple(offsets.shape), torch.complex64), (gd, (geom.n_pulses,), torch.float32),
                             (gp, (geom.n_pulses,), torch.float32)):
            if t is not None and (tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous()):
                raise TypeError(f"output gradient must be a contiguous {dt} tensor of shape {shape}")
        _need_gpu(gw, gd, gp)
    else:
        gw = torch.empty(offsets.shape, dtype=torch.complex64, device=dev) if need_w else None
        gd = torch.empty(geom.n_pulses, dtype=torch.float32, device=dev) if need_phi else None
        gp = torch.empty(geom.n_pulses, dtype=torch.float32, device=dev) if need_psi else None
    nbytes = backward_workspace_bytes(geom, grid, offsets, weights, window)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    L.check(L.lib().rosar_sparse_filter_backward(C.byref(g), C.byref(p), C.byref(v), C.byref(s), _ptr(dphi),
                                                 _ptr(dpsi), L.INTERP_CODES[interp], _ptr(grad_image), _ptr(gw),
                                                 _ptr(gd), _ptr(gp), _ptr(workspace),
                                                 workspace.numel() * workspace.element_size(), _stream(dev)),
            "rosar_sparse_filter_backward")
    return gw, gd, gp


class SparseFilterFn(torch.autograd.Function):
    """image = sparse_filter(weights, dphi, dpsi) with the hand-written adjoint as backward.

    Gradients flow to the complex weights and the per-pulse angle/phase errors (the range-
    compressed data are a constant here)."""

    @staticmethod
    def forward(ctx, weights, dphi, dpsi, geom, grid, rc, offsets, window, interp):
        img = sparse_filter(geom, grid, rc, offsets, weights.detach().contiguous(), window,
                            dphi.detach().contiguous(), dpsi.detach().contiguous(), interp)
        ctx.save_for_backward(weights, dphi, dpsi)
        ctx.cfg = (geom, grid, rc, offsets, window, interp)
        return img

    @staticmethod
    def backward(ctx, grad_img):
        weights, dphi, dpsi = ctx.saved_tensors
        geom, grid, rc, offsets, window, interp = ctx.cfg
        gw, gd, gp = sparse_filter_backward(geom, grid, rc, offsets, weights.detach().contiguous(), window,
                                            grad_img.contiguous(), dphi.detach().contiguous(),
                                            dpsi.detach().contiguous(), interp,
                                            need_w=ctx.needs_input_grad[0], need_phi=ctx.needs_input_grad[1],
                                            need_psi=ctx.needs_input_grad[2])
        return gw, gd, gp, None, None, None, None, None, None


def sparse_filter_diff(geom, grid, rc, offsets, weights, window, dphi, dpsi, interp="linear"):
    """Differentiable sparse filter (weights c64, dphi/dpsi float32 [N])."""
    return SparseFilterFn.apply(weights, dphi, dpsi, geom, grid, rc, offsets, window, interp)


class SparseFilterBandFn(torch.autograd.Function):
    """image = sparse_filter(band) for the plain filter, differentiable with respect to the
    range-compressed band [l_count, N] (complex64); backward is the band adjoint A^H g.  The
    weights and offsets are constants here."""

    @staticmethod
    def forward(ctx, band, geom, grid, l_lo, offsets, weights, window, interp):
        n = geom.n_pulses
        if band.dim() != 2:
            raise ValueError("band must be complex64 [l_count, N]")
        _arg(band, "band", torch.complex64, (band.shape[0], n), copy=True)
        halo = window // 2
        rc = empty_rc(n, l_lo, band.shape[0], halo=halo, device=band.device)
        b = band.detach().contiguous()
        # the filter reads the band in its stored layout: pulses with circular halo copies
        rc.data[:, halo:halo + n].copy_(b)
        if halo:
            rc.data[:, :halo].copy_(b[:, n - halo:])
            rc.data[:, halo + n:].copy_(b[:, :halo])
        img = sparse_filter(geom, grid, rc, offsets, weights, window, interp=interp)
        ctx.cfg = (geom, grid, rc, offsets, weights, window, interp)
        return img

    @staticmethod
    def backward(ctx, grad_img):
        geom, grid, rc, offsets, weights, window, interp = ctx.cfg
        gb = sparse_filter_adjoint_band(geom, grid, rc, offsets, weights, window, grad_img.contiguous(), interp=interp)
        return gb, None, None, None, None, None, None, None


def sparse_filter_band_diff(geom, grid, band, l_lo, offsets, weights, window, interp="nearest"):
    """Plain sparse filter differentiable with respect to the band [l_count, N] (complex64)."""
    return SparseFilterBandFn.apply(band, geom, grid, l_lo, offsets, weights, window, interp)


def autotune_sparse_filter(geom, grid, rc: RangeCompressed, offsets, weights, window, reps: int = 20,
                           out: torch.Tensor | None = None):
    """Time every launch shape of the plain sparse filter; returns ((variant, ppl, waves), microseconds)."""
    s = _set(offsets, weights, window, grid.n_range)
    dev = rc.data.device
    out = _out(out, (grid.n_range, grid.n_az), torch.complex64, dev)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    best = L.Tile()
    us = C.c_float(0)
    L.check(L.lib().rosar_autotune_sparse_filter(C.byref(g), C.byref(p), C.byref(v), C.byref(s), _ptr(out), reps,
                                                 C.byref(best), C.byref(us), _stream(dev)),
            "rosar_autotune_sparse_filter")
    return (best.variant, best.pixels_per_lane, best.waves), float(us.value)


@dataclass
class Rotation:
    """One rotation of a batch: inputs, the range-compressed scratch and the output image."""
    geom: object
    grid: object
    raw: torch.Tensor
    window: torch.Tensor | None
    rc: RangeCompressed
    offsets: torch.Tensor
    weights: torch.Tensor
    sparse_window: int
    image: torch.Tensor

    def desc(self) -> L.RotationDesc:
        _arg(self.raw, "raw", torch.complex64, (self.geom.n_pulses, self.geom.n_fast))
        _arg(self.window, "window", torch.float32, (self.geom.n_fast,))
        _arg(self.image, "image", torch.complex64, (self.grid.n_range, self.grid.n_az))
        _need_gpu(self.offsets, self.weights, self.rc.data)
        self.rc.view()   # band size check
        if self.rc.dtype != "c64" or self.weights.dtype != torch.complex64:
            raise TypeError("batched rotations use complex64 data and weights")
        return L.RotationDesc(L.geometry(self.geom), L.polar_grid(self.grid), self.raw.data_ptr(),
                              None if self.window is None else self.window.data_ptr(), self.rc.data.data_ptr(),
                              self.rc.l_lo, self.rc.l_count, self.rc.halo, 0, self.rc.ld,
                              _set(self.offsets, self.weights, self.sparse_window, self.grid.n_range),
                              self.image.data_ptr())


def _descs(rotations):
    arr = (L.RotationDesc * len(rotations))()
    for i, r in enumerate(rotations):
        arr[i] = r.desc()
    return arr


def autotune_cache(path: str | None) -> None:
    """Selects the library's autotune cache file (None: no file; results then stay in memory for
    the process).  The library's autotuners look their shape class up there before timing and
    store what they time; without a call, the ROSAR_AUTOTUNE_CACHE environment variable names
    the file."""
    L.check(L.lib().rosar_autotune(None if path is None else os.fsencode(path)), "rosar_autotune")


def autotune_lookup(key: str):
    """(variant, pixels_per_lane, waves, microseconds) stored under `key`, or None."""
    t, us, found = L.Tile(), C.c_float(0), C.c_int32(0)
    L.check(L.lib().rosar_autotune_lookup(key.encode(), C.byref(t), C.byref(us), C.byref(found)),
            "rosar_autotune_lookup")
    return (t.variant, t.pixels_per_lane, t.waves, float(us.value)) if found.value else None


def autotune_store(key: str, variant: int, pixels_per_lane: int, waves: int, us: float) -> None:
    t = L.Tile(int(variant), int(pixels_per_lane), int(waves), 0)
    L.check(L.lib().rosar_autotune_store(key.encode(), C.byref(t), float(us)), "rosar_autotune_store")


def sparse_plan_autotune(geom, grid, rc: RangeCompressed, offsets, weights, window, interp: str = "nearest",
                         reps: int = 20, out: torch.Tensor | None = None, methods: str = "all",
                         cache: str | None = None):
    """Time every plan launch shape on `rc`, and the azimuth fast convolution where the layout
    admits it; returns (tile, microseconds) with tile = (pixels_per_lane, waves) or "fastconv",
    to pass as SparsePlan(tile=...).  methods: "all", "direct" or "fastconv".  cache: selects the
    library's autotune cache file first (autotune_cache); a result cached for this GPU
    architecture and shape class is returned without timing."""
    variants = {"all": 0, "direct": L.PLAN_DIRECT, "fastconv": L.PLAN_FASTCONV}[methods]
    _need_gpu(rc.data)
    s = _set(offsets, weights, window, grid.n_range)
    dev = rc.data.device
    if cache is not None:
        autotune_cache(cache)
    out = _out(out, (grid.n_range, grid.n_az), torch.complex64, dev)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    best = L.Tile()
    us = C.c_float(0)
    L.check(L.lib().rosar_sparse_plan_autotune(C.byref(g), C.byref(p), C.byref(v), C.byref(s),
                                               L.INTERP_CODES[interp], _ptr(out), variants, reps, C.byref(best),
                                               C.byref(us),
                                               _stream(dev)), "rosar_sparse_plan_autotune")
    return ("fastconv" if best.variant == 3 else (best.pixels_per_lane, best.waves)), float(us.value)


def sparse_filter_cartesian(geom, grid, cart, rc: RangeCompressed, offsets, weights, window, interp: str = "nearest",
                            out: torch.Tensor | None = None) -> torch.Tensor:
    """Algorithm 2 for targets on the Cartesian lattice `cart` (nx, ny, x0_m, y0_m, dx_m, dy_m),
    with the weights of the polar grid rows; returns [ny, nx] complex64."""
    _need_gpu(rc.data)
    s = _set(offsets, weights, window, grid.n_range)
    out = _out(out, (cart.ny, cart.nx), torch.complex64, rc.data.device)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    c = L.CartGrid(int(cart.nx), int(cart.ny), float(cart.x0_m), float(cart.y0_m), float(cart.dx_m), float(cart.dy_m))
    L.check(L.lib().rosar_sparse_filter_cartesian(C.byref(g), C.byref(p), C.byref(c), C.byref(v), C.byref(s),
                                                  L.INTERP_CODES[interp], _ptr(out), _stream(rc.data.device)),
            "rosar_sparse_filter_cartesian")
    return out


def bp_cartesian(geom, cart, rc: RangeCompressed, angles: torch.Tensor | None = None, interp: str = "nearest",
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Full-aperture back-projection for targets on the Cartesian lattice `cart` (nx, ny, x0_m,
    y0_m, dx_m, dy_m), with the given pulse angles (nominal if None); returns [ny, nx] complex64."""
    angles = _arg(angles, "angles", torch.float64, (geom.n_pulses,), copy=True)
    _need_gpu(rc.data)
    out = _out(out, (cart.ny, cart.nx), torch.complex64, rc.data.device)
    g, v = L.geometry(geom), rc.view()
    c = L.CartGrid(int(cart.nx), int(cart.ny), float(cart.x0_m), float(cart.y0_m), float(cart.dx_m), float(cart.dy_m))
    L.check(L.lib().rosar_bp_cartesian(C.byref(g), C.byref(c), C.byref(v), None if angles is None else _ptr(angles),
                                       L.INTERP_CODES[interp], _ptr(out), _stream(rc.data.device)),
            "rosar_bp_cartesian")
    return out


def sparse_filter_polar(geom, grid, rc: RangeCompressed, offsets, weights, window, interp: str = "nearest",
                        out: torch.Tensor | None = None) -> torch.Tensor:
    """Algorithm 2 on a polar grid of grid.n_az azimuth bins, which may differ from the pulse
    count (per-pixel central phase centre); returns [n_range, n_az] complex64."""
    _need_gpu(rc.data)
    s = _set(offsets, weights, window, grid.n_range)
    out = _out(out, (grid.n_range, grid.n_az), torch.complex64, rc.data.device)
    g, p, v = L.geometry(geom), L.polar_grid(grid), rc.view()
    L.check(L.lib().rosar_sparse_filter_polar(C.byref(g), C.byref(p), C.byref(v), C.byref(s), L.INTERP_CODES[interp],
                                              _ptr(out), _stream(rc.data.device)), "rosar_sparse_filter_polar")
    return out


def bp_time_domain(geom, grid, raw: torch.Tensor, window: torch.Tensor | None = None, angles: torch.Tensor | None = None,
                   rows: tuple[int, int] | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Conventional time-domain BPA on the raw samples (exact beat frequency per pixel and
    pulse) for grid rows [first, first + count) (all rows if None); returns [count, n_az]."""
    raw = _arg(raw, "raw", torch.complex64, (geom.n_pulses, geom.n_fast), copy=True)
    window = _arg(window, "window", torch.float32, (geom.n_fast,), copy=True)
    angles = _arg(angles, "angles", torch.float64, (geom.n_pulses,), copy=True)
    first, count = (0, grid.n_range) if rows is None else rows
    out = _out(out, (count, grid.n_az), torch.complex64, raw.device)
    g, p = L.geometry(geom), L.polar_grid(grid)
    L.check(L.lib().rosar_bp_time_domain(C.byref(g), C.byref(p), _ptr(raw), _ptr(window), _ptr(angles), first, count,
                                         _ptr(out), _stream(raw.device)), "rosar_bp_time_domain")
    return out


def sas_time_domain(geom, grid, raw: torch.Tensor, offsets, weights, window_w, window: torch.Tensor | None = None,
                    rows: tuple[int, int] | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Sparse-aperture filter on the raw samples (exact beat frequency per tap) for grid rows
    [first, first + count) (all rows if None); returns [count, n_az]."""
    raw = _arg(raw, "raw", torch.complex64, (geom.n_pulses, geom.n_fast), copy=True)
    window = _arg(window, "window", torch.float32, (geom.n_fast,), copy=True)
    first, count = (0, grid.n_range) if rows is None else rows
    out = _out(out, (count, grid.n_az), torch.complex64, raw.device)
    s = _set(offsets, weights, window_w, grid.n_range)
    g, p = L.geometry(geom), L.polar_grid(grid)
    L.check(L.lib().rosar_sas_time_domain(C.byref(g), C.byref(p), _ptr(raw), _ptr(window), C.byref(s), first,
                                          count, _ptr(out), _stream(raw.device)), "rosar_sas_time_domain")
    return out


def delta_r(geom, grid, window: int, deltas: torch.Tensor, quantile: float = 0.99,
            samples: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """Monte-Carlo Delta_R per range row (eq. 37): `deltas` [window, S] float64 angle errors (draw
    minor), shared by every row.  Returns (delta_r [n_range], samples [n_range, S]), float64."""
    if not isinstance(deltas, torch.Tensor) or deltas.dim() != 2:
        raise ValueError("deltas must be a float64 [window, S] tensor")
    deltas = _arg(deltas, "deltas", torch.float64, (window, deltas.shape[1]), copy=True)
    n_s = deltas.shape[1]
    dev = deltas.device
    samples = _out(samples, (grid.n_range, n_s), torch.float64, dev)
    out = _out(out, grid.n_range, torch.float64, dev)
    g, p = L.geometry(geom), L.polar_grid(grid)
    L.check(L.lib().rosar_delta_r(C.byref(g), C.byref(p), window, _ptr(deltas), n_s, float(quantile), _ptr(samples),
                                  _ptr(out), _stream(dev)), "rosar_delta_r")
    return out, samples


def beampattern(geom, grid, offsets, weights, window: int, angles: torch.Tensor,
                delta_r: torch.Tensor | None = None, pattern: torch.Tensor | None = None,
                summary: torch.Tensor | None = None):
    """|w^H a(phi; R)| of each row's sparse weights at `angles` (float64 radians from the pixel's
    direction; angles[0] the main lobe) and the per-row worst-case summary {main, max side,
    (side + Delta_R)^2 / (main - Delta_R)^2}.  Returns (pattern [n_range, A], summary [n_range, 3])."""
    if not isinstance(angles, torch.Tensor) or angles.dim() != 1:
        raise ValueError("angles must be a float64 vector")
    angles = _arg(angles, "angles", torch.float64, copy=True)
    delta_r = _arg(delta_r, "delta_r", torch.float64, (grid.n_range,), copy=True)
    dev = angles.device
    s = _set(offsets, weights, window, grid.n_range)
    pattern = _out(pattern, (grid.n_range, angles.numel()), torch.float64, dev)
    summary = _out(summary, (grid.n_range, 3), torch.float64, dev)
    g, p = L.geometry(geom), L.polar_grid(grid)
    L.check(L.lib().rosar_beampattern(C.byref(g), C.byref(p), C.byref(s), _ptr(angles), angles.numel(),
                                      None if delta_r is None else _ptr(delta_r), _ptr(pattern), _ptr(summary),
                                      _stream(dev)), "rosar_beampattern")
    return pattern, summary


def sparse_filter_adjoint_band(geom, grid, layout: RangeCompressed, offsets, weights, window, grad_image,
                               interp: str = "nearest", out: torch.Tensor | None = None,
                               workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Gradient of a real loss with respect to the band read by the plain sparse filter,
    A^H grad_image (grad_image = dL/dRe(I) + j dL/dIm(I)).  `layout` gives the band rows; returns
    [l_count, n_pulses] complex64 (the band without its halo copies)."""
    grad_image = _arg(grad_image, "grad_image", torch.complex64, (grid.n_range, grid.n_az), copy=True)
    s = _set(offsets, weights, window, grid.n_range)
    g, p, v = L.geometry(geom), L.polar_grid(grid), layout.view()
    dev = grad_image.device
    out = _out(out, (layout.l_count, geom.n_pulses), torch.complex64, dev)
    need = C.c_size_t(0)
    L.check(L.lib().rosar_sparse_filter_adjoint_band_workspace_size(C.byref(g), C.byref(p), C.byref(v), C.byref(s),
                                                                    L.INTERP_CODES[interp], C.byref(need)),
            "rosar_sparse_filter_adjoint_band_workspace_size")
    if workspace is None:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    _need_gpu(workspace)   # its size is checked by the library
    L.check(L.lib().rosar_sparse_filter_adjoint_band(C.byref(g), C.byref(p), C.byref(v), C.byref(s),
                                                     L.INTERP_CODES[interp], _ptr(grad_image), _ptr(out),
                                                     _ptr(workspace), workspace.numel(), _stream(dev)),
            "rosar_sparse_filter_adjoint_band")
    return out


class SparsePlan:
    """A sparse-filter plan: one filter design (geometry, grid, offsets, weights, band layout)
    applied to the range-compressed data of many rotations.  `layout` is a RangeCompressed whose
    band layout every run must share; the offsets and weights are read when the plan is created.

    tile = (pixels_per_lane, waves) or None: the rows' tap tables are built once on the device
    and each run() computes the image rosar_sparse_filter gives with that launch shape, bit for
    bit.  tile = "fastconv": the same sum as an azimuth fast convolution (FFTs of the band rows
    and of each row's sparse kernels); equal to the direct sum up to float32 rounding.  Runs of
    one fast-convolution plan without a workspace share the plan's spectrum buffer: do not
    overlap them; give overlapping runs a workspace each (run(..., workspace=))."""

    def __init__(self, geom, grid, layout: RangeCompressed, offsets, weights, window, interp: str = "nearest",
                 tile: tuple[int, int] | str | None = None):
        _need_gpu(layout.data)
        s = _set(offsets, weights, window, grid.n_range)
        g, p, v = L.geometry(geom), L.polar_grid(grid), layout.view()
        if tile == "fastconv":
            t = L.Tile(3, 0, 0, 0)
        else:
            t = None if tile is None else L.Tile(2, tile[0], tile[1], 0)
        h = C.c_void_p()
        L.check(L.lib().rosar_sparse_plan_create(C.byref(g), C.byref(p), C.byref(v), C.byref(s),
                                                 L.INTERP_CODES[interp], None if t is None else C.byref(t),
                                                 _stream(layout.data.device), C.byref(h)), "rosar_sparse_plan_create")
        self._h = h
        self.grid = grid
        self.device = layout.data.device
        self._keep = (offsets, weights)

    def workspace_bytes(self) -> int:
        """Bytes of the per-run workspace run(..., workspace=) takes (0 for the direct variant)."""
        n = C.c_size_t(0)
        L.check(L.lib().rosar_sparse_plan_workspace_size(self._h, C.byref(n)), "rosar_sparse_plan_workspace_size")
        return int(n.value)

    def run(self, rc: RangeCompressed, out: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None) -> torch.Tensor:
        """The plan's image of `rc`.  workspace: a device buffer of workspace_bytes() for the
        fast convolution's band-row spectra, so that runs with distinct workspaces may overlap;
        None uses the plan's own buffer (runs must then not overlap)."""
        _need_gpu(rc.data, workspace)
        out = _out(out, (self.grid.n_range, self.grid.n_az), torch.complex64, rc.data.device)
        v = rc.view()
        if workspace is None:
            L.check(L.lib().rosar_sparse_plan_run(self._h, C.byref(v), _ptr(out), _stream(rc.data.device)),
                    "rosar_sparse_plan_run")
        else:
            L.check(L.lib().rosar_sparse_plan_run_workspace(self._h, C.byref(v), _ptr(out), _ptr(workspace),
                                                            workspace.numel() * workspace.element_size(),
                                                            _stream(rc.data.device)), "rosar_sparse_plan_run_workspace")
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.lib().rosar_sparse_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Persistent batched imaging of many rotations (range compression + sparse filter).

    The plan keeps device pointers to the rotations' tensors: keep them alive and unmoved
    while the plan is used."""

    def __init__(self, rotations, tile: tuple[int, int] | None = None):
        self.rotations = list(rotations)
        self._descs = _descs(self.rotations)
        t = None if tile is None else L.Tile(1, tile[0], tile[1], 0)
        h = C.c_void_p()
        L.check(L.lib().rosar_batch_plan_create(self._descs, len(self.rotations), None if t is None else C.byref(t),
                                                C.byref(h)), "rosar_batch_plan_create")
        self._h = h
        self.device = self.rotations[0].raw.device

    def run(self):
        L.check(L.lib().rosar_batch_run(self._h, _stream(self.device)), "rosar_batch_run")

    def info(self):
        px, rc, sf = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(L.lib().rosar_batch_plan_info(self._h, C.byref(px), C.byref(rc), C.byref(sf)), "rosar_batch_plan_info")
        return int(px.value), int(rc.value), int(sf.value)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().rosar_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_autotune(rotations, reps: int = 3):
    """Time every batch launch shape; returns ((pixels_per_lane, waves), microseconds per run)."""
    descs = _descs(rotations)
    best = L.Tile()
    us = C.c_float(0)
    L.check(L.lib().rosar_batch_autotune(descs, len(rotations), reps, C.byref(best), C.byref(us),
                                         _stream(rotations[0].raw.device)), "rosar_batch_autotune")
    return (best.pixels_per_lane, best.waves), float(us.value)
