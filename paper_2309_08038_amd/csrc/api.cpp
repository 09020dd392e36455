// Host side of the C ABI: argument validation (all of it before any device work), derived
// float64 constants, dispatch to the kernel launchers, error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>

#include "rosar_internal.hpp"

namespace {

thread_local std::string g_last_error;

rosar_status fail(rosar_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

rosar_status ok() {
  g_last_error.clear();
  return ROSAR_OK;
}

// Test hook: ROSAR_FAULT_INJECT=launch makes every entry point report a failed launch after
// validation, without touching the device, so error propagation can be exercised anywhere.
bool inject_launch_fault() {
  const char* v = std::getenv("ROSAR_FAULT_INJECT");
  return v && std::strcmp(v, "launch") == 0;
}

rosar_status from_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return ok();
  return fail(ROSAR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
bool finite(double x) { return std::isfinite(x); }
bool pow2(int32_t x) { return x > 0 && (x & (x - 1)) == 0; }

size_t dtype_bytes(int32_t dt) { return dt == ROSAR_C64 ? 8 : 4; }
bool dtype_valid(int32_t dt) { return dt == ROSAR_C64 || dt == ROSAR_C16_F16 || dt == ROSAR_C16_BF16; }

rosar_status check_geometry(const rosar_geometry* g) {
  if (!g) return fail(ROSAR_ERR_INVALID_ARG, "geometry is NULL");
  if (g->reserved != 0) return fail(ROSAR_ERR_INVALID_ARG, "geometry.reserved must be 0");
  if (g->n_pulses < 2) return fail(ROSAR_ERR_INVALID_ARG, "n_pulses must be >= 2 (got %d)", g->n_pulses);
  if (g->n_fast < 1) return fail(ROSAR_ERR_INVALID_ARG, "n_fast must be >= 1 (got %d)", g->n_fast);
  if (g->n_fft < g->n_fast) return fail(ROSAR_ERR_INVALID_ARG, "n_fft (%d) must be >= n_fast (%d)", g->n_fft, g->n_fast);
  if (!(g->radius_m > 0) || !finite(g->radius_m)) return fail(ROSAR_ERR_INVALID_ARG, "radius_m must be finite and > 0");
  if (!finite(g->fc_hz)) return fail(ROSAR_ERR_INVALID_ARG, "fc_hz must be finite");
  if (!(g->slope_hz_s > 0) || !finite(g->slope_hz_s)) return fail(ROSAR_ERR_INVALID_ARG, "slope_hz_s must be finite and > 0");
  if (!(g->fs_hz > 0) || !finite(g->fs_hz)) return fail(ROSAR_ERR_INVALID_ARG, "fs_hz must be finite and > 0");
  if (!finite(g->t_start_s)) return fail(ROSAR_ERR_INVALID_ARG, "t_start_s must be finite");
  if (!(g->c_m_s > 0) || !finite(g->c_m_s)) return fail(ROSAR_ERR_INVALID_ARG, "c_m_s must be finite and > 0");
  if (!finite(g->phi0_rad)) return fail(ROSAR_ERR_INVALID_ARG, "phi0_rad must be finite");
  return ROSAR_OK;
}

// Batched range compression: power-of-two FFT lengths in [64, 2048].
rosar_status check_fft(const rosar_geometry* g) {
  if (!pow2(g->n_fft) || g->n_fft < 64 || g->n_fft > 2048)
    return fail(ROSAR_ERR_UNSUPPORTED, "n_fft must be a power of two in [64, 2048] (got %d)", g->n_fft);
  return ROSAR_OK;
}

// Single-rotation range compression: also any 2^a 3^b 5^c <= 8192 (mixed-radix path).
rosar_status check_fft_single(const rosar_geometry* g) {
  if (!rosar::range_compress_length_supported(g->n_fft))
    return fail(ROSAR_ERR_UNSUPPORTED,
                "n_fft must be a power of two in [64, 2048] or 2^a 3^b 5^c <= 8192 (got %d)", g->n_fft);
  return ROSAR_OK;
}

rosar_status check_grid(const rosar_geometry* g, const rosar_polar_grid* p) {
  if (!p) return fail(ROSAR_ERR_INVALID_ARG, "grid is NULL");
  if (p->n_range < 1) return fail(ROSAR_ERR_INVALID_ARG, "n_range must be >= 1 (got %d)", p->n_range);
  if (p->n_az != g->n_pulses)
    return fail(ROSAR_ERR_UNSUPPORTED, "n_az (%d) must equal n_pulses (%d)", p->n_az, g->n_pulses);
  if (!(p->r0_m > 0) || !finite(p->r0_m)) return fail(ROSAR_ERR_INVALID_ARG, "r0_m must be finite and > 0");
  if (!(p->dr_m >= 0) || !finite(p->dr_m)) return fail(ROSAR_ERR_INVALID_ARG, "dr_m must be finite and >= 0");
  if ((int64_t)p->n_range * p->n_az > ((int64_t)1 << 31))
    return fail(ROSAR_ERR_UNSUPPORTED, "image larger than 2^31 pixels");
  return ROSAR_OK;
}

rosar_status check_band(const rosar_geometry* g, int32_t l_lo, int32_t l_count, int32_t halo, int64_t ld,
                        size_t elem_bytes) {
  if (l_lo < 0) return fail(ROSAR_ERR_INVALID_ARG, "l_lo must be >= 0 (got %d)", l_lo);
  if (l_count < 1) return fail(ROSAR_ERR_INVALID_ARG, "l_count must be >= 1 (got %d)", l_count);
  if ((int64_t)l_lo + l_count > g->n_fft)
    return fail(ROSAR_ERR_INVALID_ARG, "band [%d, %d) exceeds n_fft %d", l_lo, l_lo + l_count, g->n_fft);
  if (halo < 0 || halo > g->n_pulses) return fail(ROSAR_ERR_INVALID_ARG, "halo must be in [0, N] (got %d)", halo);
  if (ld < (int64_t)g->n_pulses + 2 * (int64_t)halo)
    return fail(ROSAR_ERR_INVALID_ARG, "ld (%lld) must be >= N + 2*halo (%lld)", (long long)ld,
                (long long)g->n_pulses + 2 * halo);
  // the kernels address the band through 32-bit byte offsets
  if ((int64_t)l_count * ld * (int64_t)elem_bytes >= ((int64_t)1 << 31))
    return fail(ROSAR_ERR_UNSUPPORTED, "the stored band must be smaller than 2 GiB");
  return ROSAR_OK;
}

rosar_status check_view(const rosar_geometry* g, const rosar_rc_view* v) {
  if (!v) return fail(ROSAR_ERR_INVALID_ARG, "rc view is NULL");
  if (!v->data) return fail(ROSAR_ERR_INVALID_ARG, "rc view data is NULL");
  if (v->reserved != 0) return fail(ROSAR_ERR_INVALID_ARG, "rc view reserved must be 0");
  if (!dtype_valid(v->dtype)) return fail(ROSAR_ERR_INVALID_ARG, "rc view dtype %d is not a rosar_dtype", v->dtype);
  if (!aligned(v->data, dtype_bytes(v->dtype))) return fail(ROSAR_ERR_INVALID_ARG, "rc view data is misaligned");
  if (!(v->scale > 0) || !std::isfinite(v->scale)) return fail(ROSAR_ERR_INVALID_ARG, "rc view scale must be finite and > 0");
  return check_band(g, v->l_lo, v->l_count, v->halo, v->ld, dtype_bytes(v->dtype));
}

rosar_status check_set(const rosar_geometry* g, const rosar_sparse_set* s) {
  if (!s) return fail(ROSAR_ERR_INVALID_ARG, "sparse set is NULL");
  if (s->reserved != 0) return fail(ROSAR_ERR_INVALID_ARG, "sparse set reserved must be 0");
  if (s->k < 1 || s->k > 1024) return fail(ROSAR_ERR_INVALID_ARG, "k must be in [1, 1024] (got %d)", s->k);
  if (s->window < 2 || (s->window & 1) || s->window > g->n_pulses)
    return fail(ROSAR_ERR_INVALID_ARG, "window must be even and in [2, N] (got %d)", s->window);
  if (s->k > s->window) return fail(ROSAR_ERR_INVALID_ARG, "k (%d) must be <= window (%d)", s->k, s->window);
  if (!s->offsets || !aligned(s->offsets, 4)) return fail(ROSAR_ERR_INVALID_ARG, "offsets NULL or misaligned");
  if (s->w_dtype != ROSAR_C64 && s->w_dtype != ROSAR_C16_F16)
    return fail(ROSAR_ERR_INVALID_ARG, "weights dtype must be ROSAR_C64 or ROSAR_C16_F16");
  if (!s->weights || !aligned(s->weights, dtype_bytes(s->w_dtype)))
    return fail(ROSAR_ERR_INVALID_ARG, "weights NULL or misaligned");
  return ROSAR_OK;
}

rosar_status check_image(const void* p, const char* name) {
  if (!p) return fail(ROSAR_ERR_INVALID_ARG, "%s is NULL", name);
  if (!aligned(p, 8)) return fail(ROSAR_ERR_INVALID_ARG, "%s is misaligned (needs 8 bytes)", name);
  return ROSAR_OK;
}

rosar::Geo make_geo(const rosar_geometry* g, const rosar_polar_grid* p) {
  rosar::Geo o{};
  const double two_pi = 6.283185307179586476925286766559;
  o.n = g->n_pulses;
  o.n_range = p ? p->n_range : 0;
  o.radius = g->radius_m;
  o.r0 = p ? p->r0_m : 0.0;
  o.dr = p ? p->dr_m : 0.0;
  o.beta = 2.0 * g->slope_hz_s * (double)g->n_fft / (g->fs_hz * g->c_m_s);
  o.kw = two_pi * (g->slope_hz_s * g->t_start_s + g->fc_hz) / g->c_m_s;
  o.k_over_pi = o.kw / 3.14159265358979323846;
  o.step = two_pi / (double)g->n_pulses;
  o.phi0 = g->phi0_rad;
  return o;
}

rosar::View make_view(const rosar_rc_view* v) {
  return rosar::View{v->data, v->ld, v->l_lo, v->l_count, v->halo, v->dtype, 1.0f / v->scale};
}

// Mean time in microseconds of `reps` back-to-back launches on `s`, after one untimed warm-up.
template <class F>
hipError_t time_launches(F&& launch, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* us) {
  hipError_t e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; e == hipSuccess && r < reps; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  *us = 1000.f * ms / (float)reps;
  return e;
}

#define ROSAR_TRY(expr)              \
  do {                               \
    rosar_status st_ = (expr);       \
    if (st_ != ROSAR_OK) return st_; \
  } while (0)

}  // namespace

namespace rosar {

rosar_status set_error(rosar_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

Geo geo_of(const rosar_geometry* g, const rosar_polar_grid* p) { return make_geo(g, p); }

// A batched rotation: NEAREST, uncorrected, complex float32 data and weights.
rosar_status validate_rotation(const rosar_rotation_desc& d, int index) {
  rosar_status st = check_geometry(&d.geom);
  if (st == ROSAR_OK) st = check_fft(&d.geom);
  if (st == ROSAR_OK) st = check_grid(&d.geom, &d.grid);
  if (st == ROSAR_OK && d.reserved != 0) st = fail(ROSAR_ERR_INVALID_ARG, "descriptor reserved must be 0");
  if (st == ROSAR_OK && (!d.raw || !aligned(d.raw, 8))) st = fail(ROSAR_ERR_INVALID_ARG, "raw NULL or misaligned");
  if (st == ROSAR_OK && d.window && !aligned(d.window, 4)) st = fail(ROSAR_ERR_INVALID_ARG, "window misaligned");
  if (st == ROSAR_OK && (!d.y_t || !aligned(d.y_t, 8))) st = fail(ROSAR_ERR_INVALID_ARG, "y_t NULL or misaligned");
  if (st == ROSAR_OK) st = check_band(&d.geom, d.l_lo, d.l_count, d.halo, d.ld, 8);
  if (st == ROSAR_OK) st = check_set(&d.geom, &d.set);
  if (st == ROSAR_OK && d.set.w_dtype != ROSAR_C64)
    st = fail(ROSAR_ERR_UNSUPPORTED, "batched rotations need ROSAR_C64 weights");
  if (st == ROSAR_OK) st = check_image(d.image, "image");
  if (st != ROSAR_OK) g_last_error = "rotation " + std::to_string(index) + ": " + g_last_error;
  return st;
}

}  // namespace rosar

extern "C" {

const char* rosar_version(void) { return "rosar 1.0 (gfx950)"; }

const char* rosar_status_str(rosar_status s) {
  switch (s) {
    case ROSAR_OK: return "ROSAR_OK";
    case ROSAR_ERR_INVALID_ARG: return "ROSAR_ERR_INVALID_ARG";
    case ROSAR_ERR_UNSUPPORTED: return "ROSAR_ERR_UNSUPPORTED";
    case ROSAR_ERR_HIP: return "ROSAR_ERR_HIP";
    case ROSAR_ERR_NO_MEMORY: return "ROSAR_ERR_NO_MEMORY";
    case ROSAR_ERR_WORKSPACE: return "ROSAR_ERR_WORKSPACE";
  }
  return "ROSAR_ERR_UNKNOWN";
}

const char* rosar_last_error(void) { return g_last_error.c_str(); }

rosar_status rosar_range_compress(const rosar_geometry* geom, const void* raw, const float* window,
                                  int32_t l_lo, int32_t l_count, int32_t halo, rosar_dtype out_dtype,
                                  float out_scale, void* y_t, int64_t ld, rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_fft_single(geom));
  if (!raw || !aligned(raw, 8)) return fail(ROSAR_ERR_INVALID_ARG, "raw NULL or misaligned");
  if (window && !aligned(window, 4)) return fail(ROSAR_ERR_INVALID_ARG, "window misaligned");
  if (!dtype_valid(out_dtype)) return fail(ROSAR_ERR_INVALID_ARG, "out_dtype %d is not a rosar_dtype", (int)out_dtype);
  if (!y_t || !aligned(y_t, dtype_bytes(out_dtype))) return fail(ROSAR_ERR_INVALID_ARG, "y_t NULL or misaligned");
  if (!(out_scale > 0) || !std::isfinite(out_scale)) return fail(ROSAR_ERR_INVALID_ARG, "out_scale must be finite and > 0");
  ROSAR_TRY(check_band(geom, l_lo, l_count, halo, ld, dtype_bytes(out_dtype)));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  rosar::RcArgs a{};
  a.raw = reinterpret_cast<const float2*>(raw);
  a.window = window;
  a.out = y_t;
  a.ld = ld;
  a.n = geom->n_pulses;
  a.m = geom->n_fast;
  a.l = geom->n_fft;
  a.l_lo = l_lo;
  a.l_count = l_count;
  a.halo = halo;
  a.dtype = out_dtype;
  a.scale = out_scale;
  return from_hip(rosar::launch_range_compress(a, reinterpret_cast<hipStream_t>(stream)), "range_compress launch");
}

static rosar_status sparse_common(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                  const rosar_rc_view* rc, const rosar_sparse_set* set,
                                  const float* dphi, const float* dpsi, rosar_interp interp,
                                  void* image, rosar::SparseArgs* out) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  ROSAR_TRY(check_view(geom, rc));
  ROSAR_TRY(check_set(geom, set));
  if (interp != ROSAR_NEAREST && interp != ROSAR_LINEAR)
    return fail(ROSAR_ERR_INVALID_ARG, "interp must be ROSAR_NEAREST or ROSAR_LINEAR");
  if (dphi && !aligned(dphi, 4)) return fail(ROSAR_ERR_INVALID_ARG, "dphi misaligned");
  if (dpsi && !aligned(dpsi, 4)) return fail(ROSAR_ERR_INVALID_ARG, "dpsi misaligned");
  ROSAR_TRY(check_image(image, "image"));
  out->g = make_geo(geom, grid);
  out->y = make_view(rc);
  out->offsets = set->offsets;
  out->weights = set->weights;
  out->k = set->k;
  out->window = set->window;
  out->w_dtype = set->w_dtype;
  out->interp = interp;
  out->dphi = dphi;
  out->dpsi = dpsi;
  out->image = reinterpret_cast<float2*>(image);
  return ROSAR_OK;
}

rosar_status rosar_sparse_filter_tiled(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                       const rosar_rc_view* rc, const rosar_sparse_set* set,
                                       const float* dphi, const float* dpsi, rosar_interp interp,
                                       void* image, const rosar_tile* tile, rosar_stream stream) {
  rosar::SparseArgs a{};
  ROSAR_TRY(sparse_common(geom, grid, rc, set, dphi, dpsi, interp, image, &a));
  rosar::Tile t = rosar::default_tile(geom->n_pulses, rc->dtype);
  // small images default to 1 pixel per lane, which has no planned instantiation: take 2 x 4
  if (!rosar::plan_shape_supported(t.ppl, t.waves)) t = rosar::Tile{2, 2, 4};
  if (tile && (tile->pixels_per_lane || tile->waves || tile->variant)) {
    t = rosar::Tile{tile->variant ? tile->variant : 1, tile->pixels_per_lane ? tile->pixels_per_lane : t.ppl,
                    tile->waves ? tile->waves : t.waves};
    if (!rosar::tile_supported(t))
      return fail(ROSAR_ERR_UNSUPPORTED, "tile (variant %d, %d pixels/lane, %d waves) not supported", tile->variant,
                  tile->pixels_per_lane, tile->waves);
  }
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (dphi || dpsi) return from_hip(rosar::launch_sparse_corrected(a, s), "sparse_filter (corrected) launch");
  return from_hip(rosar::launch_sparse_plain(a, t, s), "sparse_filter launch");
}

rosar_status rosar_sparse_filter(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                 const rosar_rc_view* rc, const rosar_sparse_set* set, const float* dphi,
                                 const float* dpsi, rosar_interp interp, void* image, rosar_stream stream) {
  return rosar_sparse_filter_tiled(geom, grid, rc, set, dphi, dpsi, interp, image, nullptr, stream);
}

rosar_status rosar_bp_full_workspace_size(const rosar_geometry* geom, size_t* bytes) {
  ROSAR_TRY(check_geometry(geom));
  if (!bytes) return fail(ROSAR_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = rosar::bp_workspace_bytes(geom->n_pulses);
  return ok();
}

rosar_status rosar_bp_full(const rosar_geometry* geom, const rosar_polar_grid* grid, const rosar_rc_view* rc,
                           const double* pulse_angle_rad, rosar_interp interp, void* image, void* workspace,
                           size_t workspace_bytes, rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  ROSAR_TRY(check_view(geom, rc));
  if (interp != ROSAR_NEAREST && interp != ROSAR_LINEAR)
    return fail(ROSAR_ERR_INVALID_ARG, "interp must be ROSAR_NEAREST or ROSAR_LINEAR");
  if (pulse_angle_rad && !aligned(pulse_angle_rad, 8)) return fail(ROSAR_ERR_INVALID_ARG, "pulse_angle_rad misaligned");
  ROSAR_TRY(check_image(image, "image"));
  const size_t need = rosar::bp_workspace_bytes(geom->n_pulses);
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < need)
    return fail(ROSAR_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need,
                workspace_bytes);
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  return from_hip(rosar::launch_bp_full(make_geo(geom, grid), make_view(rc), pulse_angle_rad, interp,
                                        reinterpret_cast<float2*>(image), workspace,
                                        reinterpret_cast<hipStream_t>(stream)),
                  "bp_full launch");
}

rosar_status rosar_bp_full_noalloc(const rosar_geometry* geom, const rosar_polar_grid* grid, const rosar_rc_view* rc,
                                   const double* pulse_angle_rad, rosar_interp interp, void* image,
                                   rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  ROSAR_TRY(check_view(geom, rc));
  if (interp != ROSAR_NEAREST && interp != ROSAR_LINEAR)
    return fail(ROSAR_ERR_INVALID_ARG, "interp must be ROSAR_NEAREST or ROSAR_LINEAR");
  if (pulse_angle_rad && !aligned(pulse_angle_rad, 8)) return fail(ROSAR_ERR_INVALID_ARG, "pulse_angle_rad misaligned");
  ROSAR_TRY(check_image(image, "image"));
  if (geom->n_pulses > rosar::kBpNoAllocMaxPulses)
    return fail(ROSAR_ERR_INVALID_ARG, "rosar_bp_full_noalloc takes at most %d pulses (got %d): use rosar_bp_full",
                rosar::kBpNoAllocMaxPulses, geom->n_pulses);
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  void* ws = nullptr;
  ROSAR_TRY(from_hip(rosar::bp_scratch(&ws), "bp_full_noalloc scratch address"));
  return from_hip(rosar::launch_bp_full(make_geo(geom, grid), make_view(rc), pulse_angle_rad, interp,
                                        reinterpret_cast<float2*>(image), ws, reinterpret_cast<hipStream_t>(stream)),
                  "bp_full_noalloc launch");
}

static rosar_status check_sas(const rosar_geometry* geom, const rosar_polar_grid* grid, const rosar_sas_params* p) {
  ROSAR_TRY(check_geometry(geom));
  if (!grid) return fail(ROSAR_ERR_INVALID_ARG, "grid is NULL");
  if (grid->n_range < 1 || grid->n_range > 65536) return fail(ROSAR_ERR_INVALID_ARG, "n_range must be in [1, 65536]");
  if (!(grid->r0_m > 0) || !std::isfinite(grid->r0_m) || !(grid->dr_m >= 0) || !std::isfinite(grid->dr_m))
    return fail(ROSAR_ERR_INVALID_ARG, "r0_m must be > 0 and dr_m >= 0, both finite");
  if (!p) return fail(ROSAR_ERR_INVALID_ARG, "params is NULL");
  if (p->iters < 1 || p->iters > 1000 || p->max_newton < 1 || p->max_newton > 1000)
    return fail(ROSAR_ERR_INVALID_ARG, "iters and max_newton must be in [1, 1000]");
  if (!(p->phi_mw >= 0) || !(p->d_angle > 0) || !(p->eta > 0) || !(p->u_min >= 0) || !(p->lam_b > 0) ||
      !(p->th >= 0) || !(p->eps > 0) || !(p->mu > 1) || !(p->tau0 > 0) || !(p->newton_tol > 0) ||
      !(p->ls_alpha > 0 && p->ls_alpha < 0.5) || !(p->ls_beta > 0 && p->ls_beta < 1) || !(p->ls_min > 0))
    return fail(ROSAR_ERR_INVALID_ARG, "design parameters out of range");
  return ROSAR_OK;
}

rosar_status rosar_sas_design_workspace_size(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                             const rosar_sas_params* params, size_t* bytes,
                                             int32_t* max_candidates) {
  ROSAR_TRY(check_sas(geom, grid, params));
  if (!bytes || !max_candidates) return fail(ROSAR_ERR_INVALID_ARG, "bytes or max_candidates is NULL");
  const rosar::SasSizes z = rosar::sas_sizes(make_geo(geom, grid), *params);
  *bytes = z.bytes;
  *max_candidates = z.n_max;
  return ok();
}

rosar_status rosar_sas_design(const rosar_geometry* geom, const rosar_polar_grid* grid,
                              const rosar_sas_params* params, const double* delta_r, int32_t window,
                              int32_t* offsets, void* weights, int32_t* count, double* history,
                              void* workspace, size_t workspace_bytes, rosar_stream stream) {
  ROSAR_TRY(check_sas(geom, grid, params));
  const rosar::Geo g = make_geo(geom, grid);
  const rosar::SasSizes z = rosar::sas_sizes(g, *params);
  if (window < std::max(z.n_max, 1)) return fail(ROSAR_ERR_INVALID_ARG, "window %d below the largest candidate count %d", window, z.n_max);
  if (!delta_r || !aligned(delta_r, 8)) return fail(ROSAR_ERR_INVALID_ARG, "delta_r NULL or misaligned");
  if (!offsets || !aligned(offsets, 4) || !count || !aligned(count, 4))
    return fail(ROSAR_ERR_INVALID_ARG, "offsets or count NULL or misaligned");
  ROSAR_TRY(check_image(weights, "weights"));
  if (history && !aligned(history, 8)) return fail(ROSAR_ERR_INVALID_ARG, "history misaligned");
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < z.bytes)
    return fail(ROSAR_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", z.bytes,
                workspace_bytes);
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  return from_hip(rosar::launch_sas_design(g, *params, delta_r, z, workspace, window, offsets,
                                           reinterpret_cast<float2*>(weights), count, history,
                                           reinterpret_cast<hipStream_t>(stream)),
                  "sas_design launch");
}

rosar_status rosar_sparse_filter_backward_workspace_size(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                                         const rosar_sparse_set* set, size_t* bytes) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  ROSAR_TRY(check_set(geom, set));
  if (!bytes) return fail(ROSAR_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = rosar::backward_workspace_bytes(geom->n_pulses, grid->n_range, set->k);
  return ok();
}

// Entry points that allocate, synchronise or time refuse a capturing stream before any of that:
// the capture stays valid and the caller gets an error instead of a broken graph.
static rosar_status check_not_capturing(rosar_stream stream, const char* what) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(reinterpret_cast<hipStream_t>(stream), &st) != hipSuccess)
    return fail(ROSAR_ERR_HIP, "%s: cannot query the stream's capture status", what);
  if (st != hipStreamCaptureStatusNone)
    return fail(ROSAR_ERR_INVALID_ARG, "%s allocates and synchronises: it cannot run under stream capture", what);
  return ROSAR_OK;
}

static rosar_status check_cart(const rosar_cart_grid* cart) {
  if (!cart) return fail(ROSAR_ERR_INVALID_ARG, "cart is NULL");
  if (cart->nx < 1 || cart->ny < 1 || cart->ny > 65535 || cart->nx > (1 << 24))
    return fail(ROSAR_ERR_INVALID_ARG, "cart lattice %d x %d outside [1, 2^24] x [1, 65535]", cart->nx, cart->ny);
  if (!std::isfinite(cart->x0_m) || !std::isfinite(cart->y0_m) || !(cart->dx_m > 0.0) || !(cart->dy_m > 0.0) ||
      !std::isfinite(cart->dx_m) || !std::isfinite(cart->dy_m))
    return fail(ROSAR_ERR_INVALID_ARG, "cart origin must be finite and its spacings positive");
  return ROSAR_OK;
}

rosar_status rosar_sparse_filter_cartesian(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                           const rosar_cart_grid* cart, const rosar_rc_view* rc,
                                           const rosar_sparse_set* set, rosar_interp interp, void* image,
                                           rosar_stream stream) {
  rosar::SparseArgs a{};
  ROSAR_TRY(sparse_common(geom, grid, rc, set, nullptr, nullptr, interp, image, &a));
  ROSAR_TRY(check_cart(cart));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  const rosar::CartGrid c{cart->nx, cart->ny, cart->x0_m, cart->y0_m, cart->dx_m, cart->dy_m};
  return from_hip(rosar::launch_sparse_cartesian(a, c, reinterpret_cast<hipStream_t>(stream)),
                  "Cartesian sparse filter launch");
}

rosar_status rosar_bp_cartesian(const rosar_geometry* geom, const rosar_cart_grid* cart, const rosar_rc_view* rc,
                                const double* pulse_angle_rad, rosar_interp interp, void* image,
                                rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_view(geom, rc));
  if (interp != ROSAR_NEAREST && interp != ROSAR_LINEAR)
    return fail(ROSAR_ERR_INVALID_ARG, "interp must be ROSAR_NEAREST or ROSAR_LINEAR");
  ROSAR_TRY(check_cart(cart));
  if (pulse_angle_rad && !aligned(pulse_angle_rad, 8))
    return fail(ROSAR_ERR_INVALID_ARG, "pulse_angle_rad misaligned");
  ROSAR_TRY(check_image(image, "image"));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  const rosar::CartGrid c{cart->nx, cart->ny, cart->x0_m, cart->y0_m, cart->dx_m, cart->dy_m};
  return from_hip(rosar::launch_bp_cartesian(make_geo(geom, nullptr), make_view(rc), c, pulse_angle_rad, interp,
                                             static_cast<float2*>(image), reinterpret_cast<hipStream_t>(stream)),
                  "Cartesian back-projection launch");
}

rosar_status rosar_sparse_filter_polar(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                       const rosar_rc_view* rc, const rosar_sparse_set* set, rosar_interp interp,
                                       void* image, rosar_stream stream) {
  if (!geom) return fail(ROSAR_ERR_INVALID_ARG, "geometry is NULL");
  if (!grid) return fail(ROSAR_ERR_INVALID_ARG, "grid is NULL");
  rosar_polar_grid pulses = *grid;   // rows as given, azimuth on the pulse grid for the shared checks
  pulses.n_az = geom->n_pulses;
  rosar::SparseArgs a{};
  ROSAR_TRY(sparse_common(geom, &pulses, rc, set, nullptr, nullptr, interp, image, &a));
  if (grid->n_az < 1 || grid->n_az > (1 << 24))
    return fail(ROSAR_ERR_INVALID_ARG, "n_az must be in [1, 2^24] (got %d)", grid->n_az);
  if (grid->n_range > 65535) return fail(ROSAR_ERR_UNSUPPORTED, "n_range must be <= 65535 (got %d)", grid->n_range);
  if ((int64_t)grid->n_range * grid->n_az > ((int64_t)1 << 31))
    return fail(ROSAR_ERR_UNSUPPORTED, "image larger than 2^31 pixels");
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  return from_hip(rosar::launch_sparse_polar(a, grid->n_az, reinterpret_cast<hipStream_t>(stream)),
                  "polar sparse filter launch");
}

rosar_status rosar_bp_time_domain(const rosar_geometry* geom, const rosar_polar_grid* grid, const void* raw,
                                  const float* window, const double* pulse_angle_rad, int32_t row_first,
                                  int32_t row_count, void* image, rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  if (geom->n_fast > 2048) return fail(ROSAR_ERR_UNSUPPORTED, "n_fast must be <= 2048 (got %d)", geom->n_fast);
  if (!raw || !aligned(raw, 8)) return fail(ROSAR_ERR_INVALID_ARG, "raw NULL or misaligned");
  if (window && !aligned(window, 4)) return fail(ROSAR_ERR_INVALID_ARG, "window misaligned");
  if (pulse_angle_rad && !aligned(pulse_angle_rad, 8)) return fail(ROSAR_ERR_INVALID_ARG, "pulse_angle_rad misaligned");
  if (row_first < 0 || row_count < 1 || row_count > grid->n_range - row_first)
    return fail(ROSAR_ERR_INVALID_ARG, "rows [%d, %d + %d) outside the grid's %d rows", row_first, row_first, row_count,
                grid->n_range);
  ROSAR_TRY(check_image(image, "image"));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  const rosar::Geo g = make_geo(geom, grid);
  const double cyc_per_m = 2.0 * geom->slope_hz_s / (geom->c_m_s * geom->fs_hz);   // tau K t_s per metre of R
  return from_hip(rosar::launch_bp_time_domain(g, geom->n_fast, cyc_per_m, static_cast<const float2*>(raw), window,
                                               pulse_angle_rad, row_first, row_count, static_cast<float2*>(image),
                                               reinterpret_cast<hipStream_t>(stream)),
                  "time-domain BPA launch");
}

rosar_status rosar_delta_r(const rosar_geometry* geom, const rosar_polar_grid* grid, int32_t window,
                           const double* deltas, int32_t n_samples, double quantile, double* samples,
                           double* delta_r, rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  if (window < 2 || (window & 1) || window > geom->n_pulses)
    return fail(ROSAR_ERR_INVALID_ARG, "window must be even and in [2, N] (got %d)", window);
  if (n_samples < 1 || n_samples > (1 << 24))
    return fail(ROSAR_ERR_INVALID_ARG, "n_samples must be in [1, 2^24] (got %d)", n_samples);
  if (!(quantile > 0.0 && quantile <= 1.0))
    return fail(ROSAR_ERR_INVALID_ARG, "quantile must be in (0, 1] (got %g)", quantile);
  if ((grid->n_range + rosar::delta_r_rows_per_block() - 1) / rosar::delta_r_rows_per_block() > 65535)
    return fail(ROSAR_ERR_UNSUPPORTED, "n_range %d exceeds %d rows", grid->n_range,
                65535 * rosar::delta_r_rows_per_block());
  if (!deltas || !aligned(deltas, 8)) return fail(ROSAR_ERR_INVALID_ARG, "deltas NULL or misaligned");
  if (!samples || !aligned(samples, 8)) return fail(ROSAR_ERR_INVALID_ARG, "samples NULL or misaligned");
  if (!delta_r || !aligned(delta_r, 8)) return fail(ROSAR_ERR_INVALID_ARG, "delta_r NULL or misaligned");
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  // rank of the q point: the smallest sample whose empirical CDF reaches q
  const int rank = (int)std::ceil(quantile * (double)n_samples) - 1;
  return from_hip(rosar::launch_delta_r(make_geo(geom, grid), window, n_samples, deltas, rank, samples, delta_r,
                                        reinterpret_cast<hipStream_t>(stream)),
                  "Delta_R Monte-Carlo launch");
}

rosar_status rosar_beampattern(const rosar_geometry* geom, const rosar_polar_grid* grid, const rosar_sparse_set* set,
                               const double* angles, int32_t n_angles, const double* delta_r, double* pattern,
                               double* summary, rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  ROSAR_TRY(check_set(geom, set));
  if (set->w_dtype != ROSAR_C64) return fail(ROSAR_ERR_UNSUPPORTED, "the beampattern needs ROSAR_C64 weights");
  if (n_angles < 1 || n_angles > (1 << 24))
    return fail(ROSAR_ERR_INVALID_ARG, "n_angles must be in [1, 2^24] (got %d)", n_angles);
  if (grid->n_range > 65535) return fail(ROSAR_ERR_UNSUPPORTED, "n_range must be <= 65535 (got %d)", grid->n_range);
  if (!angles || !aligned(angles, 8)) return fail(ROSAR_ERR_INVALID_ARG, "angles NULL or misaligned");
  if (delta_r && !aligned(delta_r, 8)) return fail(ROSAR_ERR_INVALID_ARG, "delta_r misaligned");
  if (!pattern || !aligned(pattern, 8)) return fail(ROSAR_ERR_INVALID_ARG, "pattern NULL or misaligned");
  if (!summary || !aligned(summary, 8)) return fail(ROSAR_ERR_INVALID_ARG, "summary NULL or misaligned");
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  return from_hip(rosar::launch_beampattern(make_geo(geom, grid), set->k, set->window, set->offsets,
                                            static_cast<const float2*>(set->weights), angles, n_angles, delta_r,
                                            pattern, summary, reinterpret_cast<hipStream_t>(stream)),
                  "beampattern launch");
}

rosar_status rosar_sas_time_domain(const rosar_geometry* geom, const rosar_polar_grid* grid, const void* raw,
                                   const float* window, const rosar_sparse_set* set, int32_t row_first,
                                   int32_t row_count, void* image, rosar_stream stream) {
  ROSAR_TRY(check_geometry(geom));
  ROSAR_TRY(check_grid(geom, grid));
  ROSAR_TRY(check_set(geom, set));
  if (set->w_dtype != ROSAR_C64) return fail(ROSAR_ERR_UNSUPPORTED, "the raw-sample filter needs ROSAR_C64 weights");
  if (geom->n_fast > 2048) return fail(ROSAR_ERR_UNSUPPORTED, "n_fast must be <= 2048 (got %d)", geom->n_fast);
  if (!raw || !aligned(raw, 8)) return fail(ROSAR_ERR_INVALID_ARG, "raw NULL or misaligned");
  if (window && !aligned(window, 4)) return fail(ROSAR_ERR_INVALID_ARG, "window misaligned");
  if (row_first < 0 || row_count < 1 || row_count > grid->n_range - row_first)
    return fail(ROSAR_ERR_INVALID_ARG, "rows [%d, %d + %d) outside the grid's %d rows", row_first, row_first, row_count,
                grid->n_range);
  ROSAR_TRY(check_image(image, "image"));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  const rosar::Geo g = make_geo(geom, grid);
  const double cyc_per_m = 2.0 * geom->slope_hz_s / (geom->c_m_s * geom->fs_hz);
  return from_hip(rosar::launch_sas_time_domain(g, geom->n_fast, cyc_per_m, static_cast<const float2*>(raw), window,
                                                set->offsets, static_cast<const float2*>(set->weights), set->k,
                                                set->window, row_first, row_count, static_cast<float2*>(image),
                                                reinterpret_cast<hipStream_t>(stream)),
                  "raw-sample sparse filter launch");
}

rosar_status rosar_sparse_filter_adjoint_band_workspace_size(const rosar_geometry* geom,
                                                             const rosar_polar_grid* grid, const rosar_rc_view* rc,
                                                             const rosar_sparse_set* set, rosar_interp interp,
                                                             size_t* bytes) {
  rosar::SparseArgs a{};
  alignas(8) static double placeholder = 0.0;   // no image is involved in the size query
  ROSAR_TRY(sparse_common(geom, grid, rc, set, nullptr, nullptr, interp, &placeholder, &a));
  if (!bytes) return fail(ROSAR_ERR_INVALID_ARG, "bytes is NULL");
  rosar::FcLayout L{};
  if (!rosar::fc_tap_layout(a, &L))
    return fail(ROSAR_ERR_UNSUPPORTED, "a range row's taps span more than 32 bin rows");
  *bytes = rosar::adjoint_band_workspace_bytes(L, grid->n_range);
  return ok();
}

rosar_status rosar_sparse_filter_adjoint_band(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                              const rosar_rc_view* rc, const rosar_sparse_set* set, rosar_interp interp,
                                              const void* grad_image, void* grad_band, void* workspace,
                                              size_t workspace_bytes, rosar_stream stream) {
  rosar::SparseArgs a{};
  // validate grad_image in the image's place
  ROSAR_TRY(sparse_common(geom, grid, rc, set, nullptr, nullptr, interp, const_cast<void*>(grad_image), &a));
  ROSAR_TRY(check_image(grad_band, "grad_band"));
  rosar::FcLayout L{};
  if (!rosar::fc_tap_layout(a, &L))
    return fail(ROSAR_ERR_UNSUPPORTED, "a range row's taps span more than 32 bin rows");
  const size_t need = rosar::adjoint_band_workspace_bytes(L, grid->n_range);
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < need)
    return fail(ROSAR_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need,
                workspace_bytes);
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  return from_hip(rosar::launch_adjoint_band(a, L, static_cast<const float2*>(grad_image),
                                             static_cast<float2*>(grad_band), workspace,
                                             reinterpret_cast<hipStream_t>(stream)),
                  "adjoint band launch");
}

rosar_status rosar_sparse_filter_backward(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                          const rosar_rc_view* rc, const rosar_sparse_set* set, const float* dphi,
                                          const float* dpsi, rosar_interp interp, const void* grad_image,
                                          void* grad_weights, float* grad_dphi, float* grad_dpsi, void* workspace,
                                          size_t workspace_bytes, rosar_stream stream) {
  rosar::SparseArgs a{};
  // the image argument is unused by the adjoint: validate grad_image in its place
  ROSAR_TRY(sparse_common(geom, grid, rc, set, dphi, dpsi, interp, const_cast<void*>(grad_image), &a));
  if (set->w_dtype != ROSAR_C64) return fail(ROSAR_ERR_UNSUPPORTED, "backward needs ROSAR_C64 weights");
  if (grad_weights && !aligned(grad_weights, 8)) return fail(ROSAR_ERR_INVALID_ARG, "grad_weights misaligned");
  if (grad_dphi && !aligned(grad_dphi, 4)) return fail(ROSAR_ERR_INVALID_ARG, "grad_dphi misaligned");
  if (grad_dpsi && !aligned(grad_dpsi, 4)) return fail(ROSAR_ERR_INVALID_ARG, "grad_dpsi misaligned");
  const size_t need = rosar::backward_workspace_bytes(geom->n_pulses, grid->n_range, set->k);
  if (!workspace || !aligned(workspace, 256) || workspace_bytes < need)
    return fail(ROSAR_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need,
                workspace_bytes);
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  return from_hip(rosar::launch_sparse_backward(a, reinterpret_cast<const float2*>(grad_image),
                                                reinterpret_cast<float2*>(grad_weights), grad_dphi, grad_dpsi,
                                                workspace, reinterpret_cast<hipStream_t>(stream)),
                  "sparse_filter_backward launch");
}

}  // extern "C"

namespace {

// Autotune cache key: GPU architecture and everything that decides which launch shape wins
// (pulses, rows and their spacing, band layout and storage, taps, window, weight type,
// interpolation).
std::string tune_key(const char* kind, const rosar::SparseArgs& a, const rosar_rc_view* rc, rosar_interp interp) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s|%s|N=%d|rows=%d|r0=%.17g|dr=%.17g|band=%d+%d|halo=%d|ld=%lld|dt=%d|K=%d|W=%d|wdt=%d|interp=%d",
           rosar::tune_arch().c_str(), kind, a.g.n, a.g.n_range, a.g.r0, a.g.dr, rc->l_lo, rc->l_count, rc->halo,
           (long long)rc->ld, rc->dtype, a.k, a.window, a.w_dtype, (int)interp);
  return buf;
}

}  // namespace

struct rosar_sparse_plan {
  rosar::SparseArgs a{};      // geometry, band layout (data NULL), set, interp
  int variant = 2;            // 2: LDS-staged direct sum; 3: azimuth fast convolution
  rosar::PlanLayout layout{};
  rosar::FcLayout fc{};
  rosar_rc_view view{};       // layout fields every run must match
  char* tabs = nullptr;       // n_range row blocks (layout.row_bytes or fc.row_bytes)
  float2* tw = nullptr;       // fast convolution: twiddle table [N]
  float2* spec = nullptr;     // fast convolution: band-row spectra [l_count][N]
  float2* gspec = nullptr;    // fast convolution: kernel spectra [pairs][N]
  int* first = nullptr;       // fast convolution: each range row's first kernel spectrum [n_range]
  int device = -1;
};

namespace {

void free_plan(rosar_sparse_plan* p) {
  if (!p) return;
  (void)hipFree(p->tabs);
  (void)hipFree(p->tw);
  (void)hipFree(p->spec);
  (void)hipFree(p->gspec);
  (void)hipFree(p->first);
  delete p;
}

// Pinned host staging and device temporaries of fc_prepare, freed on every path.
struct PinnedTmp {
  void* p = nullptr;
  ~PinnedTmp() {
    if (p) (void)hipHostFree(p);
  }
};
struct DeviceTmp {
  void* p = nullptr;
  ~DeviceTmp() {
    if (p) (void)hipFree(p);
  }
};

// Device memory of a fast-convolution plan: tables (+ a flag word), twiddles, band-row spectra,
// the kernel spectra of every (range row, bin row) pair and each row's first pair index.
// Uploads the twiddles, builds the tap lists, reads the rows' headers back, numbers the pairs on
// the host (row by row, bin rows in mask order) and builds their spectra, all on `s`, which it
// synchronises.  Every host buffer of a copy is pinned and every copy is one-dimensional, and
// the headers the device wrote are not rewritten: the first pair indices go to an array of their
// own.  UNSUPPORTED if a range row's taps span more bin rows than the row mask holds.
rosar_status fc_prepare(const rosar::SparseArgs& a, const rosar::FcLayout& fc, hipStream_t s, char** tabs, float2** tw,
                        float2** spec, float2** gspec, int** first) {
  const int n_range = a.g.n_range;
  const size_t tab_bytes = (size_t)fc.row_bytes * (size_t)n_range;
  const int n_tw = rosar::fc_twiddle_count(a.g.n);
  const size_t tw_bytes = (size_t)n_tw * sizeof(float2);
  const size_t row_spec_bytes = (size_t)a.g.n * sizeof(float2);
  if (hipMalloc(tabs, tab_bytes + 256) != hipSuccess || hipMalloc(tw, tw_bytes) != hipSuccess ||
      hipMalloc(spec, rosar::fc_spectrum_bytes(a)) != hipSuccess ||
      hipMalloc(first, (size_t)n_range * sizeof(int)) != hipSuccess)
    return fail(ROSAR_ERR_NO_MEMORY, "device allocation of the fast-convolution plan failed");
  PinnedTmp h_tw, h_bad, h_hdr, h_first;
  DeviceTmp d_hdr;
  if (hipHostMalloc(&h_tw.p, tw_bytes) != hipSuccess || hipHostMalloc(&h_bad.p, sizeof(int)) != hipSuccess ||
      hipHostMalloc(&h_hdr.p, (size_t)n_range * sizeof(int4)) != hipSuccess ||
      hipHostMalloc(&h_first.p, (size_t)n_range * sizeof(int)) != hipSuccess ||
      hipMalloc(&d_hdr.p, (size_t)n_range * sizeof(int4)) != hipSuccess)
    return fail(ROSAR_ERR_NO_MEMORY, "staging allocation of the fast-convolution plan failed");
  rosar::fc_twiddles(a.g.n, static_cast<float2*>(h_tw.p));
  int* bad_host = static_cast<int*>(h_bad.p);
  int4* hdr = static_cast<int4*>(h_hdr.p);
  int* first_host = static_cast<int*>(h_first.p);
  *bad_host = 0;
  int* bad = reinterpret_cast<int*>(*tabs + tab_bytes);
  hipError_t e = hipMemcpyAsync(*tw, h_tw.p, tw_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(bad, bad_host, sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = rosar::launch_fc_tables(a, fc, *tabs, bad, static_cast<int4*>(d_hdr.p), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the tables are complete before any read-back
  if (e == hipSuccess) e = hipMemcpyAsync(bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hdr, d_hdr.p, (size_t)n_range * sizeof(int4), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return from_hip(e, "fast-convolution plan set-up");
  if (*bad_host)
    return fail(ROSAR_ERR_UNSUPPORTED, "a range row's taps span more bin rows than the fast convolution handles (32)");
  size_t n_pairs = 0;
  for (int r = 0; r < n_range; ++r) {
    first_host[r] = (int)n_pairs;
    n_pairs += (size_t)__builtin_popcount((unsigned)hdr[r].y);
  }
  PinnedTmp h_pairs;
  DeviceTmp d_pairs;
  if (hipMalloc(gspec, std::max<size_t>(n_pairs, 1) * row_spec_bytes) != hipSuccess ||
      hipMalloc(&d_pairs.p, std::max<size_t>(n_pairs, 1) * sizeof(int2)) != hipSuccess ||
      hipHostMalloc(&h_pairs.p, std::max<size_t>(n_pairs, 1) * sizeof(int2)) != hipSuccess)
    return fail(ROSAR_ERR_NO_MEMORY, "device allocation of the kernel spectra (%zu pairs) failed", n_pairs);
  int2* pairs = static_cast<int2*>(h_pairs.p);
  size_t q = 0;
  for (int r = 0; r < n_range; ++r)
    for (unsigned m = (unsigned)hdr[r].y; m; m &= m - 1u) pairs[q++] = make_int2(r, __builtin_ctz(m));
  e = hipMemcpyAsync(*first, first_host, (size_t)n_range * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n_pairs)
    e = hipMemcpyAsync(d_pairs.p, pairs, n_pairs * sizeof(int2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = rosar::launch_fc_kernel_spectra(fc, *tabs, static_cast<const int2*>(d_pairs.p), (int)n_pairs, *tw, *gspec, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return from_hip(e, "fast-convolution kernel spectra");
  return ROSAR_OK;
}

}  // namespace

extern "C" {

rosar_status rosar_sparse_plan_create(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                      const rosar_rc_view* rc, const rosar_sparse_set* set,
                                      rosar_interp interp, const rosar_tile* tile, rosar_stream stream,
                                      rosar_sparse_plan** out) {
  rosar::clear_error();
  if (!out) return fail(ROSAR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  rosar::SparseArgs a{};
  // the plan has no image yet: sparse_common's image check gets an aligned host placeholder
  alignas(8) static double placeholder = 0.0;
  ROSAR_TRY(sparse_common(geom, grid, rc, set, nullptr, nullptr, interp, &placeholder, &a));
  if (!aligned(rc->data, 16)) return fail(ROSAR_ERR_INVALID_ARG, "rc view data must be 16-byte aligned");
  rosar::Tile t = rosar::default_tile(geom->n_pulses, rc->dtype);
  // small images default to 1 pixel per lane, which has no planned instantiation: take 2 x 4
  if (!rosar::plan_shape_supported(t.ppl, t.waves)) t = rosar::Tile{2, 2, 4};
  if (tile && tile->variant == 3) {
    rosar::FcLayout fc{};
    if (!rosar::fc_layout(a, &fc))
      return fail(ROSAR_ERR_UNSUPPORTED,
                  "the azimuth fast convolution needs N = 2^a 3^b 5^c <= 8192 and at most 32 bin rows per range row");
    ROSAR_TRY(check_not_capturing(stream, "rosar_sparse_plan_create"));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ROSAR_ERR_HIP, "cannot query the current device");
    auto* p = new (std::nothrow) rosar_sparse_plan();
    if (!p) return fail(ROSAR_ERR_NO_MEMORY, "host allocation failed");
    p->a = a;
    p->variant = 3;
    p->fc = fc;
    p->view = *rc;
    p->view.data = nullptr;
    p->device = dev;
    if (inject_launch_fault()) {
      free_plan(p);
      return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
    }
    const rosar_status st =
        fc_prepare(a, fc, reinterpret_cast<hipStream_t>(stream), &p->tabs, &p->tw, &p->spec, &p->gspec, &p->first);
    if (st != ROSAR_OK) {
      free_plan(p);
      return st;
    }
    p->a.y.data = nullptr;
    p->a.image = nullptr;
    *out = p;
    return ROSAR_OK;
  }
  if (tile && (tile->pixels_per_lane || tile->waves || tile->variant)) {
    if (tile->variant != 0 && tile->variant != 2)
      return fail(ROSAR_ERR_UNSUPPORTED, "a plan runs the LDS-staged variant (2) or the fast convolution (3), not %d",
                  tile->variant);
    t.ppl = tile->pixels_per_lane ? tile->pixels_per_lane : t.ppl;
    t.waves = tile->waves ? tile->waves : t.waves;
  }
  if (!rosar::plan_shape_supported(t.ppl, t.waves))
    return fail(ROSAR_ERR_UNSUPPORTED, "plan launch shape %d pixels/lane x %d waves not supported", t.ppl, t.waves);
  rosar::PlanLayout pl{};
  if (!rosar::sparse_plan_layout(a, t.ppl, t.waves, &pl))
    return fail(ROSAR_ERR_UNSUPPORTED,
                "this band layout cannot use the LDS-staged kernel (halo < W/2, rows not 16-byte aligned, or a "
                "staged row over the LDS budget)");
  ROSAR_TRY(check_not_capturing(stream, "rosar_sparse_plan_create"));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(ROSAR_ERR_HIP, "cannot query the current device");
  auto* p = new (std::nothrow) rosar_sparse_plan();
  if (!p) return fail(ROSAR_ERR_NO_MEMORY, "host allocation failed");
  p->a = a;
  p->a.y.data = nullptr;
  p->a.image = nullptr;
  p->layout = pl;
  p->view = *rc;
  p->view.data = nullptr;
  p->device = dev;
  const size_t bytes = (size_t)pl.row_bytes * (size_t)grid->n_range;
  if (hipMalloc(&p->tabs, bytes) != hipSuccess) {
    delete p;
    return fail(ROSAR_ERR_NO_MEMORY, "device allocation of the tap tables (%zu bytes) failed", bytes);
  }
  if (inject_launch_fault()) {
    (void)hipFree(p->tabs);
    delete p;
    return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  }
  a.y.data = rc->data;
  const rosar_status st = from_hip(rosar::launch_tap_tables(a, pl, p->tabs, reinterpret_cast<hipStream_t>(stream)),
                                   "tap table launch");
  if (st != ROSAR_OK) {
    (void)hipFree(p->tabs);
    delete p;
    return st;
  }
  *out = p;
  return ROSAR_OK;
}

}  // extern "C"

namespace {

// A run of the plan; for the fast convolution `spec` is the band-row spectrum buffer (NULL: the
// plan's own).
rosar_status plan_run(const rosar_sparse_plan* plan, const rosar_rc_view* rc, void* image, float2* spec,
                      rosar_stream stream) {
  if (!rc) return fail(ROSAR_ERR_INVALID_ARG, "rc view is NULL");
  const rosar_rc_view& v = plan->view;
  if (rc->dtype != v.dtype || rc->l_lo != v.l_lo || rc->l_count != v.l_count || rc->halo != v.halo ||
      rc->ld != v.ld || rc->scale != v.scale || rc->reserved != 0)
    return fail(ROSAR_ERR_INVALID_ARG, "rc view layout differs from the plan's");
  if (!rc->data || !aligned(rc->data, 16)) return fail(ROSAR_ERR_INVALID_ARG, "rc view data NULL or not 16-byte aligned");
  ROSAR_TRY(check_image(image, "image"));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
    return fail(ROSAR_ERR_INVALID_ARG, "plan was created on another device");
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  rosar::SparseArgs a = plan->a;
  a.y.data = rc->data;
  a.image = reinterpret_cast<float2*>(image);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (plan->variant == 3)
    return from_hip(rosar::launch_fc_run(a, plan->fc, plan->tabs, plan->first, plan->tw, spec ? spec : plan->spec,
                                         plan->gspec, s),
                    "fast convolution launch");
  return from_hip(rosar::launch_sparse_planned(a, plan->layout, plan->tabs, s), "sparse plan launch");
}

}  // namespace

extern "C" {

rosar_status rosar_sparse_plan_run(const rosar_sparse_plan* plan, const rosar_rc_view* rc, void* image,
                                   rosar_stream stream) {
  rosar::clear_error();
  if (!plan) return fail(ROSAR_ERR_INVALID_ARG, "plan is NULL");
  return plan_run(plan, rc, image, nullptr, stream);
}

rosar_status rosar_sparse_plan_workspace_size(const rosar_sparse_plan* plan, size_t* bytes) {
  rosar::clear_error();
  if (!plan || !bytes) return fail(ROSAR_ERR_INVALID_ARG, "plan or bytes is NULL");
  *bytes = plan->variant == 3 ? rosar::fc_spectrum_bytes(plan->a) : 0;
  return ROSAR_OK;
}

rosar_status rosar_sparse_plan_run_workspace(const rosar_sparse_plan* plan, const rosar_rc_view* rc, void* image,
                                             void* workspace, size_t workspace_bytes, rosar_stream stream) {
  rosar::clear_error();
  if (!plan) return fail(ROSAR_ERR_INVALID_ARG, "plan is NULL");
  if (workspace && plan->variant == 3) {
    const size_t need = rosar::fc_spectrum_bytes(plan->a);
    if (!aligned(workspace, 256) || workspace_bytes < need)
      return fail(ROSAR_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need,
                  workspace_bytes);
  }
  return plan_run(plan, rc, image, plan->variant == 3 && workspace ? reinterpret_cast<float2*>(workspace) : nullptr,
                  stream);
}

void rosar_sparse_plan_destroy(rosar_sparse_plan* plan) { free_plan(plan); }

rosar_status rosar_sparse_plan_autotune(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                        const rosar_rc_view* rc, const rosar_sparse_set* set, rosar_interp interp,
                                        void* image, int32_t variants, int32_t reps, rosar_tile* best,
                                        float* best_us, rosar_stream stream) {
  rosar::SparseArgs a{};
  ROSAR_TRY(sparse_common(geom, grid, rc, set, nullptr, nullptr, interp, image, &a));
  if (!aligned(rc->data, 16)) return fail(ROSAR_ERR_INVALID_ARG, "rc view data must be 16-byte aligned");
  if (!best || !best_us) return fail(ROSAR_ERR_INVALID_ARG, "best / best_us is NULL");
  if (reps < 1 || reps > 10000) return fail(ROSAR_ERR_INVALID_ARG, "reps must be in [1, 10000]");
  if (variants != 0 && (variants & ~(ROSAR_PLAN_DIRECT | ROSAR_PLAN_FASTCONV)) != 0)
    return fail(ROSAR_ERR_INVALID_ARG, "variants must be 0 or a mask of ROSAR_PLAN_DIRECT / ROSAR_PLAN_FASTCONV");
  const bool try_direct = variants == 0 || (variants & ROSAR_PLAN_DIRECT);
  const bool try_fc = variants == 0 || (variants & ROSAR_PLAN_FASTCONV);
  int shapes[16][2];
  int n_shapes = 0;
  for (int p : {1, 2, 4, 8})
    for (int w : {1, 2, 4, 8})
      if (try_direct && rosar::plan_shape_supported(p, w)) {
        shapes[n_shapes][0] = p;
        shapes[n_shapes][1] = w;
        ++n_shapes;
      }
  bool any = false;
  rosar::PlanLayout pl{};
  rosar::FcLayout fc{};
  for (int i = 0; i < n_shapes; ++i) any = any || rosar::sparse_plan_layout(a, shapes[i][0], shapes[i][1], &pl);
  const bool fc_ok = try_fc && rosar::fc_layout(a, &fc);
  if (!any && !fc_ok)
    return fail(ROSAR_ERR_UNSUPPORTED, "no plan variant admits this layout (direct: halo >= W/2, 16-byte aligned rows, "
                                       "a staged row within the LDS budget; fast convolution: N = 2^a 3^b 5^c <= 8192)");
  const std::string key = tune_key("plan", a, rc, interp) + "|variants=" + std::to_string(variants);
  if (rosar::tune_cache_get(key, best, best_us)) return ok();
  ROSAR_TRY(check_not_capturing(stream, "rosar_sparse_plan_autotune"));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* tabs = nullptr;   // row blocks do not depend on the shape: one buffer serves every shape
  const size_t bytes = any ? (size_t)pl.row_bytes * (size_t)grid->n_range : 256;
  if (hipMalloc(&tabs, bytes) != hipSuccess)
    return fail(ROSAR_ERR_NO_MEMORY, "device allocation of the tap tables (%zu bytes) failed", bytes);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best_t = 0.f;
  rosar::Tile best_tile{};
  bool have = false;
  for (int i = 0; i < n_shapes; ++i) {
    const int* sh = shapes[i];
    if (e != hipSuccess) break;
    if (!rosar::sparse_plan_layout(a, sh[0], sh[1], &pl)) continue;
    e = rosar::launch_tap_tables(a, pl, tabs, s);
    float us = 0.f;
    if (e == hipSuccess)
      e = time_launches([&] { return rosar::launch_sparse_planned(a, pl, tabs, s); }, reps, s, e0, e1, &us);
    if (e == hipSuccess && (!have || us < best_t)) {
      best_t = us;
      best_tile = rosar::Tile{2, sh[0], sh[1]};
      have = true;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // no run may still read the tables
  (void)hipFree(tabs);
  rosar_status st = e == hipSuccess ? ROSAR_OK : from_hip(e, "plan autotune");
  if (st == ROSAR_OK && fc_ok) {   // the azimuth fast convolution
    char* ftabs = nullptr;
    float2* tw = nullptr;
    float2* spec = nullptr;
    float2* gspec = nullptr;
    int* first = nullptr;
    const rosar_status fst = fc_prepare(a, fc, s, &ftabs, &tw, &spec, &gspec, &first);
    if (fst == ROSAR_OK) {
      float us = 0.f;
      e = time_launches([&] { return rosar::launch_fc_run(a, fc, ftabs, first, tw, spec, gspec, s); }, reps, s, e0, e1,
                        &us);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        st = from_hip(e, "plan autotune");
      } else if (!have || us < best_t) {
        best_t = us;
        best_tile = rosar::Tile{3, 0, 0};
        have = true;
      }
    } else if (fst != ROSAR_ERR_UNSUPPORTED) {
      st = fst;
    }
    (void)hipFree(ftabs);
    (void)hipFree(tw);
    (void)hipFree(spec);
    (void)hipFree(gspec);
    (void)hipFree(first);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != ROSAR_OK) return st;
  best->variant = best_tile.variant;
  best->pixels_per_lane = best_tile.ppl;
  best->waves = best_tile.waves;
  best->reserved = 0;
  *best_us = best_t;
  if (!rosar::tune_cache_put(key, *best, best_t)) return fail(ROSAR_ERR_INVALID_ARG, "cannot write the autotune cache file");
  return ok();
}

rosar_status rosar_autotune_sparse_filter(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                          const rosar_rc_view* rc, const rosar_sparse_set* set, void* image,
                                          int32_t reps, rosar_tile* best, float* best_us, rosar_stream stream) {
  rosar::SparseArgs a{};
  ROSAR_TRY(sparse_common(geom, grid, rc, set, nullptr, nullptr, ROSAR_NEAREST, image, &a));
  if (!best || !best_us) return fail(ROSAR_ERR_INVALID_ARG, "best / best_us is NULL");
  if (reps < 1 || reps > 10000) return fail(ROSAR_ERR_INVALID_ARG, "reps must be in [1, 10000]");
  const std::string key = tune_key("single", a, rc, ROSAR_NEAREST);
  if (rosar::tune_cache_get(key, best, best_us)) return ok();
  ROSAR_TRY(check_not_capturing(stream, "rosar_autotune_sparse_filter"));
  if (inject_launch_fault()) return fail(ROSAR_ERR_HIP, "injected launch failure (ROSAR_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ROSAR_ERR_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ROSAR_ERR_HIP, "hipEventCreate failed");
  }
  float best_t = 0.f;
  rosar::Tile best_tile{};
  bool have = false;
  rosar_status st = ROSAR_OK;
  const int ppls[] = {1, 2, 4, 8};
  const int waves[] = {1, 2, 4, 8};
  for (int v = 1; v <= 2 && st == ROSAR_OK; ++v) for (int p : ppls) {
    for (int w : waves) {
      rosar::Tile t{v, p, w};
      if (!rosar::tile_supported(t)) continue;
      float us = 0.f;
      const hipError_t e = time_launches([&] { return rosar::launch_sparse_plain(a, t, s); }, reps, s, e0, e1, &us);
      if (e != hipSuccess) {
        st = from_hip(e, "autotune launch");
        break;
      }
      if (!have || us < best_t) {
        best_t = us;
        best_tile = t;
        have = true;
      }
    }
    if (st != ROSAR_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ROSAR_OK) return st;
  best->variant = best_tile.variant;
  best->pixels_per_lane = best_tile.ppl;
  best->waves = best_tile.waves;
  best->reserved = 0;
  *best_us = best_t;
  if (!rosar::tune_cache_put(key, *best, best_t)) return fail(ROSAR_ERR_INVALID_ARG, "cannot write the autotune cache file");
  return ok();
}

}  // extern "C"
