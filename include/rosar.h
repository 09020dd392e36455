/*
 * rosar.h - C ABI of the MI355X (gfx950) rotating-SAR imaging library (librosar.so).
 *
 * Method: "Efficient Rotating Synthetic Aperture Radar Imaging via Robust Sparse Array
 * Synthesis" (arXiv 2309.08038).  The online imaging path is
 *   (1) range compression: a windowed FFT of every pulse along fast time (Sec. III-D, eq. 38);
 *   (2) azimuth matched filtering of every polar pixel over a sparse set of K pulses with
 *       precomputed complex weights, I = w^H y over the selected range bins
 *       (Algorithm 2 with eq. 43, only the nonzero weights as in Sec. III-C);
 * and full-aperture back-projection (FFT+BPA, eq. 43 with the BPA weights) is the comparator.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex values are interleaved (re, im).  ROSAR_C64 is 2 x float32; ROSAR_C16_F16 and
 *    ROSAR_C16_BF16 are 2 x 16-bit.  Images and gradients of complex quantities are C64.
 *  - Every array argument is a DEVICE pointer unless marked "host".  The caller owns all
 *    device memory; the library allocates device memory only inside a batch plan (freed by
 *    rosar_batch_plan_destroy).  Structs passed by pointer are host memory, read during the
 *    call only.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default stream) and never
 *    synchronise the device.  Every argument check happens on the host before any device
 *    work; a failed check enqueues nothing and returns a status, with a message available
 *    from rosar_last_error() (thread-local).  A failed kernel launch returns ROSAR_ERR_HIP.
 *  - Geometry (Sec. II-A, eqs. 1-2): pulse n is taken at angle phi0 + 2 pi n / N (plus an
 *    optional per-pulse error) on a circle of radius r; the polar grid has R_i = r0 + i dr and
 *    phi_a = phi0 + 2 pi a / n_az.  This version requires n_az == N, so pixel a is centred on
 *    pulse a (Algorithm 2's centre index) and a tap at offset o reads pulse (a + o) mod N.
 *  - k = 2 pi (K T_Start + f_c) / c (after eq. 12); the fractional FFT bin of slant range R
 *    is u = beta R with beta = 2 K L / (F_s c) (eq. 40).  NEAREST reads bin floor(u + 1/2)
 *    (eq. 40's round); LINEAR interpolates bins floor(u) and floor(u) + 1.  Bins outside the
 *    computed band [l_lo, l_lo + l_count) read as zero.
 *  - The weight vector is applied conjugated (w^H y, eq. 43).  Back-projection applies
 *    alpha_n exp(-j 2 k R_n) to pulse n, alpha_n = max(R cos D - r, 0) / R_n the cosine
 *    antenna pattern (eqs. 3-5, 8, 15): its "w" is the steering vector of eq. 16.
 */
#ifndef ROSAR_H
#define ROSAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ROSAR_VERSION_MAJOR 1
#define ROSAR_VERSION_MINOR 0

struct ihipStream_t;
typedef struct ihipStream_t* rosar_stream; /* identical to hipStream_t */

typedef enum rosar_status {
  ROSAR_OK = 0,
  ROSAR_ERR_INVALID_ARG = 1, /* null pointer, bad size, misaligned, non-finite geometry ... */
  ROSAR_ERR_UNSUPPORTED = 2, /* valid request outside what this version implements */
  ROSAR_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed */
  ROSAR_ERR_NO_MEMORY = 4,   /* device or host allocation failed (batch plans only) */
  ROSAR_ERR_WORKSPACE = 5    /* workspace pointer null or smaller than the queried size */
} rosar_status;

typedef enum rosar_dtype {
  ROSAR_C64 = 0,      /* complex float32 */
  ROSAR_C16_F16 = 1,  /* complex IEEE half */
  ROSAR_C16_BF16 = 2  /* complex bfloat16 */
} rosar_dtype;

typedef enum rosar_interp { ROSAR_NEAREST = 0, ROSAR_LINEAR = 1 } rosar_interp;

/* Radar and rotation (paper Table I/II notation).  n_fft (L) >= n_fast (M); zero padding when
 * L > M (eq. 38).  rosar_range_compress takes L a power of two in [64, 2048] (wave-per-pulse
 * kernels) or any L = 2^a 3^b 5^c <= 8192 (a workgroup per pulse, e.g. M = L = 225); batches
 * take powers of two in [64, 2048]. */
typedef struct rosar_geometry {
  int32_t n_pulses;   /* N: pulses per rotation, >= 2 */
  int32_t n_fast;     /* M: fast-time samples per pulse, >= 1 */
  int32_t n_fft;      /* L: FFT length */
  int32_t reserved;   /* must be 0 */
  double radius_m;    /* r > 0 */
  double fc_hz;       /* f_c */
  double slope_hz_s;  /* K (chirp slope) > 0 */
  double fs_hz;       /* F_s > 0 */
  double t_start_s;   /* T_Start */
  double c_m_s;       /* speed of light > 0 */
  double phi0_rad;    /* angle of pulse 0 and of azimuth bin 0 */
} rosar_geometry;

typedef struct rosar_polar_grid {
  int32_t n_range;    /* rows, >= 1 */
  int32_t n_az;       /* azimuth bins; must equal n_pulses */
  double r0_m;        /* range of row 0, > 0 */
  double dr_m;        /* row spacing, >= 0 */
} rosar_polar_grid;

/* Range-compressed data Y_T[l_count][ld], range-bin major with pulses contiguous.  Element
 * (i, j) holds FFT bin l_lo + i of pulse (j - halo) mod N, for 0 <= j < N + 2*halo; the halo
 * repeats the last/first `halo` pulses on each side so windows near azimuth 0 need no wrap.
 * Stored values are `scale` times the true spectrum (readers divide by it).  Must be aligned
 * to 4 bytes (16-bit types) or 8 bytes (C64). */
typedef struct rosar_rc_view {
  const void* data;
  int32_t dtype;      /* rosar_dtype */
  int32_t l_lo;       /* first stored FFT bin, >= 0 */
  int32_t l_count;    /* stored bins, >= 1, l_lo + l_count <= L */
  int32_t halo;       /* 0 <= halo <= N */
  int64_t ld;         /* row stride in elements, >= N + 2*halo */
  float scale;        /* > 0 */
  int32_t reserved;   /* must be 0 */
} rosar_rc_view;

/* Sparse weight set W* (Algorithm 1's output, the nonzero entries only): for range row i,
 * tap t reads pulse offset offsets[i*k + t] in [-window/2, window/2) (int32) with weight
 * weights[i*k + t] (interleaved complex, w_dtype C64 or C16_F16).  Taps whose offset lies
 * outside that range, or whose bin is outside the band, contribute zero. */
typedef struct rosar_sparse_set {
  int32_t k;          /* taps per row, 1 <= k <= 1024 */
  int32_t window;     /* W: even, 2 <= W <= N */
  const int32_t* offsets;
  const void* weights;
  int32_t w_dtype;    /* rosar_dtype: ROSAR_C64 or ROSAR_C16_F16 */
  int32_t reserved;   /* must be 0 */
} rosar_sparse_set;

/* Launch shape of the sparse filter (0 = let the library choose).  The project's autotuner
 * (rosar_autotune_sparse_filter) searches these. */
typedef struct rosar_tile {
  int32_t variant;        /* 0 auto; 1 direct cached loads; 2 LDS-staged window (falls back
                             to 1 when one staged row does not fit the LDS budget) */
  int32_t pixels_per_lane;/* 1, 2, 4 or 8 (8 x 8 waves is not supported) */
  int32_t waves;          /* waves per workgroup: 1, 2, 4 or 8 */
  int32_t reserved;
} rosar_tile;

const char* rosar_version(void);
const char* rosar_status_str(rosar_status status);
/* Message describing the last failure on the calling thread ("" if none). */
const char* rosar_last_error(void);

/* Range compression (Sec. III-D, eq. 38): for every pulse n and bin l in [l_lo, l_lo+l_count)
 *   Y_1D[n][l] = sum_{m<M} window[m] * raw[n][m] * exp(-j 2 pi l m / L),
 * stored transposed into y_t[l - l_lo][n + halo] (and halo copies, see rosar_rc_view) as
 * out_scale * Y in out_dtype (round to nearest even for 16-bit types).
 *   raw    [N][M] C64, pulse-major, 8-byte aligned.
 *   window [M] float32, or NULL for a rectangular window.
 *   y_t    [l_count][ld] of out_dtype, ld >= N + 2*halo; written, never read.
 * Errors: INVALID_ARG for null/misaligned pointers or bad sizes; UNSUPPORTED for L not a
 * power of two in [64, 2048]. */
rosar_status rosar_range_compress(const rosar_geometry* geom, const void* raw, const float* window,
                                  int32_t l_lo, int32_t l_count, int32_t halo,
                                  rosar_dtype out_dtype, float out_scale,
                                  void* y_t, int64_t ld, rosar_stream stream);

/* Sparse-aperture azimuth filter (Algorithm 2 / eq. 43): for row i and azimuth bin a
 *   image[i][a] = (1/scale) * sum_t conj(w[i,t]) * s(i, a, t),
 *   s = Y(n, u(R^)),  n = (a + o_t) mod N,  R^ = R(o_t 2 pi/N + dphi[n])  (eq. 2).
 * When dphi or dpsi is non-NULL the sample is phase-corrected to the nominal geometry,
 *   s <- s * exp(-j 2k (R^ - R(o_t 2 pi/N))) * exp(-j dpsi[n])
 * (a NULL array counts as zeros).  dphi, dpsi: [N] float32 radians (data taken at
 * phi_n + dphi[n], eq. 37).  image: [n_range][n_az] C64, 8-byte aligned, overwritten.
 * The rc view must hold C64, C16_F16 or C16_BF16 data; weights C64 or C16_F16. */
rosar_status rosar_sparse_filter(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                 const rosar_rc_view* rc, const rosar_sparse_set* set,
                                 const float* dphi, const float* dpsi, rosar_interp interp,
                                 void* image, rosar_stream stream);

/* rosar_sparse_filter with an explicit launch shape (NULL tile = automatic). */
rosar_status rosar_sparse_filter_tiled(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                       const rosar_rc_view* rc, const rosar_sparse_set* set,
                                       const float* dphi, const float* dpsi, rosar_interp interp,
                                       void* image, const rosar_tile* tile, rosar_stream stream);

/* rosar_bp_full for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the same image, with
 * the per-pulse table in a file-scope device array of the library (256 B + 8 B per pulse for
 * at most 65536 pulses, 512.25 KiB per GPU, held until the process ends) instead of a caller
 * workspace.  It calls no allocating routine.  Every call on one GPU shares that GPU's array,
 * which holds the last call's table: calls that overlap on one GPU (several streams, parallel
 * graph branches) race and must not be issued; calls on one stream are ordered.  The first call
 * on a device looks the array's address up (hipGetSymbolAddress) with that device current.
 * Errors: as rosar_bp_full without the workspace checks; INVALID_ARG for n_pulses > 65536. */
rosar_status rosar_bp_full_noalloc(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                   const rosar_rc_view* rc, const double* pulse_angle_rad,
                                   rosar_interp interp, void* image, rosar_stream stream);

/* Device workspace (bytes) needed by rosar_bp_full for this geometry. */
rosar_status rosar_bp_full_workspace_size(const rosar_geometry* geom, size_t* bytes);

/* Full-aperture back-projection over range-compressed data (FFT+BPA, eq. 43 with the BPA
 * weights of Sec. III-D):
 *   image[i][a] = (1/scale) sum over pulses n with v = R_i cos D - r > 0 of
 *                 (v / R_n) * exp(-j 2 k R_n) * Y(n, u(R_n)),
 *   D = phi_a - phi^_n,  R_n = sqrt(R_i^2 + r^2 - 2 R_i r cos D)  (eqs. 2-5, 8, 15).
 * pulse_angle_rad: [N] float64 absolute pulse angles phi^_n (true angles, eq. 37), or NULL
 * for the nominal phi0 + 2 pi n / N.  workspace: >= rosar_bp_full_workspace_size bytes,
 * 256-byte aligned, scratch owned by the caller and overwritten.  image as above. */
rosar_status rosar_bp_full(const rosar_geometry* geom, const rosar_polar_grid* grid,
                           const rosar_rc_view* rc, const double* pulse_angle_rad,
                           rosar_interp interp, void* image, void* workspace,
                           size_t workspace_bytes, rosar_stream stream);

/* Device workspace (bytes) needed by rosar_sparse_filter_backward. */
rosar_status rosar_sparse_filter_backward_workspace_size(const rosar_geometry* geom,
                                                         const rosar_polar_grid* grid,
                                                         const rosar_sparse_set* set,
                                                         size_t* bytes);

/* Adjoint of rosar_sparse_filter for a real loss L, given grad_image = dL/dRe(I) + j dL/dIm(I)
 * ([n_range][n_az] C64).  Outputs (each may be NULL to skip it; all are overwritten):
 *   grad_weights [n_range][k] C64:  sum_a conj(g[i,a]) s(i,a,t)        (same convention)
 *   grad_dphi    [N] float32:       sum_{i,t} Re(conj(g) conj(w) ds/d dphi[n]),  a = n - o_t
 *   grad_dpsi    [N] float32:       sum_{i,t} Im(conj(g) conj(w) s)
 * The derivatives are those of the corrected model (NULL dphi/dpsi = zeros); in NEAREST mode
 * the bin choice is piecewise constant and contributes no derivative.  Interpolation
 * indices are recomputed, never stored.  Weights must be C64 here.  The reductions run in a
 * fixed order (no atomics), so results are reproducible.  workspace: >= the queried size,
 * 256-byte aligned. */
rosar_status rosar_sparse_filter_backward(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                          const rosar_rc_view* rc, const rosar_sparse_set* set,
                                          const float* dphi, const float* dpsi, rosar_interp interp,
                                          const void* grad_image, void* grad_weights,
                                          float* grad_dphi, float* grad_dpsi,
                                          void* workspace, size_t workspace_bytes,
                                          rosar_stream stream);

/* ---------------------------------------------------------------- Cartesian targets
 * Algorithm 2 for targets on a Cartesian lattice x = x0 + ix dx, y = y0 + iy dy (metres, the
 * rotation centre at the origin, angles as phi0 + 2 pi n / N):
 *   R_t = |(x, y)|, phi_t = atan2(y, x); weights of the polar grid row nearest to R_t (targets
 *   more than half a row spacing outside [r0, r0 + (n_range - 1) dr] are 0); central phase
 *   centre n_c = round((phi_t - phi0) / phi_Delta); tap k reads pulse (n_c + o_k) mod N at the
 *   bin of the slant range from that pulse to the target (eq. 2, eq. 40);
 *   I = sum_k conj(w[row, k]) Y[n, u]   (eq. 43).
 * grid: the rows the weights were designed for (n_az must equal n_pulses); rc, set, interp as
 * rosar_sparse_filter (no angle/phase errors); image [ny][nx] C64, 8-byte aligned, overwritten.
 * Errors: as rosar_sparse_filter; INVALID_ARG for a NULL cart, nx outside [1, 2^24], ny
 * outside [1, 65535], or a non-finite origin / non-positive spacing. */
typedef struct rosar_cart_grid {
  int32_t nx, ny;
  double x0_m, y0_m, dx_m, dy_m;
} rosar_cart_grid;
rosar_status rosar_sparse_filter_cartesian(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                           const rosar_cart_grid* cart, const rosar_rc_view* rc,
                                           const rosar_sparse_set* set, rosar_interp interp, void* image,
                                           rosar_stream stream);

/* Full-aperture back-projection (the comparator, eq. 43 with the BPA weights, eqs. 2-5, 8) for
 * targets on the Cartesian lattice `cart`: for the target at (x, y), R_t = |(x, y)|,
 * phi_t = atan2(y, x), D = phi_t - phi_n, and
 *   I = sum over n with R_t cos D - r > 0 of (v / R_n) exp(-j 2 k R_n) Y(n, u(R_n)),
 * u = beta R_n (eq. 40; NEAREST or LINEAR as rosar_sparse_filter).  pulse_angle_rad [n_pulses]
 * float64 (device, 8-byte aligned) or NULL for the nominal phi0 + 2 pi n / N.  rc as
 * rosar_sparse_filter; image [ny][nx] C64 (8-byte aligned, overwritten).  Float64 geometry per
 * (pixel, pulse), float32 accumulation.
 * Errors: INVALID_ARG for pointers, alignment, the view, interp or the lattice (as
 * rosar_sparse_filter_cartesian). */
rosar_status rosar_bp_cartesian(const rosar_geometry* geom, const rosar_cart_grid* cart, const rosar_rc_view* rc,
                                const double* pulse_angle_rad, rosar_interp interp, void* image,
                                rosar_stream stream);

/* Algorithm 2 on a polar grid whose azimuth-bin count A = grid->n_az need not equal N: pixel
 * (i, a) is the target at R_i and phi_a = phi0 + 2 pi a / A; its central phase centre is
 * n_c = round((phi_a - phi0) / phi_Delta) (floor(x + 1/2)), tap k reads pulse (n_c + o_k) mod N
 * at the bin of the slant range from that pulse to the target (eq. 2, eq. 40), with the
 * weights of row i; eq. 43.  A = N gives rosar_sparse_filter's image (float64 geometry per
 * pixel, so not bit for bit).  rc, set, interp as rosar_sparse_filter; image [n_range][A] C64
 * (8-byte aligned, overwritten).
 * Errors: as rosar_sparse_filter for the rows, view and set; INVALID_ARG for A outside
 * [1, 2^24]; UNSUPPORTED for more than 65535 rows or 2^31 pixels. */
rosar_status rosar_sparse_filter_polar(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                       const rosar_rc_view* rc, const rosar_sparse_set* set, rosar_interp interp,
                                       void* image, rosar_stream stream);

/* ---------------------------------------------------------------- rotation-jitter bound
 * Delta_R of the robust weight design (Sec. III-C, parameter settings, eq. 37): the phase-centre
 * directions of the W-element window around a target are perturbed by drawn angle errors, and
 * for every range row R of the grid and every draw s
 *   samples[R][s] = || a^(phi; R) - a(phi; R) ||,
 * a_e = alpha_e exp(+j 2 k R_e) the steering vector of eq. 16 at D_e = (e - W/2) 2 pi / N
 * (alpha as rosar_bp_full: max(R cos D - r, 0) / R_e), a^ the same at D_e + deltas[e][s].
 * delta_r[R] is then the sample of rank ceil(quantile * n_samples) - 1 in ascending order (the
 * quantile point of the empirical CDF; the paper takes 0.99).  The draws are inputs: the caller
 * samples them (the paper: independent N(0, sigma) per element) and the same draws serve every
 * row.  Evaluated in float64 without forming differences of nearly equal ranges or phases.
 * window: even, in [2, N]; deltas [window][n_samples] float64 radians, draw-minor (device,
 * 8-byte aligned, read only); samples [n_range][n_samples] float64 and delta_r [n_range]
 * float64 (device, 8-byte aligned, overwritten).  Non-finite draws give unspecified but
 * finite-time results.
 * Errors: INVALID_ARG for pointers, alignment, window, n_samples outside [1, 2^24] or quantile
 * outside (0, 1]; UNSUPPORTED for more than 524280 range rows. */
rosar_status rosar_delta_r(const rosar_geometry* geom, const rosar_polar_grid* grid, int32_t window,
                           const double* deltas, int32_t n_samples, double quantile, double* samples,
                           double* delta_r, rosar_stream stream);

/* Beampattern of the sparse weights and the worst-case robust check of a weight design
 * (Sec. III-A: eq. 16, C1 and C2 of eq. 20 and their worst-case forms under array errors of
 * norm <= Delta_R).  For every range row R and every angle phi_j (radians, relative to the
 * pixel's direction):
 *   pattern[R][j] = | sum_k conj(w[R, k]) alpha(D_k) exp(+j 2 k R(D_k)) |,  D_k = phi_j - o_k 2 pi / N,
 * R(D) from eq. 2, alpha = max(R cos D - r, 0) / R(D); taps outside [-W/2, W/2) contribute
 * nothing.  angles[0] is the main-lobe direction (normally 0) and the others side-lobe
 * directions; per row summary[R] = {pattern[R][0], max over j >= 1 of pattern[R][j] (0 when
 * n_angles = 1), (max side + Delta_R)^2 / (main - Delta_R)^2}, the last +inf when
 * main <= Delta_R: for unit-norm weights the design meets the side-lobe level eta in the worst
 * case when it is <= eta.  Float64 throughout.
 * set: ROSAR_C64 weights (offsets and weights as rosar_sparse_filter); angles [n_angles] float64
 * (device, 8-byte aligned); delta_r [n_range] float64 or NULL (Delta_R = 0), e.g. from
 * rosar_delta_r; pattern [n_range][n_angles] and summary [n_range][3] float64 (device, 8-byte
 * aligned, overwritten).
 * Errors: INVALID_ARG for pointers, alignment, the set, n_angles outside [1, 2^24];
 * UNSUPPORTED for FP16 weights or more than 65535 rows. */
rosar_status rosar_beampattern(const rosar_geometry* geom, const rosar_polar_grid* grid, const rosar_sparse_set* set,
                               const double* angles, int32_t n_angles, const double* delta_r, double* pattern,
                               double* summary, rosar_stream stream);

/* ---------------------------------------------------------------- time-domain BPA
 * Conventional back-projection on the raw fast-time samples (the W_BP Hadamard sum of
 * Sec. II-C), the comparator of the paper's timing tables:
 *   I(R, phi_a) = sum over visible n of alpha_n exp(-j 2 k R_n)
 *                 sum_m h[m] y[n, m] exp(-j 2 pi tau_n K m t_s),   tau_n = 2 R_n / c,
 * with the exact beat frequency per (pixel, pulse), visibility and alpha as rosar_bp_full.
 * raw [n_pulses][n_fast] C64 (8-byte aligned); window [n_fast] float or NULL (rect);
 * pulse_angle_rad [n_pulses] or NULL (nominal); computes grid rows [row_first, row_first +
 * row_count) into image [row_count][n_az] C64 (8-byte aligned, overwritten).  Its cost is
 * pixels x visible pulses x n_fast, so callers time it on a few rows.
 * Errors: INVALID_ARG for pointers, alignment or a row range outside the grid; UNSUPPORTED for
 * n_fast > 2048 or n_az != n_pulses. */
rosar_status rosar_bp_time_domain(const rosar_geometry* geom, const rosar_polar_grid* grid, const void* raw,
                                  const float* window, const double* pulse_angle_rad, int32_t row_first,
                                  int32_t row_count, void* image, rosar_stream stream);

/* Sparse-aperture filter on the raw samples (the W_SA compensation of Sec. II-C followed by
 * the weights, before range compression):
 *   I[r, a] = sum_k conj(w[r, k]) sum_m h[m] y[(a + o_k) mod N, m] exp(-j 2 pi tau_k K m t_s),
 * tau_k = 2 R(o_k 2 pi / N) / c (eq. 2), the exact beat frequency where rosar_sparse_filter
 * reads the nearest FFT bin of the range-compressed data.  set as for rosar_sparse_filter
 * (ROSAR_C64 weights); raw, window, row range and image as rosar_bp_time_domain.
 * Errors: as rosar_bp_time_domain and the set checks of rosar_sparse_filter; UNSUPPORTED for
 * FP16 weights. */
rosar_status rosar_sas_time_domain(const rosar_geometry* geom, const rosar_polar_grid* grid, const void* raw,
                                   const float* window, const rosar_sparse_set* set, int32_t row_first,
                                   int32_t row_count, void* image, rosar_stream stream);

/* ---------------------------------------------------------------- adjoint w.r.t. the band
 * The plain sparse filter (Algorithm 2 with eq. 43, no angle or phase errors) is linear in the
 * range-compressed band: I[r, a] = sum_k conj(w[r, k]) c Y[l_k, (a + o_k) mod N], c = 1 for
 * NEAREST and 1 - f, f on the two bins of a LINEAR tap (eq. 40).  For a real loss with
 * grad_image = dL/dRe(I) + j dL/dIm(I) this computes the gradient with respect to the band,
 *   grad_band[l][n] = sum over taps (r, k) on bin row l_lo + l of
 *                     w[r, k] c grad_image[r][(n - o_k) mod N],
 * i.e. A^H grad_image.  rc gives the band layout (l_lo, l_count; its data is not read);
 * grad_image [n_range][n_az] C64; grad_band [l_count][n_pulses] C64 (dense, no halo), 8-byte
 * aligned, overwritten.  The workspace (size from the query, 256-byte aligned, caller-owned)
 * holds the per-row tap lists.  Deterministic (fixed summation order, no atomics on the output).
 * Errors: as rosar_sparse_filter; UNSUPPORTED if a range row's taps span more than 32 bin rows;
 * ROSAR_ERR_WORKSPACE for a NULL, misaligned or short workspace. */
rosar_status rosar_sparse_filter_adjoint_band_workspace_size(const rosar_geometry* geom,
                                                             const rosar_polar_grid* grid, const rosar_rc_view* rc,
                                                             const rosar_sparse_set* set, rosar_interp interp,
                                                             size_t* bytes);
rosar_status rosar_sparse_filter_adjoint_band(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                              const rosar_rc_view* rc, const rosar_sparse_set* set,
                                              rosar_interp interp, const void* grad_image, void* grad_band,
                                              void* workspace, size_t workspace_bytes, rosar_stream stream);

/* ---------------------------------------------------------------- batched rotations
 * Many independent rotations of uneven sizes imaged by one range-compression launch per FFT
 * length present (one workgroup per 8-pulse tile) and one persistent sparse-filter launch per
 * occupancy class (rotations grouped by how many workgroups of their LDS layout fit on a CU),
 * whose workgroups pull tiles from the class's device work counter.  The counters are reset by
 * the plan's own kernel at the start of each run, so a run can be captured in a HIP graph and
 * replayed.  NEAREST, uncorrected, C64 only. */
typedef struct rosar_rotation_desc {
  rosar_geometry geom;
  rosar_polar_grid grid;
  const void* raw;          /* [N][M] C64 */
  const float* window;      /* [M] or NULL */
  void* y_t;                /* [l_count][ld] C64 scratch written by the batch */
  int32_t l_lo, l_count, halo, reserved;
  int64_t ld;
  rosar_sparse_set set;     /* weights C64 */
  void* image;              /* [n_range][n_az] C64 */
} rosar_rotation_desc;

typedef struct rosar_batch_plan rosar_batch_plan;

/* Validates every descriptor (host), uploads a device descriptor table and tile prefix sums
 * (the plan owns that device memory until rosar_batch_plan_destroy).  tile: sparse-filter
 * launch shape for all rotations (pixels_per_lane x waves in {1x4, 2x4, 4x4, 8x4, 2x2, 4x2,
 * 8x2, 4x8}; NULL = 4x8).  Every descriptor obeys the rules of rosar_range_compress and
 * rosar_sparse_filter (C64 data and weights); the halo should cover half the window (staging
 * falls back to element copies otherwise).  y_t is written by the run (range compression) and
 * read by its sparse filter; images are overwritten.  Errors name the offending rotation.
 * It allocates and copies synchronously and takes no stream: do not call it while a graph is
 * being captured. */
rosar_status rosar_batch_plan_create(const rosar_rotation_desc* descs, int32_t n,
                                     const rosar_tile* tile, rosar_batch_plan** out);
/* Enqueues counter reset + range compression (one launch per FFT length) + the persistent
 * sparse-filter launches. */
rosar_status rosar_batch_run(rosar_batch_plan* plan, rosar_stream stream);
/* Total pixels and tiles of the plan (host values). */
rosar_status rosar_batch_plan_info(const rosar_batch_plan* plan, int64_t* pixels,
                                   int64_t* rc_tiles, int64_t* sf_tiles);
void rosar_batch_plan_destroy(rosar_batch_plan* plan);
/* Project autotuner for batches: builds a plan for every supported sparse-filter launch shape,
 * times `reps` runs of each on `stream` (outputs are overwritten) and returns the fastest
 * shape in *best with its mean run time in microseconds.  Synchronises `stream`; refuses a
 * capturing stream (INVALID_ARG, the capture stays valid). */
rosar_status rosar_batch_autotune(const rosar_rotation_desc* descs, int32_t n, int32_t reps,
                                  rosar_tile* best, float* best_us, rosar_stream stream);

/* ---------------------------------------------------------------- sparse-filter plans
 * One filter design applied to many rotations: the sparse weights of Sec. III-C are designed
 * offline, only the range-compressed data change from rotation to rotation.  A plan evaluates,
 * once, the tap table of every range row -- the float64 bin of each tap (eq. 2, eq. 40), its
 * packed weight and its offset in the LDS-staged window -- into device memory it owns; each
 * run then copies a row's table into LDS instead of building it.  A run computes the same
 * image, bit for bit, as rosar_sparse_filter_tiled with the same launch shape (variant 2).
 *
 * Variant 3 evaluates the same sum as an azimuth fast convolution.  Under the rotation symmetry
 * the taps of a range row that read bin row l form a sparse kernel over azimuth offsets, and
 * the row of the image is the sum over l of the circular correlation of band row l with it.
 * A run takes the DFT of every band row over the N pulses, and per range row the DFT of each
 * sparse kernel, multiplies and accumulates, and transforms back (mixed-radix FFTs of length N
 * in LDS, float32).  It equals the direct sum up to float32 rounding, not bit for bit.  It
 * needs N = 2^a 3^b 5^c <= 8192 and the taps of a range row on at most 32 bin rows.  The plan
 * owns the band-row spectra (l_count x N x 8 bytes), a twiddle table and per-row tap lists.  Every
 * rosar_sparse_plan_run writes the band-row spectra into that one buffer, so runs of one
 * fast-convolution plan through rosar_sparse_plan_run must not overlap (runs on one stream are
 * ordered); rosar_sparse_plan_run_workspace gives each run its own spectrum buffer. */
typedef struct rosar_sparse_plan rosar_sparse_plan;

/* Validates the arguments as rosar_sparse_filter does and enqueues the table kernel on
 * `stream` (the tables are ready in stream order).  rc fixes the band layout of every run
 * (l_lo, l_count, halo, ld, dtype, scale); its data pointer must be valid and 16-byte aligned
 * but is not read.  offsets and weights are read by the table kernel only: change them and
 * create a new plan.  tile: NULL or {0 or 2, pixels_per_lane, waves} with pixels_per_lane x
 * waves in {4x8, 8x4, 4x4, 2x8, 2x4, 8x2} (NULL = the rosar_sparse_filter default, or 2x4 where
 * that default is 1 pixel per lane, i.e. n_az <= 1024), or {3, 0, 0} for the azimuth fast
 * convolution (which uploads its twiddle table and synchronises `stream`).  No
 * angle/phase errors (those change per rotation: use rosar_sparse_filter).
 * Errors: INVALID_ARG as rosar_sparse_filter; UNSUPPORTED for another shape, a layout the
 * LDS-staged kernel cannot take (halo < W/2, rows not 16-byte aligned, one staged row over the
 * LDS budget), or for variant 3 an N with another prime factor, N > 8192 or more than 32 bin
 * rows per range row; NO_MEMORY if the table allocation ((K or 2K) x 24 bytes + 16 per row, rounded
 * to 16) fails; INVALID_ARG, before any allocation, when `stream` is capturing a graph (the
 * capture stays valid). */
rosar_status rosar_sparse_plan_create(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                      const rosar_rc_view* rc, const rosar_sparse_set* set,
                                      rosar_interp interp, const rosar_tile* tile, rosar_stream stream,
                                      rosar_sparse_plan** out);
/* Runs the plan: rc must have the layout of the plan (a different data pointer is the point);
 * image [n_range][n_az] C64, 8-byte aligned, overwritten.  Asynchronous on `stream`; the plan
 * must be used on the device it was created on.  Safe to capture in a HIP graph. */
rosar_status rosar_sparse_plan_run(const rosar_sparse_plan* plan, const rosar_rc_view* rc, void* image,
                                   rosar_stream stream);
/* Device workspace, in bytes, that one rosar_sparse_plan_run_workspace call of `plan` uses:
 * the band-row spectra (l_count x N x 8) for the fast convolution, 0 for the direct variant.
 * Errors: INVALID_ARG for NULL arguments. */
rosar_status rosar_sparse_plan_workspace_size(const rosar_sparse_plan* plan, size_t* bytes);
/* rosar_sparse_plan_run with the band-row spectra in a caller-owned workspace (at least
 * rosar_sparse_plan_workspace_size bytes, 256-byte aligned, contents undefined on entry and
 * exit) instead of the plan's own buffer.  Runs of one fast-convolution plan that use distinct
 * workspaces may overlap (several streams, parallel branches of a graph): the plan's other
 * buffers are only read by a run.  workspace NULL uses the plan's buffer, as
 * rosar_sparse_plan_run does; the direct variant ignores the workspace.
 * Errors: as rosar_sparse_plan_run; ROSAR_ERR_WORKSPACE for a misaligned or short workspace. */
rosar_status rosar_sparse_plan_run_workspace(const rosar_sparse_plan* plan, const rosar_rc_view* rc, void* image,
                                             void* workspace, size_t workspace_bytes, rosar_stream stream);
/* Frees the plan's tables (NULL is a no-op).  No run of the plan may be pending. */
void rosar_sparse_plan_destroy(rosar_sparse_plan* plan);
/* Project autotuner for plans: for every plan launch shape the layout admits, builds the tap
 * tables (in a temporary device buffer) and times `reps` runs on `stream` (image overwritten);
 * times the azimuth fast convolution too where the layout admits it, and returns the fastest
 * as {2, pixels_per_lane, waves} or {3, 0, 0} in *best, for
 * rosar_sparse_plan_create, with its mean run time in microseconds.  Arguments as
 * rosar_sparse_plan_create plus the image of rosar_sparse_filter; `variants` restricts the
 * candidates to a mask of ROSAR_PLAN_DIRECT (the LDS-staged shapes) and ROSAR_PLAN_FASTCONV
 * (0 = both).  Synchronises `stream`.
 * Errors: as rosar_sparse_plan_create (UNSUPPORTED if no candidate admits the layout);
 * INVALID_ARG for NULL best/best_us, reps outside [1, 10000] or unknown variant bits, or when
 * `stream` is capturing a graph. */
enum { ROSAR_PLAN_DIRECT = 1, ROSAR_PLAN_FASTCONV = 2 };
rosar_status rosar_sparse_plan_autotune(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                        const rosar_rc_view* rc, const rosar_sparse_set* set,
                                        rosar_interp interp, void* image, int32_t variants, int32_t reps,
                                        rosar_tile* best, float* best_us, rosar_stream stream);

/* ---------------------------------------------------------------- autotuning
 * Times every supported launch shape of rosar_sparse_filter on the given inputs (the image is
 * overwritten), `reps` timed launches each, and returns the fastest in *best with its mean
 * time in microseconds.  Synchronises `stream`; refuses a capturing stream (INVALID_ARG). */
rosar_status rosar_autotune_sparse_filter(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                          const rosar_rc_view* rc, const rosar_sparse_set* set,
                                          void* image, int32_t reps, rosar_tile* best,
                                          float* best_us, rosar_stream stream);

/* ---------------------------------------------------------------- robust weight design
 * Offline design of the sparse weights (Sec. III-A/B, Algorithm 1: FPP-SCA).  For every row i of
 * `grid` (range R_i = r0 + i dr; n_az is not used) the candidates are the phase centres that
 * see a target at the row's azimuth (eqs. 4-5): offsets o in [-h, h] with R cos(o 2 pi / N) > r.
 * Steering vectors follow eq. 16 with the cosine pattern max(R cos D - r, 0) / R(D); the main
 * lobe is the target direction, the side-lobe directions are spaced by d_angle over
 * [D_min, -phi_mw] and [phi_mw, D_max].  From w_(0) = 1/sqrt(n), U'_(0) = |w_(0)^H a_m|, each of
 * `iters` iterations solves the convex sub-problem of eq. 36 around the previous iterate
 * (linearised C1, C2, C4 of eqs. 33-35; C3; C5 with U'_min = sqrt(u_min); slacks b, b1, b2 >= 0
 * weighted by lambda_b) with the barrier method: Newton steps with a backtracking line search
 * (ls_alpha, ls_beta; a step below ls_min ends a centring), at most max_newton per centring,
 * centring stops at a Newton decrement^2 / 2 <= newton_tol, tau from tau0 multiplied by mu until
 * the duality-gap bound m / tau < eps.  Entries with |w_k| < th are set to zero. */
typedef struct {
  int32_t iters, max_newton;
  double th, phi_mw, d_angle, lam_b, eta, u_min, b_min;
  double eps, mu, tau0, newton_tol, ls_alpha, ls_beta, ls_min;
} rosar_sas_params;

/* Workspace bytes of rosar_sas_design, and the largest candidate count of any row (the
 * `window` the outputs need).  Errors: INVALID_ARG for NULL arguments, a bad geometry or grid,
 * or parameters out of range (iters in [1, 1000], max_newton in [1, 1000], angles, eta, mu > 1,
 * tau0 > 0, 0 < ls_alpha < 0.5, 0 < ls_beta < 1, eps > 0). */
rosar_status rosar_sas_design_workspace_size(const rosar_geometry* geom, const rosar_polar_grid* grid,
                                             const rosar_sas_params* params, size_t* bytes,
                                             int32_t* max_candidates);
/* Designs every row on the device, one workgroup per row, all iterations in one launch.
 *   delta_r  [n_range] float64 (device): Delta_R of each row (eq. 37; rosar_delta_r).
 *   offsets  [n_range][window] int32, weights [n_range][window] C64 (device, written): each
 *            row's nonzero taps first, in candidate order (offset relative to the target's
 *            pulse, weight applied conjugated as in eq. 43), zero-weight padding after them.
 *   count    [n_range] int32 (device, written): nonzero taps per row.
 *   history  [n_range][iters][6] float64 (device) or NULL: per iteration the objective
 *            J = ||w||_1 + lambda_b (b + b1 + b2), U', b, b1, b2 and the Newton steps taken.
 * A row whose taps are not all accepted (b + b1 + b2 >= b_min in the last iteration) still
 * gets its weights; the caller checks the history.  A row that no phase centre sees (R <= r,
 * eqs. 4-5) gets count 0, zero outputs and an all-zero history.
 * Errors: as the workspace query; INVALID_ARG for window below the largest candidate count,
 * NULL or misaligned pointers; ROSAR_ERR_WORKSPACE for a short or misaligned workspace. */
rosar_status rosar_sas_design(const rosar_geometry* geom, const rosar_polar_grid* grid,
                              const rosar_sas_params* params, const double* delta_r, int32_t window,
                              int32_t* offsets, void* weights, int32_t* count, double* history,
                              void* workspace, size_t workspace_bytes, rosar_stream stream);

/* ---------------------------------------------------------------- autotune cache
 * The autotuners above (rosar_autotune_sparse_filter, rosar_sparse_plan_autotune,
 * rosar_batch_autotune) first look their key up in the library's autotune cache and return a
 * hit without timing anything; a miss is timed and stored.  A key is the device's architecture
 * name (e.g. "gfx950") and the shape class that decides the winning launch shape: pulses, rows
 * and their spacing, band layout and storage type, taps, window, weight type, interpolation
 * (plans also the candidate mask; batches a hash of every rotation's sizes).  The cache is
 * process-wide, behind one mutex, and mirrored to a JSON file:
 * {"<key>": {"variant": v, "pixels_per_lane": p, "waves": w, "us": t}, ...}.  A store rereads
 * the file, adds its entry and replaces the file through a temporary file and a rename, so
 * processes sharing a file keep each other's entries and readers never see a partial file.
 *
 * rosar_autotune selects the cache file (NULL: no file, entries kept in memory only) and loads
 * its entries; a missing or unparsable file reads as empty.  Without a call, the first cache
 * use takes the file named by the ROSAR_AUTOTUNE_CACHE environment variable, if set.  Host
 * only (no device work).  Errors: none (always ROSAR_OK). */
rosar_status rosar_autotune(const char* cache_path);
/* Looks `key` up: *found = 1 and the stored shape and time, or *found = 0.
 * Errors: INVALID_ARG for a NULL argument. */
rosar_status rosar_autotune_lookup(const char* key, rosar_tile* tile, float* us, int32_t* found);
/* Stores a result under `key` (and in the file, if one is selected).
 * Errors: INVALID_ARG for an empty or NULL key, a NULL tile, us < 0, or a file that cannot be
 * written (the entry is still kept in memory). */
rosar_status rosar_autotune_store(const char* key, const rosar_tile* tile, float us);

#ifdef __cplusplus
}
#endif
#endif /* ROSAR_H */
