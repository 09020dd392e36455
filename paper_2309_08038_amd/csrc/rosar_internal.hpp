// Internal declarations shared by the host-side API and the HIP kernels of librosar.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/rosar.h"

namespace rosar {

// Derived geometry, computed on the host in float64 and passed by value to the kernels.
struct Geo {
  int32_t n;          // pulses per rotation N (== azimuth bins)
  int32_t n_range;    // grid rows
  double radius;      // r
  double r0, dr;      // R_i = r0 + i * dr
  double beta;        // FFT bins per metre of slant range (eq. 40)
  double kw;          // wavenumber k (after eq. 12)
  double k_over_pi;   // k / pi: revolutions of exp(j 2 k R) per metre
  double step;        // 2 pi / N
  double phi0;
};

// Range-compressed data as stored by rosar_range_compress (see rosar_rc_view).
struct View {
  const void* data;
  int64_t ld;
  int32_t l_lo, l_count, halo, dtype;
  float inv_scale;
};

struct RcArgs {
  const float2* raw;
  const float* window;
  void* out;
  int64_t ld;
  int32_t n, m, l, l_lo, l_count, halo, dtype;
  float scale;
};

struct SparseArgs {
  Geo g;
  View y;
  const int32_t* offsets;
  const void* weights;
  int32_t k, window, w_dtype, interp;
  const float* dphi;
  const float* dpsi;
  float2* image;
};

struct Tile {
  int variant, ppl, waves;
};

// Cartesian target lattice: x = x0 + ix dx, y = y0 + iy dy.
struct CartGrid {
  int32_t nx, ny;
  double x0, y0, dx, dy;
};

// Launchers (kernels live in the .hip files).  Each returns hipGetLastError() after launching.
// Range compression: power-of-two L in [64, 2048] by the radix-8/4/2 wave kernels, any other
// 2^a 3^b 5^c <= 8192 by the mixed-radix workgroup kernel.
bool range_compress_length_supported(int32_t l);
hipError_t launch_range_compress(const RcArgs& a, hipStream_t s);
hipError_t launch_sparse_plain(const SparseArgs& a, const Tile& t, hipStream_t s);
hipError_t launch_sparse_corrected(const SparseArgs& a, hipStream_t s);
hipError_t launch_sparse_cartesian(const SparseArgs& a, const CartGrid& c, hipStream_t s);
hipError_t launch_sparse_polar(const SparseArgs& a, int32_t n_az, hipStream_t s);
hipError_t launch_bp_cartesian(const Geo& g, const View& y, const CartGrid& c, const double* angles, int32_t interp,
                               float2* image, hipStream_t s);
size_t bp_workspace_bytes(int32_t n);
// Allocation-free back-projection: the workspace is a file-scope device array sized for at most
// kBpNoAllocMaxPulses pulses; bp_scratch gives its address on the current device.
constexpr int32_t kBpNoAllocMaxPulses = 1 << 16;
hipError_t bp_scratch(void** out);
hipError_t launch_sas_time_domain(const Geo& g, int m_fast, double cyc_per_m, const float2* raw, const float* window,
                                  const int32_t* offsets, const float2* weights, int k, int window_w, int row_first,
                                  int row_count, float2* image, hipStream_t s);
hipError_t launch_delta_r(const Geo& g, int window, int n_samples, const double* deltas, int rank, double* samples,
                          double* delta_r, hipStream_t s);
int delta_r_rows_per_block();
hipError_t launch_beampattern(const Geo& g, int k, int window, const int32_t* offsets, const float2* weights,
                              const double* angles, int n_ang, const double* delta_r, double* pattern,
                              double* summary, hipStream_t s);
hipError_t launch_bp_time_domain(const Geo& g, int m_fast, double cyc_per_m, const float2* raw, const float* window,
                                 const double* angles, int row_first, int row_count, float2* image, hipStream_t s);
hipError_t launch_bp_full(const Geo& g, const View& y, const double* angles, int32_t interp,
                          float2* image, void* ws, hipStream_t s);
size_t backward_workspace_bytes(int32_t n, int32_t n_range, int32_t k);
hipError_t launch_sparse_backward(const SparseArgs& a, const float2* grad_image, float2* grad_w,
                                  float* grad_dphi, float* grad_dpsi, void* ws, hipStream_t s);

// Thread-local error of the C ABI (rosar_last_error) and the per-rotation checks of batch plans.
rosar_status set_error(rosar_status st, const std::string& msg);
void clear_error();
rosar_status validate_rotation(const rosar_rotation_desc& d, int index);
Geo geo_of(const rosar_geometry* g, const rosar_polar_grid* p);

// Sparse-filter plans: the LDS layout a plan fixes, the kernel that writes every row's tap table
// (row_bytes each) and the filter launch that copies them into LDS.
struct PlanLayout {
  int ppl, waves;
  int rows_cap, stride, shift, row_bytes;
  double cos_hw;
  size_t lds_bytes;
};
bool plan_shape_supported(int ppl, int waves);
bool sparse_plan_layout(const SparseArgs& a, int ppl, int waves, PlanLayout* out);
hipError_t launch_tap_tables(const SparseArgs& a, const PlanLayout& pl, char* tabs, hipStream_t s);
hipError_t launch_sparse_planned(const SparseArgs& a, const PlanLayout& pl, const char* tabs, hipStream_t s);

// Azimuth fast convolution (plans of variant 3): the radix sequence of the azimuth FFT length,
// the per-row tap-list layout, the plan's kernels (tap lists, then the spectrum of every (range
// row, bin row) pair's sparse kernel) and the two kernels of a run (band-row spectra, then one
// workgroup per range row).
constexpr int kFftMaxPasses = 16;
struct FftFactors {
  int32_t n, n_pass;
  int32_t radix[kFftMaxPasses];
};
struct FcLayout {
  FftFactors f;
  int ne, row_bytes;   // entries per row (K or 2K) and bytes of a row's block
  int rows_cap;        // bin rows one range row may touch (at most 32)
  double cos_hw;
  size_t lds_bytes;
};
bool fft_factors(int n, FftFactors* out);   // n = 2^a 3^b 5^c <= 8192 (radix 8, 4, 2, 5, 3 passes)
bool fc_layout(const SparseArgs& a, FcLayout* out);
bool fc_tap_layout(const SparseArgs& a, FcLayout* out);   // tap-list fields only (any N)

// Adjoint of the plain sparse filter with respect to the band (per band row, a gather over the
// range rows whose taps read it): tap lists in the workspace, then the gather.
size_t adjoint_band_workspace_bytes(const FcLayout& L, int32_t n_range);
hipError_t launch_adjoint_band(const SparseArgs& a, const FcLayout& L, const float2* grad_image, float2* grad_band,
                               void* ws, hipStream_t s);
size_t fc_spectrum_bytes(const SparseArgs& a);
int fc_twiddle_count(int n);
void fc_twiddles(int n, float2* host_tw);   // fc_twiddle_count(n) entries
// hdr_out (may be NULL): each row's header {lfirst, bin mask, ne, 0}, for the host
hipError_t launch_fc_tables(const SparseArgs& a, const FcLayout& L, char* tabs, int* bad, int4* hdr_out, hipStream_t s);
hipError_t launch_fc_kernel_spectra(const FcLayout& L, const char* tabs, const int2* pairs, int n_pairs,
                                   const float2* tw, float2* gspec, hipStream_t s);
// first_pair[row]: index of the row's first kernel spectrum in gspec
hipError_t launch_fc_run(const SparseArgs& a, const FcLayout& L, const char* tabs, const int* first_pair,
                         const float2* tw, float2* spec, const float2* gspec, hipStream_t s);

// Tile chosen when the caller leaves it to the library.
Tile default_tile(int32_t n, int32_t y_dtype);
bool tile_supported(const Tile& t);

// Robust sparse-array synthesis (Algorithm 1): per-bin candidate and side-lobe counts decide
// the workspace layout (a uniform stride per bin).
using SasDesignParams = rosar_sas_params;
struct SasSizes {
  int n_max, s_max;     // most candidates / side-lobe directions of any bin
  size_t stride, bytes; // workspace bytes per bin and in all
};
SasSizes sas_sizes(const Geo& g, const SasDesignParams& p);
hipError_t launch_sas_design(const Geo& g, const SasDesignParams& p, const double* delta_r, const SasSizes& z,
                             void* ws, int32_t window, int32_t* offsets, float2* weights, int32_t* count,
                             double* hist, hipStream_t s);

// Autotune cache (rosar_autotune): results keyed by GPU architecture and shape class, behind one
// mutex, mirrored to the selected JSON file.  put returns false if the file cannot be written.
bool tune_cache_get(const std::string& key, rosar_tile* tile, float* us);
bool tune_cache_put(const std::string& key, const rosar_tile& tile, float us);
std::string tune_arch();   // the current device's architecture name, e.g. "gfx950"

}  // namespace rosar
