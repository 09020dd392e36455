// Azimuth fast convolution of the sparse-aperture filter (Algorithm 2 with eq. 43, no angle or
// phase errors).  Under the rotation symmetry the taps of range row r form, for each bin row l
// they touch, a sparse kernel g_{r,l}[o] = sum of conj(w) (times the LINEAR fraction) over the
// taps with offset o and bin l, and
//   I[r, a] = sum_l sum_o g_{r,l}[o] Y_l[(a + o) mod N],
// a circular correlation along azimuth.  With Yhat_l the DFT of band row l and
// G_{r,l}[m] = sum_o g_{r,l}[o] exp(+j 2 pi o m / N),
//   I[r, .] = IDFT( sum_l G_{r,l} * Yhat_l ).
// The sparse kernels, hence the G_{r,l}, depend on the filter design alone: a plan builds the
// tap lists (the bins come from the same float64 expression, eq. 2 and eq. 40, as the direct
// filter's tap tables) and then G for every (range row, bin row) pair, one workgroup per pair
// scattering the kernel into LDS and transforming it.  A run computes Yhat for every band row
// (one workgroup per row), then one workgroup per range row accumulates the products G * Yhat
// in registers and transforms the sum back.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mixed_fft.hpp"
#include "sparse_device.hpp"

namespace rosar {
namespace {

using mfft::kFftMaxN;
using mfft::kFftThreads;

constexpr int kFcMaxRows = 32;   // bin rows one range row may touch (a 32-bit mask)
constexpr int kFcMaxQ = (kFftMaxN + kFftThreads - 1) / kFftThreads;

// Row block: int4 header {lfirst, bin mask, ne, 0}, then ne entries
// int4 {azimuth index (o mod N), bin row - lfirst (-1: no contribution), coef.x, coef.y}.  The
// header also goes to hdr_out[row] (when given) for the host, which numbers the row's G spectra
// (one per mask bit in bit order) and uploads each row's first pair index as an array of its own.
template <int WDT, int INTERP>
__global__ __launch_bounds__(256) void fc_table_kernel(Geo g, View y, int32_t k, int32_t window, int rows_cap,
                                                       double cos_hw, const int32_t* __restrict__ offsets,
                                                       const void* __restrict__ weights, char* __restrict__ tabs,
                                                       int row_bytes, int* __restrict__ bad, int4* __restrict__ hdr_out) {
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  const int row = blockIdx.x;
  const int half_w = window / 2;
  int4* blk = reinterpret_cast<int4*>(tabs + (size_t)row * row_bytes);
  const sparse::RowSpan sp = sparse::row_span<INTERP>(g, y, row, rows_cap, cos_hw);
  __shared__ unsigned s_mask;
  __shared__ int s_bad;
  if (threadIdx.x == 0) {
    s_mask = 0u;
    s_bad = 0;
  }
  __syncthreads();
  const int64_t wrow = (int64_t)row * k;
  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    const int o = offsets[wrow + t];
    const float2 w = load_w<WDT>(weights, wrow + t);
    const bool inwin = o >= -half_w && o < half_w;
    int l = 0;
    float f = 0.f;
    if (inwin) {
      const double u = g.beta * sqrt(c1 - c2 * cos(o * g.step));
      l = sparse::tap_bin<INTERP>(u, g, rr, o) - y.l_lo;
      if constexpr (INTERP == ROSAR_LINEAR) f = (float)(u - floor(u));
    }
    const int pos = inwin ? (o < 0 ? o + g.n : o) : 0;
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      const int ls = l + s;
      const bool ok = inwin && ls >= 0 && ls < y.l_count;
      const int rel = ls - sp.lfirst;
      const bool in_mask = ok && rel >= 0 && rel < kFcMaxRows;
      if (ok && !in_mask) atomicOr(&s_bad, 1);
      if (in_mask) atomicOr(&s_mask, 1u << rel);
      const float fs = INTERP == ROSAR_NEAREST ? 1.f : (s == 0 ? 1.f - f : f);
      // the filter applies conj(w) (eq. 43)
      blk[1 + t * NSUB + s] = make_int4(pos, in_mask ? rel : -1, __float_as_int(w.x * fs), __float_as_int(-w.y * fs));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    blk[0] = make_int4(sp.lfirst, (int)s_mask, k * NSUB, 0);
    if (hdr_out) hdr_out[row] = blk[0];
    if (s_bad) atomicOr(bad, 1);
  }
}

// Yhat_l = DFT of band row l over the N pulses (the stored halo copies are not read).
template <int DT>
__global__ __launch_bounds__(kFftThreads) void fc_spectrum_kernel(View y, FftFactors f, const float2* __restrict__ tw,
                                                                  float2* __restrict__ spec) {
  extern __shared__ float2 buf[];   // [n] row, then the twiddle tables (all dynamic LDS)
  const int l = blockIdx.x;
  const int n = f.n;
  const int tid = threadIdx.x;
  mfft::Twiddles& s_tw = *reinterpret_cast<mfft::Twiddles*>(buf + n);
  const int64_t row = (int64_t)l * y.ld + y.halo;
  mfft::load_twiddles(s_tw, tw, n, tid);
  for (int i = tid; i < n; i += kFftThreads) buf[i] = load_c<DT>(y.data, row + i);
  __syncthreads();
  mfft::block_fft<-1>(buf, f, s_tw, tid);
  float2* out = spec + (size_t)l * n;
  for (int i = tid; i < n; i += kFftThreads) out[i] = buf[i];
}

// G of one (range row, bin row) pair: the row's entries on that bin row scattered into a
// zeroed LDS row (entries that share an azimuth index add up, as in the direct sum), then the
// unnormalised inverse-direction transform.  One thread adds the entries in table order, so a
// repeated azimuth index sums in a fixed order and every plan build gives the same bits (the
// scatter is K or 2K additions, once per plan).
__global__ __launch_bounds__(kFftThreads) void fc_kernel_spectra_kernel(FftFactors f, const char* __restrict__ tabs,
                                                                        int row_bytes, const int2* __restrict__ pairs,
                                                                        const float2* __restrict__ tw,
                                                                        float2* __restrict__ gspec) {
  extern __shared__ float2 buf[];   // [n] row, then the twiddle tables (all dynamic LDS)
  const int p = blockIdx.x;
  const int n = f.n;
  const int tid = threadIdx.x;
  mfft::Twiddles& s_tw = *reinterpret_cast<mfft::Twiddles*>(buf + n);
  const int2 pr = pairs[p];
  mfft::load_twiddles(s_tw, tw, n, tid);
  const int4* blk = reinterpret_cast<const int4*>(tabs + (size_t)pr.x * row_bytes);
  const int ne = blk[0].z;
  for (int i = tid; i < n; i += kFftThreads) buf[i] = make_float2(0.f, 0.f);
  __syncthreads();
  if (tid == 0) {
    for (int e = 0; e < ne; ++e) {
      const int4 t = blk[1 + e];
      if (t.y == pr.y) {
        buf[t.x].x += __int_as_float(t.z);
        buf[t.x].y += __int_as_float(t.w);
      }
    }
  }
  __syncthreads();
  mfft::block_fft<+1>(buf, f, s_tw, tid);
  float2* out = gspec + (size_t)p * n;
  for (int i = tid; i < n; i += kFftThreads) out[i] = buf[i];
}

// One range row: I[r, .] = IDFT(sum over the row's bin rows of G_{r,l} * Yhat_l).
__global__ __launch_bounds__(kFftThreads) void fc_rows_kernel(FftFactors f, int n_range, const char* __restrict__ tabs,
                                                              int row_bytes, const int* __restrict__ first_pair,
                                                              const float2* __restrict__ tw,
                                                              const float2* __restrict__ spec,
                                                              const float2* __restrict__ gspec, float inv_scale,
                                                              float2* __restrict__ image) {
  extern __shared__ float2 buf[];   // [n] row, then the twiddle tables (all dynamic LDS)
  const int row = xcd_logical_block(blockIdx.x, n_range);
  const int n = f.n;
  const int tid = threadIdx.x;
  mfft::Twiddles& s_tw = *reinterpret_cast<mfft::Twiddles*>(buf + n);
  mfft::load_twiddles(s_tw, tw, n, tid);
  const int4 hdr = reinterpret_cast<const int4*>(tabs + (size_t)row * row_bytes)[0];
  const int lfirst = hdr.x;
  unsigned mask = (unsigned)hdr.y;
  const float2* gp = gspec + (size_t)first_pair[row] * n;

  float2 acc[kFcMaxQ];
#pragma unroll
  for (int q = 0; q < kFcMaxQ; ++q) acc[q] = make_float2(0.f, 0.f);
  while (mask) {
    const int rel = __builtin_ctz(mask);
    mask &= mask - 1u;
    const float2* sp = spec + (size_t)(lfirst + rel) * n;
#pragma unroll
    for (int q = 0; q < kFcMaxQ; ++q) {
      const int i = tid + q * kFftThreads;
      if (i < n) {
        const float2 gv = gp[i], yv = sp[i];
        acc[q].x = fmaf(gv.x, yv.x, fmaf(-gv.y, yv.y, acc[q].x));
        acc[q].y = fmaf(gv.x, yv.y, fmaf(gv.y, yv.x, acc[q].y));
      }
    }
    gp += n;
  }
#pragma unroll
  for (int q = 0; q < kFcMaxQ; ++q) {
    const int i = tid + q * kFftThreads;
    if (i < n) buf[i] = acc[q];
  }
  __syncthreads();
  mfft::block_fft<+1>(buf, f, s_tw, tid);
  const float s = inv_scale / (float)n;
  float2* out = image + (size_t)row * n;
  for (int i = tid; i < n; i += kFftThreads) out[i] = make_float2(buf[i].x * s, buf[i].y * s);
}

template <int WDT, int INTERP>
hipError_t launch_tables_t(const SparseArgs& a, const FcLayout& L, char* tabs, int* bad, int4* hdr_out, hipStream_t s) {
  fc_table_kernel<WDT, INTERP><<<a.g.n_range, 256, 0, s>>>(a.g, a.y, a.k, a.window, L.rows_cap, L.cos_hw, a.offsets,
                                                          a.weights, tabs, L.row_bytes, bad, hdr_out);
  return hipGetLastError();
}

}  // namespace

bool fc_tap_layout(const SparseArgs& a, FcLayout* out) {
  const int rows = sparse::staged_rows_bound(a.g, a.g.n_range, a.window, a.interp, a.y.l_count);
  if (rows > kFcMaxRows) return false;
  const int nsub = a.interp == ROSAR_LINEAR ? 2 : 1;
  out->ne = a.k * nsub;
  out->row_bytes = 16 * (1 + out->ne);
  out->rows_cap = kFcMaxRows;
  out->cos_hw = cos((a.window / 2) * a.g.step);
  return true;
}

bool fft_factors(int n, FftFactors* out) {
  if (n < 2 || n > kFftMaxN) return false;
  FftFactors f{};
  f.n = n;
  int rem = n;
  for (int r : {8, 4, 2, 5, 3}) {
    while (rem % r == 0) {
      if (f.n_pass == kFftMaxPasses) return false;
      f.radix[f.n_pass++] = r;
      rem /= r;
    }
  }
  if (rem != 1) return false;
  *out = f;
  return true;
}

bool fc_layout(const SparseArgs& a, FcLayout* out) {
  FftFactors f{};
  if (!fft_factors(a.g.n, &f)) return false;
  if (!fc_tap_layout(a, out)) return false;
  out->f = f;
  out->lds_bytes = (size_t)a.g.n * sizeof(float2) + sizeof(mfft::Twiddles);
  return true;
}

size_t fc_spectrum_bytes(const SparseArgs& a) { return (size_t)a.y.l_count * (size_t)a.g.n * sizeof(float2); }

int fc_twiddle_count(int n) { return mfft::twiddle_count(n); }

void fc_twiddles(int n, float2* host_tw) {
  const double two_pi = 6.283185307179586476925286766559;
  const int cnt = mfft::twiddle_count(n);
  for (int i = 0; i < cnt; ++i) {
    const int t = i < mfft::kTwLo ? i : (i - mfft::kTwLo) * mfft::kTwLo;
    const double ang = two_pi * (double)t / (double)n;
    host_tw[i] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
  }
}

hipError_t launch_fc_tables(const SparseArgs& a, const FcLayout& L, char* tabs, int* bad, int4* hdr_out, hipStream_t s) {
  const bool lin = a.interp == ROSAR_LINEAR;
  if (a.w_dtype == ROSAR_C64)
    return lin ? launch_tables_t<0, ROSAR_LINEAR>(a, L, tabs, bad, hdr_out, s)
               : launch_tables_t<0, ROSAR_NEAREST>(a, L, tabs, bad, hdr_out, s);
  return lin ? launch_tables_t<1, ROSAR_LINEAR>(a, L, tabs, bad, hdr_out, s)
             : launch_tables_t<1, ROSAR_NEAREST>(a, L, tabs, bad, hdr_out, s);
}

hipError_t launch_fc_kernel_spectra(const FcLayout& L, const char* tabs, const int2* pairs, int n_pairs,
                                   const float2* tw, float2* gspec, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  fc_kernel_spectra_kernel<<<n_pairs, kFftThreads, L.lds_bytes, s>>>(L.f, tabs, L.row_bytes, pairs, tw, gspec);
  return hipGetLastError();
}

hipError_t launch_fc_run(const SparseArgs& a, const FcLayout& L, const char* tabs, const int* first_pair,
                         const float2* tw, float2* spec, const float2* gspec, hipStream_t s) {
  switch (a.y.dtype) {
    case ROSAR_C64: fc_spectrum_kernel<0><<<a.y.l_count, kFftThreads, L.lds_bytes, s>>>(a.y, L.f, tw, spec); break;
    case ROSAR_C16_F16: fc_spectrum_kernel<1><<<a.y.l_count, kFftThreads, L.lds_bytes, s>>>(a.y, L.f, tw, spec); break;
    default: fc_spectrum_kernel<2><<<a.y.l_count, kFftThreads, L.lds_bytes, s>>>(a.y, L.f, tw, spec); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fc_rows_kernel<<<a.g.n_range, kFftThreads, L.lds_bytes, s>>>(L.f, a.g.n_range, tabs, L.row_bytes, first_pair, tw,
                                                                spec, gspec, a.y.inv_scale, a.image);
  return hipGetLastError();
}

}  // namespace rosar
