// Monte-Carlo bound of the steering-vector error under rotation jitter (Sec. III-C, parameter
// settings, eq. 37): for every range row R and every draw s of the phase-centre angle errors,
//   D^_e = D_e + delta[e, s],  D_e = (e - W/2) 2 pi / N,
//   Delta^_R[s] = || a^(phi; R) - a(phi; R) ||,  a_e = alpha_e exp(+j 2 k R_e)  (eq. 16),
// and Delta_R is the order statistic of rank ceil(q S) - 1 of those S values (the 99 % point of
// their CDF for q = 0.99).  Each element adds (alpha^ - alpha)^2 + 4 alpha alpha^ sin^2(psi / 2),
// psi = 2 k (R^ - R), with R^ - R = 2 R r (cos D - cos D^) / (R^ + R): no difference of two
// nearly equal ranges or phases is ever formed, so float64 keeps its relative precision at
// millimetre wavelengths.  The per-draw terms sin(delta/2), cos(delta/2) depend on the draw only,
// and the per-row terms R_e, alpha_e on the row only: a workgroup owns 256 draws and kDrRows
// rows, evaluates each draw's trigonometry once for all its rows and reads the row terms from LDS.
#include <hip/hip_runtime.h>

#include "rosar_internal.hpp"

namespace rosar {
namespace {

constexpr int kDrThreads = 256;   // draws per workgroup (one per lane)
constexpr int kDrRows = 8;        // range rows per workgroup
constexpr int kDrChunk = 256;     // window elements whose row terms sit in LDS at once

__global__ __launch_bounds__(kDrThreads) void delta_r_samples_kernel(Geo g, int window, int n_samples,
                                                                     const double* __restrict__ deltas,
                                                                     double* __restrict__ samples) {
  __shared__ double s_rn[kDrRows][kDrChunk];   // R_e of each row
  __shared__ double s_al[kDrRows][kDrChunk];   // alpha_e of each row
  __shared__ double s_cd[kDrChunk], s_sd[kDrChunk];
  const int s = blockIdx.x * kDrThreads + threadIdx.x;
  const int row0 = blockIdx.y * kDrRows;
  const int rows = min(kDrRows, g.n_range - row0);
  const bool valid = s < n_samples;
  double acc[kDrRows];
#pragma unroll
  for (int i = 0; i < kDrRows; ++i) acc[i] = 0.0;
  for (int e0 = 0; e0 < window; e0 += kDrChunk) {
    const int cnt = min(kDrChunk, window - e0);
    __syncthreads();   // the previous chunk's row terms are no longer read
    if (threadIdx.x < cnt) {
      const int e = e0 + threadIdx.x;
      double sd, cd;
      sincos((e - window / 2) * g.step, &sd, &cd);
      s_cd[threadIdx.x] = cd;
      s_sd[threadIdx.x] = sd;
      for (int i = 0; i < rows; ++i) {
        const double rr = g.r0 + (row0 + i) * g.dr;
        const double rn = sqrt(rr * rr + g.radius * g.radius - 2.0 * rr * g.radius * cd);
        s_rn[i][threadIdx.x] = rn;
        s_al[i][threadIdx.x] = fmax(rr * cd - g.radius, 0.0) / rn;
      }
    }
    __syncthreads();
    if (!valid) continue;
    for (int j = 0; j < cnt; ++j) {
      const double d = deltas[(int64_t)(e0 + j) * n_samples + s];
      double sh, ch;
      sincos(0.5 * d, &sh, &ch);
      const double cd = s_cd[j], sd = s_sd[j];
      const double t1 = 2.0 * sh * sh;   // 1 - cos(delta)
      const double t2 = 2.0 * sh * ch;   // sin(delta)
      const double ch_hat = cd - (cd * t1 + sd * t2);   // cos(D + delta)
      const double q = cd * t1 + sd * t2;               // cos D - cos D^
#pragma unroll
      for (int i = 0; i < kDrRows; ++i) {
        if (i >= rows) break;
        const double rr = g.r0 + (row0 + i) * g.dr;
        const double rh = sqrt(rr * rr + g.radius * g.radius - 2.0 * rr * g.radius * ch_hat);
        const double rn = s_rn[i][j], al = s_al[i][j];
        // one reciprocal serves both quotients: alpha^ = v / R^ and psi / 2 = k 2 R r q / (R^ + R)
        const double sum = rh + rn;
        const double inv = 1.0 / (rh * sum);
        const double alh = fmax(rr * ch_hat - g.radius, 0.0) * sum * inv;
        const double half_psi = g.kw * 2.0 * rr * g.radius * q * rh * inv;
        const double sn = sin(half_psi);
        const double da = alh - al;
        acc[i] += da * da + 4.0 * al * alh * sn * sn;
      }
    }
  }
  if (!valid) return;
  for (int i = 0; i < rows; ++i) samples[(int64_t)(row0 + i) * n_samples + s] = sqrt(acc[i]);
}

// The order statistic of rank k among a row's S non-negative samples, by radix selection on their
// IEEE-754 bit patterns (which order non-negative doubles as unsigned integers): eight passes of
// an 8-bit digit, each counting in LDS the samples that share the digits chosen so far.
__global__ __launch_bounds__(kDrThreads) void delta_r_select_kernel(const double* __restrict__ samples,
                                                                    int n_samples, int rank,
                                                                    double* __restrict__ out) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ unsigned s_rank;
  const double* v = samples + (int64_t)blockIdx.x * n_samples;
  unsigned long long prefix = 0, mask = 0;
  unsigned k = (unsigned)rank;
  for (int shift = 56; shift >= 0; shift -= 8) {
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n_samples; i += kDrThreads) {
      const unsigned long long u = (unsigned long long)__double_as_longlong(v[i]);
      if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      // k < (samples matching the prefix), so some digit takes the running count past k
      unsigned cum = 0;
      int d = 0;
      for (; d < 255; ++d) {
        if (cum + hist[d] > k) break;
        cum += hist[d];
      }
      s_prefix = prefix | ((unsigned long long)d << shift);
      s_rank = k - cum;
    }
    __syncthreads();
    prefix = s_prefix;
    k = s_rank;
    mask |= 255ull << shift;
    __syncthreads();   // s_prefix and hist are rewritten in the next pass
  }
  if (threadIdx.x == 0) out[blockIdx.x] = __longlong_as_double((long long)prefix);
}

}  // namespace

hipError_t launch_delta_r(const Geo& g, int window, int n_samples, const double* deltas, int rank, double* samples,
                          double* delta_r, hipStream_t s) {
  const dim3 grid((n_samples + kDrThreads - 1) / kDrThreads, (g.n_range + kDrRows - 1) / kDrRows);
  delta_r_samples_kernel<<<grid, kDrThreads, 0, s>>>(g, window, n_samples, deltas, samples);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  delta_r_select_kernel<<<g.n_range, kDrThreads, 0, s>>>(samples, n_samples, rank, delta_r);
  return hipGetLastError();
}

int delta_r_rows_per_block() { return kDrRows; }

}  // namespace rosar
