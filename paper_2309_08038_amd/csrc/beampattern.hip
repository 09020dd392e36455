// Beampattern of the sparse weights and the worst-case robust check of the weight design
// (Sec. III-A: eq. 16, the constraints C1 and C2 of eq. 20 and their worst-case forms): for range
// row R and a target at angle phi from the pixel's direction, tap k (pulse a + o_k) sees it at
// D_k = phi - o_k phi_Delta, so
//   P(R, phi) = | sum_k conj(w_k) alpha(D_k) exp(+j 2 k R(D_k)) | = |w^H a(phi; R)|,
// R(D) from eq. 2 and alpha = max(R cos D - r, 0) / R(D).  Taps outside the window contribute
// nothing, as in the filter.  A thread owns one (row, angle) and sums the taps in float64, with
// the carrier phase reduced in revolutions before its sine and cosine.  The summary takes angle
// index 0 as the main-lobe direction and the others as side-lobe directions: per row
// {P_main, max P_side, (max P_side + Delta_R)^2 / (P_main - Delta_R)^2} (+inf when
// P_main <= Delta_R), the worst case over array errors of norm <= Delta_R for a unit-norm w.
#include <hip/hip_runtime.h>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kBpatThreads = 256;

__global__ __launch_bounds__(kBpatThreads) void beampattern_kernel(Geo g, int k, int half_w,
                                                                   const int32_t* __restrict__ offsets,
                                                                   const float2* __restrict__ weights,
                                                                   const double* __restrict__ angles, int n_ang,
                                                                   double* __restrict__ pattern) {
  const int j = blockIdx.x * kBpatThreads + threadIdx.x;
  const int row = blockIdx.y;
  if (j >= n_ang) return;   // no barrier in this kernel
  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  const double phi = angles[j];
  double ax = 0.0, ay = 0.0;
  for (int t = 0; t < k; ++t) {
    const int o = offsets[(int64_t)row * k + t];
    if (o < -half_w || o >= half_w) continue;   // outside the window: no contribution
    const float2 w = weights[(int64_t)row * k + t];
    const double cd = cos(phi - o * g.step);
    const double rn = sqrt(c1 - c2 * cd);
    const double al = fmax(rr * cd - g.radius, 0.0) / rn;
    const double rev = rn * g.k_over_pi;   // exp(+j 2 k R) (eq. 16) in revolutions
    double s, c;
    sincospi(2.0 * (rev - rint(rev)), &s, &c);
    const double ex = al * c, ey = al * s;
    // conj(w) * a
    ax += (double)w.x * ex + (double)w.y * ey;
    ay += (double)w.x * ey - (double)w.y * ex;
  }
  pattern[(int64_t)row * n_ang + j] = sqrt(ax * ax + ay * ay);
}

__global__ __launch_bounds__(kBpatThreads) void robust_summary_kernel(const double* __restrict__ pattern, int n_ang,
                                                                      const double* __restrict__ delta_r,
                                                                      double* __restrict__ summary) {
  __shared__ double s_max[kBpatThreads / kWave];
  const int row = blockIdx.x;
  const double* p = pattern + (int64_t)row * n_ang;
  double m = 0.0;   // patterns are >= 0
  for (int j = 1 + threadIdx.x; j < n_ang; j += kBpatThreads) m = fmax(m, p[j]);
  for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & (kWave - 1)) == 0) s_max[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double side = 0.0;
    for (int i = 0; i < kBpatThreads / kWave; ++i) side = fmax(side, s_max[i]);
    const double main = p[0];
    const double d = delta_r ? delta_r[row] : 0.0;
    const double lo = main - d, hi = side + d;
    summary[(int64_t)row * 3 + 0] = main;
    summary[(int64_t)row * 3 + 1] = side;
    summary[(int64_t)row * 3 + 2] = lo > 0.0 ? (hi * hi) / (lo * lo) : __builtin_inf();
  }
}

}  // namespace

hipError_t launch_beampattern(const Geo& g, int k, int window, const int32_t* offsets, const float2* weights,
                              const double* angles, int n_ang, const double* delta_r, double* pattern,
                              double* summary, hipStream_t s) {
  const dim3 grid((n_ang + kBpatThreads - 1) / kBpatThreads, g.n_range);
  beampattern_kernel<<<grid, kBpatThreads, 0, s>>>(g, k, window / 2, offsets, weights, angles, n_ang, pattern);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  robust_summary_kernel<<<g.n_range, kBpatThreads, 0, s>>>(pattern, n_ang, delta_r, summary);
  return hipGetLastError();
}

}  // namespace rosar
