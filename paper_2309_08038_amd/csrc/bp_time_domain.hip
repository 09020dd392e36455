// Conventional time-domain back-projection (the W_BP Hadamard sum of Sec. II-C, before range
// compression), the comparator the paper measures its method against:
//   I(R, phi_a) = sum over visible n of alpha_n exp(-j 2 k R_n)
//                 sum_m h[m] y[n, m] exp(-j 2 pi tau_n K m t_s),   tau_n = 2 R_n / c,
// with visibility and alpha as in the FFT+BPA kernel (eqs. 3-5, 8, 15).  A thread owns one
// pixel; the workgroup walks the pulses in order, so every lane reads the same windowed samples:
// blocks of kTdPulses pulses are staged in LDS and read as broadcasts, and only the ramp differs
// per lane.  Geometry is float64 per (pixel, pulse); the ramp exp(-j 2 pi f m) (f = 2 K R_n /
// (c F_s) cycles per sample) advances by float32 complex multiplies in eight interleaved streams
// and restarts every 64 samples from its float64-reduced exact value.
#include <hip/hip_runtime.h>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kTdThreads = 256;
constexpr int kTdPulses = 4;      // pulses staged per block
constexpr int kTdReseed = 64;     // ramp restart interval (samples)
constexpr int kTdStreams = 8;     // interleaved ramps per segment (kTdReseed is a multiple)

__global__ __launch_bounds__(kTdThreads) void bp_time_domain_kernel(Geo g, int m_fast, double cyc_per_m,
                                                                    const float2* __restrict__ raw,
                                                                    const float* __restrict__ window,
                                                                    const double* __restrict__ angles, int row_first,
                                                                    int tiles, float2* __restrict__ image) {
  extern __shared__ float2 s_hy[];   // kTdPulses windowed pulses of m_fast samples
  const int row_local = blockIdx.x / tiles;
  const int a = (blockIdx.x % tiles) * kTdThreads + threadIdx.x;
  const int n_p = g.n;
  const bool valid = a < n_p;
  const double rr = g.r0 + (row_first + row_local) * g.dr;
  const double phi_a = g.phi0 + a * g.step;
  const double two_pi = 6.283185307179586476925286766559;
  float2 acc = make_float2(0.f, 0.f);
  for (int nb = 0; nb < n_p; nb += kTdPulses) {
    const int cnt = min(kTdPulses, n_p - nb);
    __syncthreads();   // the previous block's samples are no longer read
    for (int i = threadIdx.x; i < cnt * m_fast; i += kTdThreads) {
      const int p = i / m_fast, m = i - p * m_fast;
      float2 y = raw[(int64_t)(nb + p) * m_fast + m];
      const float w = window ? window[m] : 1.f;
      s_hy[i] = make_float2(y.x * w, y.y * w);
    }
    __syncthreads();
    for (int p = 0; p < cnt; ++p) {
      const int n = nb + p;
      const double phi_n = angles ? angles[n] : g.phi0 + n * g.step;
      double d = phi_a - phi_n;
      d -= two_pi * rint(d / two_pi);   // wrapped to [-pi, pi]
      const double cd = cos(d);
      const double v = rr * cd - g.radius;
      if (!valid || v <= 0.0) continue;   // outside the field of view (eqs. 4-5)
      const double rn = sqrt(rr * rr + g.radius * g.radius - 2.0 * rr * g.radius * cd);
      const double f = rn * cyc_per_m;   // beat frequency, cycles per sample
      const float fr = (float)(f - rint(f));
      float ss, cs;
      sincospif(-2.0f * fr, &ss, &cs);
      const float2 step = make_float2(cs, ss);
      const float2* hy = s_hy + p * m_fast;
      // kTdStreams interleaved ramps (samples m0 + s + kTdStreams i) so that the complex
      // multiplies of the recurrence form independent chains
      float2 sum[kTdStreams];
#pragma unroll
      for (int q = 0; q < kTdStreams; ++q) sum[q] = make_float2(0.f, 0.f);
      const double fs = f * kTdStreams;
      sincospif(-2.0f * (float)(fs - rint(fs)), &ss, &cs);
      const float2 stride = make_float2(cs, ss);   // exp(-j 2 pi f kTdStreams)
      for (int m0 = 0; m0 < m_fast; m0 += kTdReseed) {
        float2 ramp[kTdStreams];
        const double q0 = f * m0;
        sincospif(-2.0f * (float)(q0 - rint(q0)), &ss, &cs);
        ramp[0] = make_float2(cs, ss);
#pragma unroll
        for (int q = 1; q < kTdStreams; ++q) ramp[q] = cmul(ramp[q - 1], step);
        const int m1 = min(m0 + kTdReseed, m_fast);
        if (m1 - m0 == kTdReseed) {
          for (int m = m0; m < m1; m += kTdStreams) {
#pragma unroll
            for (int q = 0; q < kTdStreams; ++q) {
              const float2 y = hy[m + q];
              sum[q].x = fmaf(y.x, ramp[q].x, fmaf(-y.y, ramp[q].y, sum[q].x));
              sum[q].y = fmaf(y.x, ramp[q].y, fmaf(y.y, ramp[q].x, sum[q].y));
              ramp[q] = cmul(ramp[q], stride);
            }
          }
        } else {   // the last, partial segment: one sample at a time
          float2 r = ramp[0];
          for (int m = m0; m < m1; ++m) {
            const float2 y = hy[m];
            sum[0].x = fmaf(y.x, r.x, fmaf(-y.y, r.y, sum[0].x));
            sum[0].y = fmaf(y.x, r.y, fmaf(y.y, r.x, sum[0].y));
            r = cmul(r, step);
          }
        }
      }
#pragma unroll
      for (int q = 1; q < kTdStreams; ++q) {
        sum[0].x += sum[q].x;
        sum[0].y += sum[q].y;
      }
      // alpha exp(-j 2 k R_n): the carrier phase in revolutions, reduced in float64
      const double rev = rn * g.k_over_pi;
      sincospif(-2.0f * (float)(rev - rint(rev)), &ss, &cs);
      const float al = (float)(v / rn);
      const float2 c = make_float2(al * cs, al * ss);
      acc.x += c.x * sum[0].x - c.y * sum[0].y;
      acc.y += c.x * sum[0].y + c.y * sum[0].x;
    }
  }
  if (valid) image[(size_t)row_local * n_p + a] = acc;
}

// The sparse-aperture filter on the raw samples (the W_SA compensation of Sec. II-C followed by
// the weights):  I[r, a] = sum_k conj(w[r, k]) sum_m h[m] y[(a + o_k) mod N, m]
// exp(-j 2 pi f_k m), f_k = 2 K R(o_k 2 pi / N) / (c F_s).  The ramp of a tap is the same for
// every pixel of the row; each lane reads its own pulse (a + o_k), from global memory.
__global__ __launch_bounds__(kTdThreads) void sas_time_domain_kernel(Geo g, int m_fast, double cyc_per_m,
                                                                     const float2* __restrict__ raw,
                                                                     const float* __restrict__ window,
                                                                     const int32_t* __restrict__ offsets,
                                                                     const float2* __restrict__ weights, int k,
                                                                     int half_w, int row_first, int tiles,
                                                                     float2* __restrict__ image) {
  extern __shared__ float s_win[];   // the range window (1 for rect)
  const int row_local = blockIdx.x / tiles;
  const int row = row_first + row_local;
  const int a = (blockIdx.x % tiles) * kTdThreads + threadIdx.x;
  const int n_p = g.n;
  for (int m = threadIdx.x; m < m_fast; m += kTdThreads) s_win[m] = window ? window[m] : 1.f;
  __syncthreads();
  if (a >= n_p) return;   // no barrier below
  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  float2 acc = make_float2(0.f, 0.f);
  for (int t = 0; t < k; ++t) {
    const int o = offsets[(int64_t)row * k + t];
    if (o < -half_w || o >= half_w) continue;   // outside the window: no contribution
    const float2 w = weights[(int64_t)row * k + t];
    int n = a + o;
    n += n < 0 ? n_p : 0;
    n -= n >= n_p ? n_p : 0;
    const double f = sqrt(c1 - c2 * cos(o * g.step)) * cyc_per_m;   // beat frequency (eq. 2)
    float ss, cs;
    sincospif(-2.0f * (float)(f - rint(f)), &ss, &cs);
    const float2 step = make_float2(cs, ss);
    const double fs = f * kTdStreams;
    sincospif(-2.0f * (float)(fs - rint(fs)), &ss, &cs);
    const float2 stride = make_float2(cs, ss);
    const float2* y = raw + (int64_t)n * m_fast;
    float2 sum[kTdStreams];
#pragma unroll
    for (int q = 0; q < kTdStreams; ++q) sum[q] = make_float2(0.f, 0.f);
    for (int m0 = 0; m0 < m_fast; m0 += kTdReseed) {
      float2 ramp[kTdStreams];
      const double q0 = f * m0;
      sincospif(-2.0f * (float)(q0 - rint(q0)), &ss, &cs);
      ramp[0] = make_float2(cs, ss);
#pragma unroll
      for (int q = 1; q < kTdStreams; ++q) ramp[q] = cmul(ramp[q - 1], step);
      const int m1 = min(m0 + kTdReseed, m_fast);
      if (m1 - m0 == kTdReseed) {
        for (int m = m0; m < m1; m += kTdStreams) {
#pragma unroll
          for (int q = 0; q < kTdStreams; ++q) {
            const float2 yv = y[m + q];
            const float hw = s_win[m + q];
            const float yx = yv.x * hw, yy = yv.y * hw;
            sum[q].x = fmaf(yx, ramp[q].x, fmaf(-yy, ramp[q].y, sum[q].x));
            sum[q].y = fmaf(yx, ramp[q].y, fmaf(yy, ramp[q].x, sum[q].y));
            ramp[q] = cmul(ramp[q], stride);
          }
        }
      } else {   // the last, partial segment
        float2 r = ramp[0];
        for (int m = m0; m < m1; ++m) {
          const float2 yv = y[m];
          const float yx = yv.x * s_win[m], yy = yv.y * s_win[m];
          sum[0].x = fmaf(yx, r.x, fmaf(-yy, r.y, sum[0].x));
          sum[0].y = fmaf(yx, r.y, fmaf(yy, r.x, sum[0].y));
          r = cmul(r, step);
        }
      }
    }
#pragma unroll
    for (int q = 1; q < kTdStreams; ++q) {
      sum[0].x += sum[q].x;
      sum[0].y += sum[q].y;
    }
    cmac_conj(acc, w, sum[0]);   // acc += conj(w) * sum (eq. 43)
  }
  image[(size_t)row_local * n_p + a] = acc;
}

}  // namespace

hipError_t launch_sas_time_domain(const Geo& g, int m_fast, double cyc_per_m, const float2* raw, const float* window,
                                  const int32_t* offsets, const float2* weights, int k, int window_w, int row_first,
                                  int row_count, float2* image, hipStream_t s) {
  const int tiles = (g.n + kTdThreads - 1) / kTdThreads;
  sas_time_domain_kernel<<<row_count * tiles, kTdThreads, (size_t)m_fast * sizeof(float), s>>>(
      g, m_fast, cyc_per_m, raw, window, offsets, weights, k, window_w / 2, row_first, tiles, image);
  return hipGetLastError();
}

hipError_t launch_bp_time_domain(const Geo& g, int m_fast, double cyc_per_m, const float2* raw, const float* window,
                                 const double* angles, int row_first, int row_count, float2* image, hipStream_t s) {
  const int tiles = (g.n + kTdThreads - 1) / kTdThreads;
  const size_t lds = (size_t)kTdPulses * m_fast * sizeof(float2);
  bp_time_domain_kernel<<<row_count * tiles, kTdThreads, lds, s>>>(g, m_fast, cyc_per_m, raw, window, angles,
                                                                   row_first, tiles, image);
  return hipGetLastError();
}

}  // namespace rosar
