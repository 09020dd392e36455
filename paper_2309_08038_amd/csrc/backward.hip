// Adjoint of the sparse filter with respect to the weights and the per-pulse angle and phase
// errors, for a real loss with grad_image = dL/dRe(I) + j dL/dIm(I):
//   grad_w[i,t]  = sum_a conj(g[i,a]) s(i,a,t)
//   grad_dphi[n] = sum_{i,t} Re(conj(g[i,a]) conj(w[i,t]) ds/d dphi_n),   a = (n - o_t) mod N
//   grad_dpsi[n] = sum_{i,t} Im(conj(g[i,a]) conj(w[i,t]) s)
//   ds/d dphi = rot (beta dY/du - j 2k Y) R_i r sin(D) / R^,  rot = exp(-j (2k (R^ - R_nom) + psi)).
// (Chain rule through eq. 2 and the eq.-40 bin position; dY/du is the LINEAR slope, zero for
// NEAREST.)
//
// Gather formulation, deterministic without atomics: a workgroup owns one range row and each
// thread owns pulses n (so the angle/phase terms of n stay in registers and the per-row
// contribution to grad_dphi[n] accumulates in that thread).  For each tap the thread visits
// pixel a = n - o_t, recomputes the sample and its derivative (indices are never stored), and
// feeds conj(g) s into a per-tap partial reduced across the wavefront and then across the
// waves in a fixed order.  The taps' nominal geometry (float64 bin of R_nom, R_nom, sin/cos of
// D0 = 2 pi o / N) and weights sit in an LDS table; per (pulse, tap) only the angle-error
// correction is evaluated in float32.  As in the corrected forward it is either the cubic
// Taylor polynomial of R(D0 + d) - R(D0) in d (and its derivative for dR^/dd), taken when the
// workgroup's fourth-derivative remainder bound at the rotation's largest |d| is below 1e-6 rad
// of carrier phase and 2^-20 bins, or otherwise the exact form without cancellation:
//   R^2 - R_nom^2 = 4 R r sin(D0 + d/2) sin(d/2),   R^ - R_nom = (R^2 - R_nom^2)/(R^ + R_nom),
// with the bin formed in float64 and the samples read through buffer loads (out-of-band rows
// read zero).  Row partials of grad_dphi/grad_dpsi go to the workspace; a two-stage reduction
// sums them over rows in a fixed order (groups of rows, then the groups).
#include <type_traits>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kBwThreads = 256;
constexpr int kBwWaves = kBwThreads / kWave;
constexpr int kBwPpt = 8;      // pulses per thread per pass
constexpr int kBwChunk = kBwThreads;   // taps per LDS table chunk
constexpr int kRedGroups = 32;         // row groups of the first reduction stage

// Nominal geometry and weight of one tap, 80 bytes.
struct alignas(16) BwTap {
  SplitBin u;     // band-relative bin beta * R_nom - l_lo (+ 1/2 for NEAREST), split
  float r2;       // R_nom^2
  float rnom;     // R_nom
  float sd, cd;   // sin, cos of D0
  float wr, wi;   // weight
  int32_t o;      // offset
  int32_t valid;  // offset inside the window
  float q1, q2, q3;   // Taylor coefficients at D0: R(D0 + d) - R_nom = d (q1 + d (q2 + d q3))
  float p2, p3;       // 2 q2, 3 q3: dR^/dd = q1 + d (p2 + d p3)
};

__device__ __forceinline__ float2 wave_sum(float2 v) {
  for (int off = kWave / 2; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  return v;
}

template <int DT, int INTERP>
__global__ __launch_bounds__(kBwThreads) void backward_row_kernel(
    Geo g, View y, int32_t k, int32_t window, int nblocks,
    const int32_t* __restrict__ offsets, const float2* __restrict__ weights,
    const float* __restrict__ dphi, const float* __restrict__ dpsi,
    const float2* __restrict__ gimg, const char* __restrict__ ydata,
    float2* __restrict__ grad_w, float* __restrict__ part_d, float* __restrict__ part_p) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr float kInv2Pi = 0.15915494309189533577f;
  extern __shared__ float2 s_gw[];   // [kBwWaves][k]: per-wave grad_w partials
  __shared__ BwTap s_tap[kBwChunk];
  __shared__ float s_red[kBwWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int row = xcd_logical_block(blockIdx.x, nblocks);
  const int n = g.n;
  const int half_w = window / 2;
  for (int t = threadIdx.x; t < k; t += kBwThreads)
    for (int w = 0; w < kBwWaves; ++w) s_gw[w * k + t] = make_float2(0.f, 0.f);

  const double rr = g.r0 + row * g.dr;
  // the series path when the remainder bound (see the corrected forward) holds at max |d|
  bool series = false;
  {
    float dmax = 0.f;
    if (dphi)
      for (int pn = threadIdx.x; pn < n; pn += kBwThreads) dmax = fmaxf(dmax, fabsf(dphi[pn]));
    for (int off = kWave / 2; off > 0; off >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, off));
    if (lane == 0) s_red[wave] = dmax;
    __syncthreads();
    dmax = s_red[0];
#pragma unroll
    for (int w = 1; w < kBwWaves; ++w) dmax = fmaxf(dmax, s_red[w]);
    const double rho = rr - g.radius;
    if (rho > 0.0 && dmax == dmax) {
      const double c = 2.0 * rr * g.radius;
      const double m4 = 2.0 * (c / (2.0 * rho) + 0.75 * c * c / (rho * rho * rho));
      const double d2 = (double)dmax * (double)dmax;
      const double rem = m4 * d2 * d2 / 24.0;   // metres
      series = rem * (kTwoPiD * g.k_over_pi) <= 1e-6 && rem * g.beta <= 0x1p-20 &&
               g.beta * g.radius * (double)dmax < 0.5 && g.k_over_pi * g.radius * (double)dmax < 64.0;
    }
  }
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  const float c4 = (float)(2.0 * c2);          // 4 R r
  const float rrr = (float)(rr * g.radius);    // R r
  const float two_k = (float)(2.0 * g.kw);
  const float kpi = (float)g.k_over_pi;
  const float beta = (float)g.beta;
  const float isc = y.inv_scale;
  const double u_shift = INTERP == ROSAR_NEAREST ? 0.5 - y.l_lo : -(double)y.l_lo;
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(ydata, (uint32_t)((int64_t)y.l_count * y.ld * ES));
  const int ld_es = (int)(y.ld * ES);
  const int64_t wrow = (int64_t)row * k;
  const float2* grow = gimg + (int64_t)row * n;

  auto passes = [&](auto series_tag) {
  constexpr bool SERIES = decltype(series_tag)::value;
  for (int base = 0; base < n; base += kBwThreads * kBwPpt) {
    float sh[kBwPpt], ch[kBwPpt], pr[kBwPpt], dn[kBwPpt], gd[kBwPpt], gp[kBwPpt];
    int cb[kBwPpt];   // byte offset of the pulse's column within a row
#pragma unroll
    for (int j = 0; j < kBwPpt; ++j) {
      const int pn = min(base + (int)threadIdx.x + kBwThreads * j, n - 1);
      sh[j] = 0.f;
      ch[j] = 1.f;
      dn[j] = dphi ? dphi[pn] : 0.f;
      if (dphi) sincosf(0.5f * dn[j], &sh[j], &ch[j]);
      pr[j] = dpsi ? dpsi[pn] * kInv2Pi : 0.f;
      pr[j] -= rintf(pr[j]);
      cb[j] = (pn + y.halo) * ES;
      gd[j] = 0.f;
      gp[j] = 0.f;
    }
    for (int c0 = 0; c0 < k; c0 += kBwChunk) {
      const int cnt = min(kBwChunk, k - c0);
      __syncthreads();   // the previous chunk's table is no longer read
      if ((int)threadIdx.x < cnt) {
        const int t = c0 + (int)threadIdx.x;
        const int o = offsets[wrow + t];
        double sd, cd;
        sincos(o * g.step, &sd, &cd);
        const double r2 = c1 - c2 * cd;
        const double rn = sqrt(r2);
        const float2 w = weights[wrow + t];
        BwTap e;
        e.u = split_bin(g.beta * rn + u_shift);
        if constexpr (SERIES) e.u.i = min(max(e.u.i, -3), y.l_count + 2);
        // derivatives of R(D) = sqrt(S), S = c1 - c2 cos D, at D0 (S' = c2 sin D0, S'' = c2 cos D0)
        const double s1 = c2 * sd, s2 = c2 * cd;
        const double ir = 1.0 / rn, ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
        const double q1 = 0.5 * s1 * ir;
        const double q2 = 0.5 * (0.5 * s2 * ir - 0.25 * s1 * s1 * ir3);
        const double q3 = (-0.5 * s1 * ir - 0.75 * s1 * s2 * ir3 + 0.375 * s1 * s1 * s1 * ir5) / 6.0;
        e.q1 = (float)q1;
        e.q2 = (float)q2;
        e.q3 = (float)q3;
        e.p2 = (float)(2.0 * q2);
        e.p3 = (float)(3.0 * q3);
        e.r2 = (float)r2;
        e.rnom = (float)rn;
        e.sd = (float)sd;
        e.cd = (float)cd;
        e.wr = w.x;
        e.wi = w.y;
        e.o = o;
        e.valid = (o >= -half_w && o < half_w) ? 1 : 0;
        s_tap[threadIdx.x] = e;
      }
      __syncthreads();
      for (int tt = 0; tt < cnt; ++tt) {
        const BwTap tp = s_tap[tt];
        if (!tp.valid) continue;   // uniform
        float2 gw = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kBwPpt; ++j) {
          const int pn = base + (int)threadIdx.x + kBwThreads * j;
          int ap = min(pn, n - 1) - tp.o;
          ap += (ap < 0) ? n : 0;
          ap -= (ap >= n) ? n : 0;
          // pulses past N (last pass) take a zero gradient sample: they add nothing
          const float2 gv = pn < n ? grow[ap] : make_float2(0.f, 0.f);
          float diff, dr;   // R^ - R_nom and dR^/dd
          if constexpr (SERIES) {
            diff = dn[j] * fmaf(dn[j], fmaf(dn[j], tp.q3, tp.q2), tp.q1);
            dr = fmaf(dn[j], fmaf(dn[j], tp.p3, tp.p2), tp.q1);
          } else {
            const float s_mid = fmaf(tp.sd, ch[j], tp.cd * sh[j]);   // sin(D0 + d/2)
            const float dd = c4 * s_mid * sh[j];                      // R^2 - R_nom^2
            const float r2 = fmaxf(tp.r2 + dd, 1e-30f);
            const float rs = __builtin_amdgcn_rsqf(r2);
            const float rh = r2 * rs;
            diff = dd * __builtin_amdgcn_rcpf(rh + tp.rnom);
            // dR^/dd = R r sin(D) / R^,  D = D0 + d:
            // sin D = sin D0 (1 - 2 sin^2(d/2)) + cos D0 2 sin(d/2) cos(d/2)
            const float sind = fmaf(tp.sd, fmaf(-2.f * sh[j], sh[j], 1.f), tp.cd * 2.f * sh[j] * ch[j]);
            dr = rrr * sind * rs;
          }
          const float corr = beta * diff;
          float fr;
          bool tie;
          int l = corr_bin(tp.u, corr, &fr, &tie);
          float2 yv, dy = make_float2(0.f, 0.f);
          if constexpr (INTERP == ROSAR_NEAREST) {
            if (__builtin_expect(tie, 0)) {
              // plain float64 bin at the angle (o 2 pi) / N + delta_n of the oracle's definition
              const double d = (double)tp.o * g.step + (dphi ? (double)dphi[min(pn, n - 1)] : 0.0);
              l = (int)floor(plain_bin_half(rr, g.radius, d, g.beta)) - y.l_lo;
              l = min(max(l, -1), y.l_count);
            }
            if constexpr (!SERIES) l = min(max(l, -1), y.l_count);
            yv = buf_load<DT>(rsrc, (uint32_t)(__mul24(l, ld_es) + cb[j]), 0u);
          } else {
            if constexpr (!SERIES) l = min(max(l, -2), y.l_count);
            const uint32_t off0 = (uint32_t)(__mul24(l, ld_es) + cb[j]);
            const float2 y0 = buf_load<DT>(rsrc, off0, 0u);
            const float2 y1 = buf_load<DT>(rsrc, off0 + (uint32_t)ld_es, 0u);
            dy = make_float2((y1.x - y0.x) * isc, (y1.y - y0.y) * isc);
            yv = make_float2(fmaf(fr, y1.x - y0.x, y0.x), fmaf(fr, y1.y - y0.y, y0.y));
          }
          yv.x *= isc;
          yv.y *= isc;
          float rev = fmaf(kpi, diff, pr[j]);
          if constexpr (!SERIES) rev -= floorf(rev);
          const float2 rot = make_float2(cos_rev(rev), -sin_rev(rev));
          const float2 s = cmul(yv, rot);
          // conj(g) s
          gw.x = fmaf(gv.x, s.x, fmaf(gv.y, s.y, gw.x));
          gw.y = fmaf(gv.x, s.y, fmaf(-gv.y, s.x, gw.y));
          // ds/d dphi = rot (beta dY/du - j 2k Y) dR^/dd
          const float2 inner = make_float2(beta * dy.x + two_k * yv.y, beta * dy.y - two_k * yv.x);
          const float2 dsd = cmul(rot, inner);
          // z = conj(g) conj(w) = conj(g w)
          const float2 gw_ = cmul(gv, make_float2(tp.wr, tp.wi));
          const float2 z = make_float2(gw_.x, -gw_.y);
          const float2 zd = cmul(z, dsd);
          const float2 zs = cmul(z, s);
          gd[j] = fmaf(zd.x, dr, gd[j]);
          gp[j] += zs.y;
        }
        gw = wave_sum(gw);
        if (lane == 0) {
          float2 cur = s_gw[wave * k + c0 + tt];
          s_gw[wave * k + c0 + tt] = make_float2(cur.x + gw.x, cur.y + gw.y);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kBwPpt; ++j) {
      const int pn = base + threadIdx.x + kBwThreads * j;
      if (pn < n) {
        part_d[(int64_t)row * n + pn] = gd[j];
        part_p[(int64_t)row * n + pn] = gp[j];
      }
    }
  }
  };
  if (series)
    passes(std::true_type{});
  else
    passes(std::false_type{});
  __syncthreads();
  if (grad_w) {
    for (int t = threadIdx.x; t < k; t += kBwThreads) {
      float2 sum = s_gw[t];
      for (int w = 1; w < kBwWaves; ++w) sum = make_float2(sum.x + s_gw[w * k + t].x, sum.y + s_gw[w * k + t].y);
      grad_w[wrow + t] = sum;
    }
  }
}

// Stage 1: group gy sums rows [gy * rows_per, min((gy + 1) * rows_per, n_range)) of the row
// partials, row by row, into group partials.  Stage 2 adds the groups in order.
__global__ __launch_bounds__(256) void backward_reduce_rows_kernel(int32_t n, int32_t n_range, int32_t rows_per,
                                                                   const float* __restrict__ part_d,
                                                                   const float* __restrict__ part_p,
                                                                   float* __restrict__ grp_d,
                                                                   float* __restrict__ grp_p) {
  const int pn = blockIdx.x * blockDim.x + threadIdx.x;
  const int gy = blockIdx.y;
  if (pn >= n) return;
  const int r0 = gy * rows_per;
  const int r1 = min(r0 + rows_per, n_range);
  float sd = 0.f, sp = 0.f;
  for (int r = r0; r < r1; ++r) {
    sd += part_d[(int64_t)r * n + pn];
    sp += part_p[(int64_t)r * n + pn];
  }
  grp_d[(int64_t)gy * n + pn] = sd;
  grp_p[(int64_t)gy * n + pn] = sp;
}

__global__ __launch_bounds__(256) void backward_reduce_groups_kernel(int32_t n, int32_t groups,
                                                                     const float* __restrict__ grp_d,
                                                                     const float* __restrict__ grp_p,
                                                                     float* __restrict__ grad_dphi,
                                                                     float* __restrict__ grad_dpsi) {
  const int pn = blockIdx.x * blockDim.x + threadIdx.x;
  if (pn >= n) return;
  float sd = 0.f, sp = 0.f;
  for (int gy = 0; gy < groups; ++gy) {
    sd += grp_d[(int64_t)gy * n + pn];
    sp += grp_p[(int64_t)gy * n + pn];
  }
  if (grad_dphi) grad_dphi[pn] = sd;
  if (grad_dpsi) grad_dpsi[pn] = sp;
}

template <int DT>
hipError_t launch_dt(const SparseArgs& a, const float2* gimg, float2* grad_w, float* pd, float* pp,
                     hipStream_t s) {
  const int nblocks = a.g.n_range;
  const char* yd = reinterpret_cast<const char*>(a.y.data);
  const float2* w = reinterpret_cast<const float2*>(a.weights);
  const size_t lds = (size_t)kBwWaves * a.k * sizeof(float2);
  if (a.interp == ROSAR_LINEAR)
    backward_row_kernel<DT, ROSAR_LINEAR><<<nblocks, kBwThreads, lds, s>>>(
        a.g, a.y, a.k, a.window, nblocks, a.offsets, w, a.dphi, a.dpsi, gimg, yd, grad_w, pd, pp);
  else
    backward_row_kernel<DT, ROSAR_NEAREST><<<nblocks, kBwThreads, lds, s>>>(
        a.g, a.y, a.k, a.window, nblocks, a.offsets, w, a.dphi, a.dpsi, gimg, yd, grad_w, pd, pp);
  return hipGetLastError();
}

}  // namespace

// Row partials (2 x n_range x N floats) followed by the group partials (2 x kRedGroups x N).
size_t backward_workspace_bytes(int32_t n, int32_t n_range, int32_t k) {
  (void)k;
  return 2 * (size_t)n * ((size_t)n_range + kRedGroups) * sizeof(float);
}

hipError_t launch_sparse_backward(const SparseArgs& a, const float2* grad_image, float2* grad_w,
                                  float* grad_dphi, float* grad_dpsi, void* ws, hipStream_t s) {
  const int n = a.g.n, nr = a.g.n_range;
  float* pd = reinterpret_cast<float*>(ws);
  float* pp = pd + (size_t)n * nr;
  float* gd = pp + (size_t)n * nr;
  float* gp = gd + (size_t)n * kRedGroups;
  hipError_t e;
  switch (a.y.dtype) {
    case ROSAR_C64: e = launch_dt<0>(a, grad_image, grad_w, pd, pp, s); break;
    case ROSAR_C16_F16: e = launch_dt<1>(a, grad_image, grad_w, pd, pp, s); break;
    default: e = launch_dt<2>(a, grad_image, grad_w, pd, pp, s); break;
  }
  if (e != hipSuccess) return e;
  if (grad_dphi || grad_dpsi) {
    const int rows_per = (nr + kRedGroups - 1) / kRedGroups;
    const int groups = (nr + rows_per - 1) / rows_per;
    const dim3 grid1((n + 255) / 256, groups);
    backward_reduce_rows_kernel<<<grid1, 256, 0, s>>>(n, nr, rows_per, pd, pp, gd, gp);
    backward_reduce_groups_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, groups, gd, gp, grad_dphi, grad_dpsi);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace rosar
