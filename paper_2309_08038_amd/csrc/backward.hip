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
// waves in a fixed order.  Row partials of grad_dphi/grad_dpsi go to the workspace and a
// second kernel sums them over rows, row by row, in a fixed order.
#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kBwThreads = 256;
constexpr int kBwWaves = kBwThreads / kWave;
constexpr int kBwPpt = 8;      // pulses per thread per pass
constexpr int kBwMaxK = 1024;

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
  __shared__ float2 s_gw[kBwWaves][kBwMaxK];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int row = xcd_logical_block(blockIdx.x, nblocks);
  const int n = g.n;
  const int half_w = window / 2;
  for (int t = threadIdx.x; t < k; t += kBwThreads)
    for (int w = 0; w < kBwWaves; ++w) s_gw[w][t] = make_float2(0.f, 0.f);
  __syncthreads();

  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  const double rrr = rr * g.radius;
  const float two_k = (float)(2.0 * g.kw);
  const float beta = (float)g.beta;
  const float isc = y.inv_scale;
  constexpr double kInv2Pi = 0.15915494309189533577;
  const int64_t wrow = (int64_t)row * k;
  const float2* grow = gimg + (int64_t)row * n;

  for (int base = 0; base < n; base += kBwThreads * kBwPpt) {
    double cd[kBwPpt], sd[kBwPpt];
    float ps[kBwPpt], gd[kBwPpt], gp[kBwPpt];
#pragma unroll
    for (int j = 0; j < kBwPpt; ++j) {
      const int pn = base + threadIdx.x + kBwThreads * j;
      const double d = (pn < n && dphi) ? (double)dphi[pn] : 0.0;
      sincos(d, &sd[j], &cd[j]);
      ps[j] = (pn < n && dpsi) ? dpsi[pn] : 0.f;
      gd[j] = 0.f;
      gp[j] = 0.f;
    }
    for (int c0 = 0; c0 < k; c0 += kWave) {
      const int t = c0 + lane;
      int ofs = 0;
      double cd0 = 1.0, sd0 = 0.0, rnom = 0.0;
      if (t < k) {
        ofs = offsets[wrow + t];
        sincos(ofs * g.step, &sd0, &cd0);
        rnom = sqrt(c1 - c2 * cd0);
      }
      const int cnt = min(kWave, k - c0);
      for (int tt = 0; tt < cnt; ++tt) {
        const int o = readlane(ofs, tt);
        if (o < -half_w || o >= half_w) continue;
        const double cD0 = readlane(cd0, tt);
        const double sD0 = readlane(sd0, tt);
        const double rN = readlane(rnom, tt);
        const float2 w = weights[wrow + c0 + tt];
        float2 gw = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kBwPpt; ++j) {
          const int pn = base + threadIdx.x + kBwThreads * j;
          if (pn < n) {
            int ap = pn - o;
            ap += (ap < 0) ? n : 0;
            ap -= (ap >= n) ? n : 0;
            const float2 gv = grow[ap];
            const double cosd = cD0 * cd[j] - sD0 * sd[j];
            const double sind = sD0 * cd[j] + cD0 * sd[j];
            const double rh = sqrt(c1 - c2 * cosd);
            const double u = g.beta * rh;
            const int64_t col = pn + y.halo;
            float2 yv, dy = make_float2(0.f, 0.f);
            if constexpr (INTERP == ROSAR_NEAREST) {
              const int l = (int)floor(u + 0.5) - y.l_lo;
              yv = (l >= 0 && l < y.l_count) ? load_c<DT>(ydata, l * y.ld + col) : make_float2(0.f, 0.f);
            } else {
              const double fl = floor(u);
              const float f = (float)(u - fl);
              const int l = (int)fl - y.l_lo;
              const float2 y0 = (l >= 0 && l < y.l_count) ? load_c<DT>(ydata, l * y.ld + col) : make_float2(0.f, 0.f);
              const float2 y1 = (l + 1 >= 0 && l + 1 < y.l_count) ? load_c<DT>(ydata, (l + 1) * y.ld + col)
                                                                   : make_float2(0.f, 0.f);
              dy = make_float2((y1.x - y0.x) * isc, (y1.y - y0.y) * isc);
              yv = make_float2(fmaf(f, y1.x - y0.x, y0.x), fmaf(f, y1.y - y0.y, y0.y));
            }
            yv.x *= isc;
            yv.y *= isc;
            const float fr = frac_rev(g.k_over_pi * (rh - rN) + (double)ps[j] * kInv2Pi);
            const float2 rot = make_float2(cos_rev(fr), -sin_rev(fr));
            const float2 s = cmul(yv, rot);
            // conj(g) s
            gw.x = fmaf(gv.x, s.x, fmaf(gv.y, s.y, gw.x));
            gw.y = fmaf(gv.x, s.y, fmaf(-gv.y, s.x, gw.y));
            // ds/d dphi
            const float dr = (float)(rrr * sind / rh);
            const float2 inner = make_float2(beta * dy.x + two_k * yv.y, beta * dy.y - two_k * yv.x);
            const float2 dsd = cmul(rot, inner);
            // z = conj(g) conj(w) = conj(g w)
            const float2 gw_ = cmul(gv, w);
            const float2 z = make_float2(gw_.x, -gw_.y);
            const float2 zd = cmul(z, dsd);
            const float2 zs = cmul(z, s);
            gd[j] = fmaf(zd.x, dr, gd[j]);
            gp[j] += zs.y;
          }
        }
        gw = wave_sum(gw);
        if (lane == 0) {
          float2 cur = s_gw[wave][c0 + tt];
          s_gw[wave][c0 + tt] = make_float2(cur.x + gw.x, cur.y + gw.y);
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
  __syncthreads();
  if (grad_w) {
    for (int t = threadIdx.x; t < k; t += kBwThreads) {
      float2 sum = s_gw[0][t];
      for (int w = 1; w < kBwWaves; ++w) sum = make_float2(sum.x + s_gw[w][t].x, sum.y + s_gw[w][t].y);
      grad_w[wrow + t] = sum;
    }
  }
}

__global__ __launch_bounds__(256) void backward_reduce_kernel(int32_t n, int32_t n_range,
                                                              const float* __restrict__ part_d,
                                                              const float* __restrict__ part_p,
                                                              float* __restrict__ grad_dphi,
                                                              float* __restrict__ grad_dpsi) {
  const int pn = blockIdx.x * blockDim.x + threadIdx.x;
  if (pn >= n) return;
  float sd = 0.f, sp = 0.f;
  for (int r = 0; r < n_range; ++r) {
    sd += part_d[(int64_t)r * n + pn];
    sp += part_p[(int64_t)r * n + pn];
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
  if (a.interp == ROSAR_LINEAR)
    backward_row_kernel<DT, ROSAR_LINEAR><<<nblocks, kBwThreads, 0, s>>>(
        a.g, a.y, a.k, a.window, nblocks, a.offsets, w, a.dphi, a.dpsi, gimg, yd, grad_w, pd, pp);
  else
    backward_row_kernel<DT, ROSAR_NEAREST><<<nblocks, kBwThreads, 0, s>>>(
        a.g, a.y, a.k, a.window, nblocks, a.offsets, w, a.dphi, a.dpsi, gimg, yd, grad_w, pd, pp);
  return hipGetLastError();
}

}  // namespace

size_t backward_workspace_bytes(int32_t n, int32_t n_range, int32_t k) {
  (void)k;
  return 2 * (size_t)n * (size_t)n_range * sizeof(float);
}

hipError_t launch_sparse_backward(const SparseArgs& a, const float2* grad_image, float2* grad_w,
                                  float* grad_dphi, float* grad_dpsi, void* ws, hipStream_t s) {
  float* pd = reinterpret_cast<float*>(ws);
  float* pp = pd + (size_t)a.g.n * a.g.n_range;
  hipError_t e;
  switch (a.y.dtype) {
    case ROSAR_C64: e = launch_dt<0>(a, grad_image, grad_w, pd, pp, s); break;
    case ROSAR_C16_F16: e = launch_dt<1>(a, grad_image, grad_w, pd, pp, s); break;
    default: e = launch_dt<2>(a, grad_image, grad_w, pd, pp, s); break;
  }
  if (e != hipSuccess) return e;
  if (grad_dphi || grad_dpsi) {
    backward_reduce_kernel<<<(a.g.n + 255) / 256, 256, 0, s>>>(a.g.n, a.g.n_range, pd, pp, grad_dphi,
                                                               grad_dpsi);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace rosar
