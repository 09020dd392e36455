// Adjoint of the sparse filter with respect to the weights and the per-pulse angle and phase
// errors, for a real loss with grad_image = dL/dRe(I) + j dL/dIm(I):
//   grad_w[i,t]  = sum_a conj(g[i,a]) s(i,a,t)
//   grad_dphi[n] = sum_{i,t} Re(conj(g[i,a]) conj(w[i,t]) ds/d dphi_n),   a = (n - o_t) mod N
//   grad_dpsi[n] = sum_{i,t} Im(conj(g[i,a]) conj(w[i,t]) s)
//   ds/d dphi = rot (beta dY/du - j 2k Y) R_i r sin(D) / R^,  rot = exp(-j (2k (R^ - R_nom) + psi)).
// (Chain rule through eq. 2 and the eq.-40 bin position; dY/du is the LINEAR slope, zero for
// NEAREST.)
//
// Gather formulation, deterministic without atomics: each thread owns pulses n (so the
// angle/phase terms of n stay in registers and the row's contribution to grad_dphi[n]
// accumulates in that thread).  For each tap the thread visits pixel a = n - o_t, recomputes the
// sample and its derivative (indices are never stored), and feeds conj(g) s into a per-tap
// partial reduced across the wavefront and then across the waves in a fixed order.  The taps'
// nominal geometry (float64 bin of R_nom, R_nom, sin/cos of D0 = 2 pi o / N) and weights sit in
// an LDS table; per (pulse, tap) only the angle-error correction is evaluated in float32.  As in
// the corrected forward it is either the cubic Taylor polynomial of R(D0 + d) - R(D0) in d (and
// its derivative for dR^/dd), taken when the fourth-derivative remainder bound at the largest
// |d| is below 1e-6 rad of carrier phase and 2^-20 bins, or otherwise the exact form without
// cancellation:
//   R^2 - R_nom^2 = 4 R r sin(D0 + d/2) sin(d/2),   R^ - R_nom = (R^2 - R_nom^2)/(R^ + R_nom).
// The main kernel works on tiles of one range row and kBtTile pulses, with the gradient columns
// and, on the series path, the band rows in LDS (backward_tile); windows too wide for that keep
// one workgroup per row reading the band through buffer loads (backward_row_kernel, out-of-band
// rows read zero).  Row partials of grad_dphi/grad_dpsi go to the workspace and a two-stage
// reduction sums them over rows in a fixed order (groups of rows, then the groups); the tiles'
// grad_w partials are added in order by their own kernel.
#include <climits>
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

constexpr int kBtWaves = 4;
constexpr int kBtThreads = kBtWaves * kWave;
constexpr int kBtP = 4;                        // pulses per lane (64 apart)
constexpr int kBtTile = kBtThreads * kBtP;     // pulses per workgroup
constexpr int kBtChunk = kWave;                // taps per table chunk (one per lane of wave 0)
constexpr int kBtMaxCols = 4096;               // largest T + W whose gradient columns sit in LDS
constexpr int kBtStageCols = 2048;             // largest T + W whose band rows are staged too
constexpr int kBtStageRows = 2;                // band rows (LINEAR: (row, next - row) pairs) staged
constexpr int kBtStageLoads = kBtStageRows + 1;
constexpr int kGBatch = 8;                     // gradient columns per thread whose loads are issued together

// Nominal geometry and weight of one tap, 64 bytes.
struct alignas(16) BtTap {
  SplitBin u;         // band-relative bin beta * R_nom - l_lo (+ 1/2 for NEAREST), split
  float r2;           // R_nom^2
  float rnom;         // R_nom
  float sd, cd;       // sin, cos of D0
  float q1, q2, q3;   // series in e = beta d: R(D0 + d) - R_nom = d (q1 + e (q2 + e q3)) + O(d^4)
  float p2, p3;       // dR^/dd = q1 + e (p2 + e p3)
  float wr, wi;       // weight
  int32_t o;          // offset (zero outside the window)
  int32_t idx;        // tap index within its chunk
  int32_t ub;         // staged: byte offset of (row u.i - lmin, column 0); series from global
                      // memory: the nominal row clamped to [-3, l_count + 2], times the row pitch
};
static_assert(sizeof(BtTap) == 64, "tap entry size");


// Sum of v over the 64 lanes, complete in lane 63: quad, half-row and row steps by DPP lane
// swizzles, then the row broadcasts of lane 15 and lane 31 into the following rows.
__device__ __forceinline__ float wave_sum_to_63(float v) {
  v += __builtin_amdgcn_update_dpp(0.f, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x140, 0xF, 0xF, false);   // row_mirror
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x142, 0xA, 0xF, false);   // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x143, 0xC, 0xF, false);   // row_bcast:31 into rows 2, 3
  return v;
}

__device__ __forceinline__ int floor_to_int(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// One workgroup per (range row, tile of kBtTile pulses); lane-owned pulses n = p0 + loc, with
// loc = 64 (P w + j) + lane.  The tile's gradient columns a = n - o, [p0 - W/2, p0 + T + W/2),
// are copied into LDS once.  On the series path, when the rows the pairs can reach (floor of
// the nominal bin +- beta r max|d|) fit kBtStageRows, the band rows of the tile's own columns
// n are copied into LDS as well, scaled by 1/scale and turned by exp(-j psi_n) (LINEAR: as
// (y_l, y_l+1 - y_l)), and taps whose pairs all keep floor(x) = 0 run first without the bin
// arithmetic; otherwise the pairs read the band from global memory as in the corrected
// forward.  Per pair, with h = conj(g) exp(-j 2 pi rev), Y the (interpolated) sample and dY
// its LINEAR slope:
//   grad_w     += h Y
//   grad_dphi  += dR^/dd (beta Re(conj(w) h dY) + 2k Im(conj(w) h Y))
//   grad_dpsi  += Im(conj(w) h Y)
// grad_w is reduced per tap across the wave and then across the waves in a fixed order into a
// per-tile partial; the row partials of grad_dphi / grad_dpsi are one value per pulse.
template <int DT, int INTERP>
__device__ __forceinline__ void backward_tile(
    Geo g, View y, int32_t k, int32_t window, int tiles, int nblocks, int stage_rows,
    const int32_t* __restrict__ offsets, const float2* __restrict__ weights,
    const float* __restrict__ dphi, const float* __restrict__ dpsi,
    const float2* __restrict__ gimg, const char* __restrict__ ydata,
    float2* __restrict__ gw_part, float* __restrict__ part_d, float* __restrict__ part_p) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr bool LIN = INTERP == ROSAR_LINEAR;
  constexpr int EB = LIN ? 16 : 8;   // bytes per staged element
  constexpr float kInv2Pi = 0.15915494309189533577f;
  __shared__ BtTap s_tap[kBtChunk];
  __shared__ float2 s_gwc[kBtWaves][kBtChunk];
  __shared__ float s_red[kBtWaves];
  __shared__ int s_redi[2 * kBtWaves];
  __shared__ int s_nfast;
  extern __shared__ float4 s_dyn[];   // gradient columns (T + W), then the staged band rows (16-byte aligned)
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles;
  const int tile = blk - row * tiles;
  const int n = g.n;
  const int half_w = window / 2;
  const int cols = kBtTile + window;
  const int p0 = tile * kBtTile;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int i_wave = wave * kWave * kBtP;
  const double rr = g.r0 + row * g.dr;
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
  float2* s_g = reinterpret_cast<float2*>(s_dyn);
  char* band = reinterpret_cast<char*>(s_dyn) + ((cols * 8 + 15) & ~15);
  const bool wave_live = p0 + i_wave < n;

  // the first chunk's offsets and weights, requested before anything waits on memory
  int o_next = (int)threadIdx.x < min(kBtChunk, k) ? offsets[wrow + threadIdx.x] : 0;
  float2 w_next = (int)threadIdx.x < min(kBtChunk, k) ? weights[wrow + threadIdx.x] : make_float2(0.f, 0.f);

  // lane-owned pulses
  float dj[kBtP], psj[kBtP];
#pragma unroll
  for (int j = 0; j < kBtP; ++j) {
    const int pc = min(p0 + i_wave + lane + kWave * j, n - 1);
    dj[j] = dphi ? dphi[pc] : 0.f;
    psj[j] = dpsi ? dpsi[pc] : 0.f;
  }
  // the float64 geometry of one tap (ub left zero); its nominal bin in *u64
  auto nominal = [&](int o, double& sd, double& cd, double& r2) {
    sincos(o * g.step, &sd, &cd);
    r2 = c1 - c2 * cd;
    return g.beta * sqrt(r2) + u_shift;
  };
  auto make_tap = [&](int o, float2 w, int idx, bool& inwin, double& u64) {
    BtTap e{};
    inwin = o >= -half_w && o < half_w;
    double sd, cd, r2;
    u64 = nominal(o, sd, cd, r2);
    const double rn = sqrt(r2);
    e.u = split_bin(u64);
    e.r2 = (float)r2;
    e.rnom = (float)rn;
    e.sd = (float)sd;
    e.cd = (float)cd;
    const double s1 = c2 * sd, s2 = c2 * cd;
    const double ir = 1.0 / rn, ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
    const double ib = 1.0 / g.beta;
    const double q1 = 0.5 * s1 * ir;
    const double q2 = 0.5 * (0.5 * s2 * ir - 0.25 * s1 * s1 * ir3);
    const double q3 = (-0.5 * s1 * ir - 0.75 * s1 * s2 * ir3 + 0.375 * s1 * s1 * s1 * ir5) / 6.0;
    e.q1 = (float)q1;
    e.q2 = (float)(q2 * ib);
    e.q3 = (float)(q3 * ib * ib);
    e.p2 = (float)(2.0 * q2 * ib);
    e.p3 = (float)(3.0 * q3 * ib * ib);
    e.wr = w.x;
    e.wi = w.y;
    e.o = inwin ? o : 0;
    e.idx = idx;
    return e;
  };
  // with at most one chunk of taps, wave 0 builds the table once, while the loads are in flight
  // (parked in its LDS slot until the chunk loop files it)
  const bool fused = k <= kBtChunk;
  bool inwin0 = false;
  double u0 = 0.0;
  if (fused && wave == 0 && lane < k) s_tap[lane] = make_tap(o_next, w_next, lane, inwin0, u0);
  // gradient columns: pixel p0 - W/2 + c, wrapped; the loads of a thread's columns issued together
  for (int cb = threadIdx.x; cb < cols; cb += kGBatch * kBtThreads) {
    float2 gv[kGBatch];
#pragma unroll
    for (int j = 0; j < kGBatch; ++j) {
      const int c = cb + j * kBtThreads;
      if (c < cols) {
        int a = p0 - half_w + c;
        if (a < 0 || a >= n) a = ((a % n) + n) % n;
        gv[j] = grow[a];
      }
    }
#pragma unroll
    for (int j = 0; j < kGBatch; ++j) {
      const int c = cb + j * kBtThreads;
      if (c < cols) s_g[c] = gv[j];
    }
  }
  float dmax = 0.f;
#pragma unroll
  for (int j = 0; j < kBtP; ++j)
    if (p0 + i_wave + lane + kWave * j < n) dmax = fmaxf(dmax, fabsf(dj[j]));
  for (int off = kWave / 2; off > 0; off >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, off));
  if (lane == 0) s_red[wave] = dmax;
  __syncthreads();
  dmax = s_red[0];
#pragma unroll
  for (int w = 1; w < kBtWaves; ++w) dmax = fmaxf(dmax, s_red[w]);

  // the series path when the remainder bound (see the corrected forward) holds at max |d|
  bool series = false, staged = false;
  double cm = 0.0;       // bound on |x - u.f| of a series pair, in bins
  float tie_err = 0.f;   // series, NEAREST: bound on the error of the float32 bin sum
  int lmin = 0, nrows = 0;
  const double rho = rr - g.radius;
  if (rho > 0.0 && dmax == dmax) {
    const double c = 2.0 * rr * g.radius;
    const double m4 = 2.0 * (c / (2.0 * rho) + 0.75 * c * c / (rho * rho * rho));
    const double d2 = (double)dmax * (double)dmax;
    const double rem = m4 * d2 * d2 / 24.0;   // metres
    series = rem * (kTwoPiD * g.k_over_pi) <= 1e-6 && rem * g.beta <= 0x1p-20 &&
             g.beta * g.radius * (double)dmax < 0.5 && g.k_over_pi * g.radius * (double)dmax < 64.0;
    const double cmax = g.beta * g.radius * (double)dmax + 0x1p-20;
    cm = cmax * (1.0 + 0x1p-10) + 0x1p-16;
    tie_err = (float)(0x1p-18 + cmax * 0x1p-12);
  }
  if (series && stage_rows > 0) {
    // rows the pairs can reach: floor(u +- cm) over the in-window taps
    int lo = INT_MAX, hi = INT_MIN;
    if (fused) {
      if (wave == 0 && lane < k && inwin0) {
        lo = (int)floor(u0 - cm);
        hi = (int)floor(u0 + cm);
      }
    } else {
     for (int t = threadIdx.x; t < k; t += kBtThreads) {
      const int o = t == (int)threadIdx.x && t < kBtChunk ? o_next : offsets[wrow + t];
      if (o >= -half_w && o < half_w) {
        double sd, cd, r2;
        const double u = nominal(o, sd, cd, r2);
        lo = min(lo, (int)floor(u - cm));
        hi = max(hi, (int)floor(u + cm));
      }
     }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
      lo = min(lo, __shfl_xor(lo, off));
      hi = max(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
      s_redi[2 * wave] = lo;
      s_redi[2 * wave + 1] = hi;
    }
    __syncthreads();
    lo = s_redi[0];
    hi = s_redi[1];
#pragma unroll
    for (int w = 1; w < kBtWaves; ++w) {
      lo = min(lo, s_redi[2 * w]);
      hi = max(hi, s_redi[2 * w + 1]);
    }
    if (hi < lo) lo = hi = 0;   // no tap inside the window
    lmin = lo;
    nrows = hi - lo + 1;
    staged = nrows <= stage_rows;
  }

  // per-pulse values: e = beta d, (k / pi) d, psi / 2 pi reduced; the exact path's half angle
  float ej[kBtP], kdj[kBtP], prj[kBtP], shj[kBtP], chj[kBtP];
#pragma unroll
  for (int j = 0; j < kBtP; ++j) {
    ej[j] = beta * dj[j];
    kdj[j] = kpi * dj[j];
    prj[j] = psj[j] * kInv2Pi;
    prj[j] -= rintf(prj[j]);
    shj[j] = 0.f;
    chj[j] = 1.f;
    if (!series && dphi) sincosf(0.5f * dj[j], &shj[j], &chj[j]);
  }
  if (staged) {
    // the tile's own band columns, rows lmin .., scaled by 1/scale and turned by exp(-j psi)
    const int nload = nrows + (LIN ? 1 : 0);
#pragma unroll
    for (int j = 0; j < kBtP; ++j) {
      const int loc = i_wave + lane + kWave * j;
      const int pn = p0 + loc;
      const uint32_t colb = (uint32_t)((min(pn, n - 1) + y.halo) * ES);
      float2 v[kBtStageLoads];
#pragma unroll
      for (int r = 0; r < kBtStageLoads; ++r) {
        const int l = lmin + r;
        v[r] = make_float2(0.f, 0.f);
        if (pn < n && r < nload && l >= 0 && l < y.l_count) v[r] = buf_load<DT>(rsrc, (uint32_t)__mul24(l, ld_es) + colb, 0u);
      }
      const float sp = isc * sin_rev(prj[j]), cp = isc * cos_rev(prj[j]);
#pragma unroll
      for (int r = 0; r < kBtStageLoads; ++r) v[r] = make_float2(fmaf(v[r].x, cp, v[r].y * sp), fmaf(v[r].y, cp, -v[r].x * sp));
#pragma unroll
      for (int r = 0; r < kBtStageRows; ++r) {
        if (r >= nrows) break;
        if constexpr (LIN) {
          reinterpret_cast<float4*>(band)[r * kBtTile + loc] =
              make_float4(v[r].x, v[r].y, v[r + 1].x - v[r].x, v[r + 1].y - v[r].y);
        } else {
          reinterpret_cast<float2*>(band)[r * kBtTile + loc] = v[r];
        }
      }
    }
  }

  float gd[kBtP], gp[kBtP];
#pragma unroll
  for (int j = 0; j < kBtP; ++j) gd[j] = gp[j] = 0.f;
  const int laneb = (i_wave + lane) * EB;
  const int rowb = kBtTile * EB;

  // common tail of a pair: rev the phase in revolutions, Y and dY the sample and its slope
  auto pair_tail = [&](int j, const BtTap& tp, float2 gv, float rev, float dr, float2 Y, float2 dY,
                       float2& gw) {
    const float c = cos_rev(rev), sn = sin_rev(rev);
    const float2 h = make_float2(fmaf(gv.x, c, -gv.y * sn), fmaf(-gv.x, sn, -gv.y * c));   // conj(g) rot
    gw.x = fmaf(h.x, Y.x, fmaf(-h.y, Y.y, gw.x));
    gw.y = fmaf(h.x, Y.y, fmaf(h.y, Y.x, gw.y));
    const float2 zr = make_float2(fmaf(tp.wr, h.x, tp.wi * h.y), fmaf(tp.wr, h.y, -tp.wi * h.x));   // conj(w) h
    const float im = fmaf(zr.x, Y.y, zr.y * Y.x);
    if constexpr (LIN) {
      const float re = fmaf(zr.x, dY.x, -zr.y * dY.y);
      gd[j] = fmaf(dr, fmaf(beta, re, two_k * im), gd[j]);
    } else {
      gd[j] = fmaf(dr, two_k * im, gd[j]);
    }
    gp[j] += im;
  };
  // NEAREST tie: the plain float64 bin at the angle (o 2 pi) / N + delta_n of the oracle's
  // definition, sampled from the band in global memory (not turned, scaled)
  auto tie_sample = [&](int j, const BtTap& tp) {
    if (p0 + i_wave + lane + kWave * j >= n) return make_float2(0.f, 0.f);   // a pulse past N
    const int pc = p0 + i_wave + lane + kWave * j;
    const double d = (double)tp.o * g.step + (double)dj[j];
    int l = (int)floor(plain_bin_half(rr, g.radius, d, g.beta)) - y.l_lo;
    l = min(max(l, -1), y.l_count);
    const float2 v = buf_load<DT>(rsrc, (uint32_t)(__mul24(l, ld_es) + (pc + y.halo) * ES), 0u);
    return make_float2(v.x * isc, v.y * isc);
  };
  // gradient sample of pulse j's pixel n - o; pulses past N add nothing (on the staged path
  // their band columns are zero already, so their g needs no mask there)
  auto grad_at = [&](int j, int o) {
    const float2 v = s_g[i_wave + lane + kWave * j - o + half_w];
    return p0 + i_wave + lane + kWave * j < n ? v : make_float2(0.f, 0.f);
  };
  auto grad_at_staged = [&](int j, int o) { return s_g[i_wave + lane + kWave * j - o + half_w]; };

  for (int c0 = 0; c0 < k; c0 += kBtChunk) {
    const int cnt = min(kBtChunk, k - c0);
    if (wave == 0) {
      // tap table of the chunk: wave 0, one tap per lane, staged taps filed fast ones first
      const bool valid = lane < cnt;
      BtTap e{};
      bool inwin = false;
      if (valid) {
        double u;
        if (fused) {
          e = s_tap[lane];   // each lane reads its own slot before any lane files into the table
          inwin = inwin0;
        } else {
          e = make_tap(o_next, w_next, lane, inwin, u);
        }
        if (staged) {
          e.ub = (e.u.i - lmin) * rowb;
        } else if (series) {
          e.u.i = min(max(e.u.i, -3), y.l_count + 2);
          e.ub = e.u.i * ld_es;
        }
      }
      const bool live = valid && inwin;
      const double margin = INTERP == ROSAR_NEAREST ? (double)tie_err : 0.0;
      const bool fast = staged && live && (double)e.u.f - cm >= margin && (double)e.u.f + cm < 1.0 - margin;
      const uint64_t fm = __builtin_amdgcn_ballot_w64(fast);
      const uint64_t sm = __builtin_amdgcn_ballot_w64(live && !fast);
      const uint64_t below = (1ull << lane) - 1ull;
      const int nf = __builtin_popcountll(fm);
      if (live) s_tap[fast ? __builtin_popcountll(fm & below) : nf + __builtin_popcountll(sm & below)] = e;
      if (lane == 0) {
        s_nfast = nf;
        s_redi[0] = nf + __builtin_popcountll(sm);   // taps to apply
      }
      // the next chunk's offsets and weights, in flight during this chunk's pairs
      const int c1n = c0 + kBtChunk;
      if (lane < min(kBtChunk, k - c1n)) {
        o_next = offsets[wrow + c1n + lane];
        w_next = weights[wrow + c1n + lane];
      }
    }
    for (int t = threadIdx.x; t < kBtWaves * kBtChunk; t += kBtThreads) s_gwc[t / kBtChunk][t % kBtChunk] = make_float2(0.f, 0.f);
    __syncthreads();
    const int nfast = __builtin_amdgcn_readfirstlane(wave_live ? s_nfast : 0);
    const int napply = __builtin_amdgcn_readfirstlane(wave_live ? s_redi[0] : 0);
    if (staged) {
      // taps whose pairs all sample their nominal row: x = u.f + e s lies in [0, 1)
      for (int t = 0; t < nfast; ++t) {
        const BtTap tp = s_tap[t];
        const char* bt = band + (tp.ub + laneb);
        float2 gw = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kBtP; ++j) {
          const float e = ej[j];
          const float s = fmaf(e, fmaf(e, tp.q3, tp.q2), tp.q1);
          const float dr = fmaf(e, fmaf(e, tp.p3, tp.p2), tp.q1);
          const char* at = bt + kWave * EB * j;
          float2 Y, dY = make_float2(0.f, 0.f);
          if constexpr (LIN) {
            const float x = fmaf(e, s, tp.u.f);
            const float4 v = *reinterpret_cast<const float4*>(at);
            Y = make_float2(fmaf(x, v.z, v.x), fmaf(x, v.w, v.y));
            dY = make_float2(v.z, v.w);
          } else {
            Y = *reinterpret_cast<const float2*>(at);
          }
          pair_tail(j, tp, grad_at_staged(j, tp.o), kdj[j] * s, dr, Y, dY, gw);
        }
        gw = make_float2(wave_sum_to_63(gw.x), wave_sum_to_63(gw.y));
        if (lane == kWave - 1) s_gwc[wave][tp.idx] = gw;
      }
      for (int t = nfast; t < napply; ++t) {
        const BtTap tp = s_tap[t];
        const char* bt = band + (tp.ub + laneb);
        float2 gw = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kBtP; ++j) {
          const float e = ej[j];
          const float s = fmaf(e, fmaf(e, tp.q3, tp.q2), tp.q1);
          const float dr = fmaf(e, fmaf(e, tp.p3, tp.p2), tp.q1);
          const float x = fmaf(e, s, tp.u.f);
          const float fr = __builtin_amdgcn_fractf(x);
          const char* at = bt + __mul24(floor_to_int(x), rowb) + kWave * EB * j;
          float rev = kdj[j] * s;
          float2 Y, dY = make_float2(0.f, 0.f);
          if constexpr (LIN) {
            const float4 v = *reinterpret_cast<const float4*>(at);
            Y = make_float2(fmaf(fr, v.z, v.x), fmaf(fr, v.w, v.y));
            dY = make_float2(v.z, v.w);
          } else {
            Y = *reinterpret_cast<const float2*>(at);
            if (__builtin_expect(fr < tie_err || fr > 1.f - tie_err, 0)) {
              Y = tie_sample(j, tp);
              rev += prj[j];
            }
          }
          pair_tail(j, tp, grad_at_staged(j, tp.o), rev, dr, Y, dY, gw);
        }
        gw = make_float2(wave_sum_to_63(gw.x), wave_sum_to_63(gw.y));
        if (lane == kWave - 1) s_gwc[wave][tp.idx] = gw;
      }
    } else {
      // gathers from global memory, series (clamped nominal row) or exact correction
      for (int t = 0; t < napply; ++t) {
        const BtTap tp = s_tap[t];
        float2 gw = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kBtP; ++j) {
          const int pc = min(p0 + i_wave + lane + kWave * j, n - 1);
          float diff, dr;   // R^ - R_nom and dR^/dd
          if (series) {
            const float e = ej[j];
            diff = dj[j] * fmaf(e, fmaf(e, tp.q3, tp.q2), tp.q1);
            dr = fmaf(e, fmaf(e, tp.p3, tp.p2), tp.q1);
          } else {
            const float s_mid = fmaf(tp.sd, chj[j], tp.cd * shj[j]);   // sin(D0 + d/2)
            const float dd = c4 * s_mid * shj[j];                        // R^2 - R_nom^2
            const float r2 = fmaxf(tp.r2 + dd, 1e-30f);
            const float rs = __builtin_amdgcn_rsqf(r2);
            diff = dd * __builtin_amdgcn_rcpf(r2 * rs + tp.rnom);
            // dR^/dd = R r sin(D) / R^,  D = D0 + d
            const float sind = fmaf(tp.sd, fmaf(-2.f * shj[j], shj[j], 1.f), tp.cd * 2.f * shj[j] * chj[j]);
            dr = rrr * sind * rs;
          }
          const float corr = beta * diff;
          const float x = tp.u.f + corr;
          const float fr = __builtin_amdgcn_fractf(x);
          int l = tp.u.i + floor_to_int(x);
          if (!series) l = min(max(l, INTERP == ROSAR_NEAREST ? -1 : -2), y.l_count);
          const uint32_t off0 = (uint32_t)(__mul24(l, ld_es) + (pc + y.halo) * ES);
          float rev = fmaf(kpi, diff, prj[j]);
          if (!series) rev -= floorf(rev);
          float2 Y, dY = make_float2(0.f, 0.f);
          if constexpr (LIN) {
            const float2 y0 = buf_load<DT>(rsrc, off0, 0u);
            const float2 y1 = buf_load<DT>(rsrc, off0 + (uint32_t)ld_es, 0u);
            dY = make_float2((y1.x - y0.x) * isc, (y1.y - y0.y) * isc);
            Y = make_float2(fmaf(fr, y1.x - y0.x, y0.x) * isc, fmaf(fr, y1.y - y0.y, y0.y) * isc);
          } else {
            const float err = series ? tie_err : 0x1p-18f + fabsf(corr) * 0x1p-12f;
            const float2 v = buf_load<DT>(rsrc, off0, 0u);
            Y = make_float2(v.x * isc, v.y * isc);
            if (__builtin_expect(fr < err || fr > 1.f - err, 0)) Y = tie_sample(j, tp);
          }
          pair_tail(j, tp, grad_at(j, tp.o), rev, dr, Y, dY, gw);
        }
        gw = make_float2(wave_sum_to_63(gw.x), wave_sum_to_63(gw.y));
        if (lane == kWave - 1) s_gwc[wave][tp.idx] = gw;
      }
    }
    __syncthreads();
    // the chunk's grad_w partial of this tile: the waves in a fixed order
    if ((int)threadIdx.x < cnt) {
      float2 sum = s_gwc[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kBtWaves; ++w) sum = make_float2(sum.x + s_gwc[w][threadIdx.x].x, sum.y + s_gwc[w][threadIdx.x].y);
      gw_part[((int64_t)row * tiles + tile) * k + c0 + threadIdx.x] = sum;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kBtP; ++j) {
    const int pn = p0 + i_wave + lane + kWave * j;
    if (pn < n) {
      part_d[(int64_t)row * n + pn] = gd[j];
      part_p[(int64_t)row * n + pn] = gp[j];
    }
  }
}

#define ROSAR_BT_ARGS                                                                             \
  Geo g, View y, int32_t k, int32_t window, int tiles, int nblocks, int stage_rows,              \
      const int32_t *__restrict__ offsets, const float2 *__restrict__ weights,                   \
      const float *__restrict__ dphi, const float *__restrict__ dpsi,                            \
      const float2 *__restrict__ gimg, const char *__restrict__ ydata,                           \
      float2 *__restrict__ gw_part, float *__restrict__ part_d, float *__restrict__ part_p
#define ROSAR_BT_PASS g, y, k, window, tiles, nblocks, stage_rows, offsets, weights, dphi, dpsi, gimg, ydata, gw_part, part_d, part_p

// LINEAR: the staged rows (48 KB of LDS) allow three workgroups per CU.
template <int DT>
__global__ __launch_bounds__(kBtThreads) void backward_tile_linear_kernel(ROSAR_BT_ARGS) {
  backward_tile<DT, ROSAR_LINEAR>(ROSAR_BT_PASS);
}
// NEAREST stages half as much: four workgroups per CU once the registers fit 128 per lane (the
// few spills sit in the table set-up and the tie branch, not in the pair loops).
template <int DT>
__global__ __launch_bounds__(kBtThreads) __attribute__((amdgpu_waves_per_eu(4))) void backward_tile_nearest_kernel(
    ROSAR_BT_ARGS) {
  backward_tile<DT, ROSAR_NEAREST>(ROSAR_BT_PASS);
}
#undef ROSAR_BT_ARGS
#undef ROSAR_BT_PASS

// grad_w[row, t]: the tiles' partials added in order.
__global__ __launch_bounds__(256) void backward_reduce_w_kernel(int32_t k, int32_t n_range, int32_t tiles,
                                                                const float2* __restrict__ gw_part,
                                                                float2* __restrict__ grad_w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_range * k) return;
  const int64_t row = i / k, t = i - row * k;
  float2 sum = gw_part[row * tiles * k + t];
  for (int tl = 1; tl < tiles; ++tl) {
    const float2 v = gw_part[(row * tiles + tl) * k + t];
    sum = make_float2(sum.x + v.x, sum.y + v.y);
  }
  grad_w[i] = sum;
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
hipError_t launch_dt(const SparseArgs& a, const float2* gimg, float2* grad_w, float* pd, float* pp, float2* gwp,
                     hipStream_t s) {
  const char* yd = reinterpret_cast<const char*>(a.y.data);
  const float2* w = reinterpret_cast<const float2*>(a.weights);
  const bool lin = a.interp == ROSAR_LINEAR;
  const int cols = kBtTile + a.window;
  if (cols <= kBtMaxCols) {
    const int tiles = (a.g.n + kBtTile - 1) / kBtTile;
    const int nblocks = tiles * a.g.n_range;
    const int stage = cols <= kBtStageCols ? kBtStageRows : 0;
    const size_t lds = (((size_t)cols * sizeof(float2) + 15) & ~(size_t)15) + (size_t)stage * kBtTile * (lin ? 16 : 8);
    if (lin)
      backward_tile_linear_kernel<DT><<<nblocks, kBtThreads, lds, s>>>(
          a.g, a.y, a.k, a.window, tiles, nblocks, stage, a.offsets, w, a.dphi, a.dpsi, gimg, yd, gwp, pd, pp);
    else
      backward_tile_nearest_kernel<DT><<<nblocks, kBtThreads, lds, s>>>(
          a.g, a.y, a.k, a.window, tiles, nblocks, stage, a.offsets, w, a.dphi, a.dpsi, gimg, yd, gwp, pd, pp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grad_w) return e;
    const int64_t total = (int64_t)a.g.n_range * a.k;
    backward_reduce_w_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(a.k, a.g.n_range, tiles, gwp, grad_w);
    return hipGetLastError();
  }
  // windows too wide for the tile's gradient columns in LDS: one workgroup per row
  const int nblocks = a.g.n_range;
  const size_t lds = (size_t)kBwWaves * a.k * sizeof(float2);
  if (lin)
    backward_row_kernel<DT, ROSAR_LINEAR><<<nblocks, kBwThreads, lds, s>>>(
        a.g, a.y, a.k, a.window, nblocks, a.offsets, w, a.dphi, a.dpsi, gimg, yd, grad_w, pd, pp);
  else
    backward_row_kernel<DT, ROSAR_NEAREST><<<nblocks, kBwThreads, lds, s>>>(
        a.g, a.y, a.k, a.window, nblocks, a.offsets, w, a.dphi, a.dpsi, gimg, yd, grad_w, pd, pp);
  return hipGetLastError();
}

}  // namespace

// Row partials (2 x n_range x N floats), the group partials (2 x kRedGroups x N), then the
// per-tile grad_w partials (n_range x tiles x K complex).
size_t backward_workspace_bytes(int32_t n, int32_t n_range, int32_t k) {
  const size_t tiles = ((size_t)n + kBtTile - 1) / kBtTile;
  return 2 * (size_t)n * ((size_t)n_range + kRedGroups) * sizeof(float) + (size_t)n_range * tiles * k * sizeof(float2);
}

hipError_t launch_sparse_backward(const SparseArgs& a, const float2* grad_image, float2* grad_w,
                                  float* grad_dphi, float* grad_dpsi, void* ws, hipStream_t s) {
  const int n = a.g.n, nr = a.g.n_range;
  float* pd = reinterpret_cast<float*>(ws);
  float* pp = pd + (size_t)n * nr;
  float* gd = pp + (size_t)n * nr;
  float* gp = gd + (size_t)n * kRedGroups;
  float2* gwp = reinterpret_cast<float2*>(gp + (size_t)n * kRedGroups);
  hipError_t e;
  switch (a.y.dtype) {
    case ROSAR_C64: e = launch_dt<0>(a, grad_image, grad_w, pd, pp, gwp, s); break;
    case ROSAR_C16_F16: e = launch_dt<1>(a, grad_image, grad_w, pd, pp, gwp, s); break;
    default: e = launch_dt<2>(a, grad_image, grad_w, pd, pp, gwp, s); break;
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
