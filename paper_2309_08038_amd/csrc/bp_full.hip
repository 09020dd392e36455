// Full-aperture back-projection over range-compressed data (FFT+BPA, eq. 43 with the BPA
// weights alpha_n exp(-j 2 k R_n)), the comparator of the sparse filter.
//
// Prep kernel (one workgroup): per pulse, the deviation d_n of its angle from the nominal
// phi0 + 2 pi n / N (wrapped to (-pi, pi]) as (sin(d_n / 2), cos(d_n / 2)) in float32, and the
// largest |d_n|, written to the caller's workspace.
//
// Main kernel: a workgroup owns one range row and kBpTile consecutive azimuth bins (kBpP per
// lane, 64 apart).  It walks the pulse offsets o = n - a that can be visible from its row:
// |o| up to (acos(r / R) + max |d|) / (2 pi / N) + 1, or every pulse once when that covers the
// rotation.  With D0 = 2 pi o / N the angle between pixel a and pulse n is D = D0 + d_n (eqs.
// 2-5 with the pixel centred on pulse a).  Per chunk of offsets the workgroup computes the
// nominal geometry in float64 (R_nom = R(D0), beta R_nom of eq. 40, the phase 2 k R_nom in
// revolutions) into LDS, and stages the pulse corrections of the columns the chunk touches.
// Per (pixel, pulse) only the correction is evaluated, in float32, one of two ways chosen per
// workgroup (as in the corrected sparse filter):
//  - series, when the fourth-derivative remainder bound at the largest |d| is below 1e-6 rad of
//    carrier phase and 2^-20 bins (and beta r max|d| < 1/2): R_n - R_nom = d (q1 + d (q2 + d q3))
//    and v = R cos D - r = v0 + d (v1 + d (v2 + d v3)) (Taylor coefficients at D0 in float64 per
//    offset; the cosine's remainder R d^4 / 24 is required below 1e-8 m);
//  - exact otherwise, without cancellation:
//    R_n^2 - R_nom^2 = 4 R r sin(D0 + d/2) sin(d/2),  R_n - R_nom = (R_n^2 - R_nom^2)/(R_n + R_nom),
//    v = (R^2 - r^2 - R_n^2) / (2 r).
// The bin is beta R_nom + beta (R_n - R_nom) in float64, the phase adds 2 k (R_n - R_nom), and
// alpha = max(v, 0) / R_n (eqs. 3, 8, 15).
// Neighbouring lanes read neighbouring columns of the same bin row: coalesced loads.
#include <mutex>
#include <type_traits>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kBpThreads = 256;
constexpr int kBpP = 2;                          // pixels per lane
constexpr int kBpTile = kBpThreads * kBpP;       // pixels per workgroup
constexpr int kBpChunk = kBpThreads;             // offsets per chunk (one per thread)
constexpr size_t kBpHeader = 256;                // bytes before the per-pulse table

// Nominal geometry of one offset o (no angle error), 64 bytes.
struct alignas(16) BpTap {
  SplitBin u;     // beta * R_nom - l_lo (+ 1/2 for NEAREST): FFT bin of eq. 40, split
  float r2;       // R_nom^2
  float rnom;     // R_nom
  float sd, cd;   // sin, cos of D0 = 2 pi o / N
  float ph;       // k R_nom / pi - rint(.): revolutions of exp(j 2 k R_nom), in [-1/2, 1/2]
  int32_t near;   // NEAREST: a correction of this offset can bring the bin near a rounding tie
  float q1, q2, q3;   // R(D0 + d) - R_nom = d (q1 + d (q2 + d q3))
  float v0, v1, v2, v3;   // R cos(D0 + d) - r = v0 + d (v1 + d (v2 + d v3))
};

__global__ __launch_bounds__(1024) void bp_prep_kernel(int32_t n, double phi0, double step,
                                                       const double* __restrict__ angles,
                                                       double* __restrict__ ws) {
  __shared__ double red[1024 / kWave];
  float2* table = reinterpret_cast<float2*>(reinterpret_cast<char*>(ws) + kBpHeader);
  double dmax = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double d = 0.0;
    if (angles) {
      d = angles[i] - (phi0 + step * i);
      d -= 6.283185307179586477 * rint(d * 0.15915494309189533577);
    }
    double s, c;
    sincos(0.5 * d, &s, &c);
    table[i] = make_float2((float)s, (float)c);
    dmax = fmax(dmax, fabs(d));
  }
  for (int off = kWave / 2; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, red[w]);
    ws[0] = m;
  }
}

template <int DT, int INTERP>
__global__ __launch_bounds__(kBpThreads) void bp_kernel(Geo g, View y, int tiles_per_row, int nblocks,
                                                       const double* __restrict__ ws,
                                                       const double* __restrict__ angles,
                                                       const char* __restrict__ ydata,
                                                       float2* __restrict__ image) {
  __shared__ BpTap s_tap[kBpChunk];
  __shared__ float2 s_del[kBpChunk + kBpTile];   // pulse corrections of columns a0 + c0 + j
  __shared__ float s_d[kBpChunk + kBpTile];      // their angle errors d (series path)
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int a0 = tile * kBpTile;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int i_wave = wave * kWave * kBpP;   // first pixel of this wave within the tile

  const double rr = g.r0 + row * g.dr;
  const double r = g.radius;
  float2 acc[kBpP];
#pragma unroll
  for (int p = 0; p < kBpP; ++p) acc[p] = make_float2(0.f, 0.f);

  if (rr > r) {   // otherwise no pulse sees the row (v <= R - r <= 0)
    const float2* del = reinterpret_cast<const float2*>(reinterpret_cast<const char*>(ws) + kBpHeader);
    const double dmax = ws[0];
    const double reach = (acos(r / rr) + dmax) / g.step;
    bool series = false;
    {
      const double rho = rr - r;
      const double c = 2.0 * rr * r;
      const double m4 = 2.0 * (c / (2.0 * rho) + 0.75 * c * c / (rho * rho * rho));
      const double rem = m4 * dmax * dmax * dmax * dmax / 24.0;   // metres
      series = rem * (kTwoPiD * g.k_over_pi) <= 1e-6 && rem * g.beta <= 0x1p-20 && g.beta * r * dmax < 0.5 &&
               rr * dmax * dmax * dmax * dmax / 24.0 <= 1e-8;
    }
    const int span = reach >= (double)n ? n : (int)reach + 1;
    int o_lo, o_hi;   // inclusive offset range, each pulse at most once per pixel
    if (2 * span + 1 >= n) {
      o_lo = -(n / 2);
      o_hi = o_lo + n - 1;
    } else {
      o_lo = -span;
      o_hi = span;
    }
    const double c1 = rr * rr + r * r;
    const double c2 = 2.0 * rr * r;
    const float c4 = (float)(2.0 * c2);         // 4 R r
    const float k1 = (float)(rr * rr - r * r);  // R^2 - r^2
    const float inv2r = (float)(0.5 / r);
    const float kpi = (float)g.k_over_pi;
    const float beta = (float)g.beta;
    constexpr int ES = Elem<DT>::bytes;
    // band rows as one buffer: a bin outside the band is an offset past its end (or a negative
    // offset, i.e. above 2^31 as unsigned), which the range check turns into a zero sample
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(ydata, (uint32_t)((int64_t)y.l_count * y.ld * ES));
    const int ld_es = (int)(y.ld * ES);
    const double u_shift = INTERP == ROSAR_NEAREST ? 0.5 - y.l_lo : -(double)y.l_lo;
    int acol[kBpP];   // pixel column, clamped into the rotation for padding lanes
#pragma unroll
    for (int p = 0; p < kBpP; ++p) acol[p] = min(a0 + i_wave + lane + kWave * p, n - 1);

    auto chunks = [&](auto series_tag) {
    constexpr bool SERIES = decltype(series_tag)::value;
    for (int c0 = o_lo; c0 <= o_hi; c0 += kBpChunk) {
      const int cnt = min(kBpChunk, o_hi - c0 + 1);
      if ((int)threadIdx.x < cnt) {
        const int o = c0 + (int)threadIdx.x;
        double s, c;
        sincos(o * g.step, &s, &c);
        const double r2 = c1 - c2 * c;
        const double rn = sqrt(r2);
        const double ph = g.k_over_pi * rn;
        BpTap t;
        t.u = split_bin(g.beta * rn + u_shift);   // band-relative bin (+ 1/2 for rounding to nearest)
        t.r2 = (float)r2;
        t.rnom = (float)rn;
        t.sd = (float)s;
        t.cd = (float)c;
        t.ph = (float)(ph - rint(ph));
        // |R_n - R_nom| is at most the chord r |d| between the nominal and the true phase centre,
        // so the corrected fraction stays within beta r max|d| of the nominal one
        const float fmax_corr = (float)(g.beta * r * dmax) * 1.0001f + 0x1p-17f;
        t.near = (t.u.f < fmax_corr || t.u.f > 1.f - fmax_corr) ? 1 : 0;
        // derivatives of R(D) = sqrt(S), S = c1 - c2 cos D, and of R cos D - r, at D0
        const double s1 = c2 * s, s2 = c2 * c;
        const double ir = 1.0 / rn, ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
        t.q1 = (float)(0.5 * s1 * ir);
        t.q2 = (float)(0.5 * (0.5 * s2 * ir - 0.25 * s1 * s1 * ir3));
        t.q3 = (float)((-0.5 * s1 * ir - 0.75 * s1 * s2 * ir3 + 0.375 * s1 * s1 * s1 * ir5) / 6.0);
        t.v0 = (float)(rr * c - r);
        t.v1 = (float)(-rr * s);
        t.v2 = (float)(-0.5 * rr * c);
        t.v3 = (float)(rr * s / 6.0);
        if constexpr (SERIES) t.u.i = min(max(t.u.i, -3), y.l_count + 2);
        s_tap[threadIdx.x] = t;
      }
      for (int j = threadIdx.x; j < cnt - 1 + kBpTile; j += kBpThreads) {
        int pn = (a0 + c0 + j) % n;
        pn += pn < 0 ? n : 0;
        s_del[j] = del[pn];
        if constexpr (SERIES) {
          // d = 2 atan2(sin(d/2), cos(d/2)) would cost; the angle error itself is recomputed
          const double dn = angles ? angles[pn] - (g.phi0 + g.step * pn) : 0.0;
          s_d[j] = (float)(dn - kTwoPiD * rint(dn / kTwoPiD));
        }
      }
      __syncthreads();
      int pc[kBpP];   // pulse column of offset c0 for each pixel, in [0, N)
#pragma unroll
      for (int p = 0; p < kBpP; ++p) {
        pc[p] = acol[p] + c0;
        pc[p] += (pc[p] < 0) ? n : 0;
        pc[p] -= (pc[p] >= n) ? n : 0;
      }
      for (int t = 0; t < cnt; ++t) {
        const BpTap tp = s_tap[t];
#pragma unroll
        for (int p = 0; p < kBpP; ++p) {
          float diff, alpha;   // R_n - R_nom, max(v, 0) / R_n
          if constexpr (SERIES) {
            const float dn = s_d[i_wave + lane + kWave * p + t];
            diff = dn * fmaf(dn, fmaf(dn, tp.q3, tp.q2), tp.q1);
            const float v = fmaf(dn, fmaf(dn, fmaf(dn, tp.v3, tp.v2), tp.v1), tp.v0);
            alpha = fmaxf(v, 0.f) * __builtin_amdgcn_rcpf(tp.rnom + diff);
          } else {
            const float2 dl = s_del[i_wave + lane + kWave * p + t];   // (sin(d/2), cos(d/2))
            const float s_mid = fmaf(tp.sd, dl.y, tp.cd * dl.x);    // sin(D0 + d/2)
            const float dd = c4 * s_mid * dl.x;                      // R_n^2 - R_nom^2
            const float r2 = fmaxf(tp.r2 + dd, 1e-30f);
            const float rs = __builtin_amdgcn_rsqf(r2);
            const float rn = r2 * rs;
            diff = dd * __builtin_amdgcn_rcpf(rn + tp.rnom);
            alpha = fmaxf((k1 - r2) * inv2r, 0.f) * rs;
          }
          const float corr = beta * diff;
          float fr;
          bool tie;
          int l = corr_bin(tp.u, corr, &fr, &tie);
          int pn = pc[p] + t;
          pn -= (pn >= n) ? n : 0;
          const int cb = (pn + y.halo) * ES;   // byte offset of the column within a row
          // rows clamped to just outside either band edge: an out-of-band sample reads zero
          float2 smp;
          if constexpr (INTERP == ROSAR_NEAREST) {
            if (tp.near && tie) {
              // plain float64 bin at D = phi_a - phi^_n (the step 2 pi / N multiplied, not divided:
              // the angles may differ from the definition's in the last bit)
              const double phi_a = g.phi0 + (double)acol[p] * g.step;
              const double phi_n = angles ? angles[pn] : g.phi0 + (double)pn * g.step;
              l = (int)floor(plain_bin_half(rr, r, phi_a - phi_n, g.beta)) - y.l_lo;
              l = min(max(l, -1), y.l_count);
            }
            if constexpr (!SERIES) l = min(max(l, -1), y.l_count);
            smp = buf_load<DT>(rsrc, (uint32_t)(__mul24(l, ld_es) + cb), 0u);
          } else {
            if constexpr (!SERIES) l = min(max(l, -2), y.l_count);
            const uint32_t off0 = (uint32_t)(__mul24(l, ld_es) + cb);
            const float2 y0 = buf_load<DT>(rsrc, off0, 0u);
            const float2 y1 = buf_load<DT>(rsrc, off0 + (uint32_t)ld_es, 0u);
            smp = make_float2(fmaf(fr, y1.x - y0.x, y0.x), fmaf(fr, y1.y - y0.y, y0.y));
          }
          float rev = fmaf(kpi, diff, tp.ph);
          if constexpr (!SERIES) rev -= floorf(rev);
          // coefficient alpha exp(-j 2 k R_n); acc += coef * smp
          const float cr = alpha * cos_rev(rev);
          const float ci = -alpha * sin_rev(rev);
          acc[p].x = fmaf(cr, smp.x, acc[p].x);
          acc[p].x = fmaf(-ci, smp.y, acc[p].x);
          acc[p].y = fmaf(cr, smp.y, acc[p].y);
          acc[p].y = fmaf(ci, smp.x, acc[p].y);
        }
      }
      __syncthreads();
    }
    };
    if (series)
      chunks(std::true_type{});
    else
      chunks(std::false_type{});
  }
  float2* out = image + (int64_t)row * n;
#pragma unroll
  for (int p = 0; p < kBpP; ++p) {
    const int a = a0 + i_wave + lane + kWave * p;
    if (a < n) out[a] = make_float2(acc[p].x * y.inv_scale, acc[p].y * y.inv_scale);
  }
}

template <int DT>
hipError_t launch_dt(const Geo& g, const View& y, int32_t interp, float2* image, const double* ws,
                     const double* angles, hipStream_t s) {
  const int tiles = (g.n + kBpTile - 1) / kBpTile;
  const int nblocks = tiles * g.n_range;
  const char* yd = reinterpret_cast<const char*>(y.data);
  if (interp == ROSAR_LINEAR)
    bp_kernel<DT, ROSAR_LINEAR><<<nblocks, kBpThreads, 0, s>>>(g, y, tiles, nblocks, ws, angles, yd, image);
  else
    bp_kernel<DT, ROSAR_NEAREST><<<nblocks, kBpThreads, 0, s>>>(g, y, tiles, nblocks, ws, angles, yd, image);
  return hipGetLastError();
}

}  // namespace

size_t bp_workspace_bytes(int32_t n) { return kBpHeader + (size_t)n * sizeof(float2); }

// The allocation-free entry point's per-pulse table lives in this file-scope device array, one
// copy per GPU (the largest angle error, then (sin(d_n/2), cos(d_n/2)) per pulse).  Host code
// never passes the array's name to a kernel: it takes the device address from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[kBpHeader + (size_t)kBpNoAllocMaxPulses * sizeof(float2)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t bp_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_bp_full(const Geo& g, const View& y, const double* angles, int32_t interp,
                          float2* image, void* ws, hipStream_t s) {
  double* w = reinterpret_cast<double*>(ws);
  bp_prep_kernel<<<1, 1024, 0, s>>>(g.n, g.phi0, g.step, angles, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (y.dtype) {
    case ROSAR_C64: return launch_dt<0>(g, y, interp, image, w, angles, s);
    case ROSAR_C16_F16: return launch_dt<1>(g, y, interp, image, w, angles, s);
    default: return launch_dt<2>(g, y, interp, image, w, angles, s);
  }
}

}  // namespace rosar
