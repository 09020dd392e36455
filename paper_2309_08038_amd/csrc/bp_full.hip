// Full-aperture back-projection over range-compressed data (FFT+BPA, eq. 43 with the BPA
// weights alpha_n exp(-j 2 k R_n)), the comparator of the sparse filter.
//
// Prep kernel (one workgroup): per-pulse float64 table (cos phi^_n, sin phi^_n) and the largest
// deviation of any pulse angle from its nominal position, written to the caller's workspace.
// Main kernel: a workgroup owns one range row and 256 consecutive azimuth bins (one per lane).
// It walks the pulses that can be visible from any of its pixels: |a - n| steps up to
// (acos(r/R) + max deviation) / (2 pi / N) + 1, or the whole rotation when that covers it.
// Per (pixel, pulse), in float64: cos D = cos phi_a cos phi^_n + sin phi_a sin phi^_n (table
// values arrive through scalar loads, the pulse being wave-uniform), visibility v = R cos D - r
// (eqs. 4-5), R_n (eq. 2), the bin (eq. 40) and the phase 2 k R_n reduced to revolutions; then
// in float32 alpha = v / R_n (eqs. 3, 8, 15), the hardware sine/cosine and the complex MAC.
#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kBpThreads = 256;
constexpr size_t kBpHeader = 256;  // bytes before the per-pulse table

__global__ __launch_bounds__(1024) void bp_prep_kernel(int32_t n, double phi0, double step,
                                                       const double* __restrict__ angles,
                                                       double* __restrict__ ws) {
  __shared__ double red[1024 / kWave];
  double* table = ws + kBpHeader / sizeof(double);
  double dmax = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double nominal = phi0 + step * i;
    const double ang = angles ? angles[i] : nominal;
    double s, c;
    sincos(ang, &s, &c);
    table[2 * i] = c;
    table[2 * i + 1] = s;
    double d = ang - nominal;
    d -= 6.283185307179586477 * rint(d * 0.15915494309189533577);
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
                                                       const char* __restrict__ ydata,
                                                       float2* __restrict__ image) {
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int a0 = tile * kBpThreads;
  const int a = a0 + threadIdx.x;
  if (a0 + (int)(threadIdx.x & ~(kWave - 1)) >= n) return;
  const int ac = min(a, n - 1);
  const int a_last = min(a0 + kBpThreads, n) - 1;

  const double rr = g.r0 + row * g.dr;
  const double r = g.radius;
  float2 acc = make_float2(0.f, 0.f);
  if (rr > r) {
    const double c1 = rr * rr + r * r;
    const double c2 = 2.0 * rr * r;
    const double* table = ws + kBpHeader / sizeof(double);
    const double dmax = ws[0];
    double sa, ca;
    sincos(g.phi0 + g.step * ac, &sa, &ca);
    // pulses that may be visible from some pixel of this block
    const double reach = (acos(r / rr) + dmax) / g.step;
    const int span = reach >= (double)n ? n : (int)reach + 1;
    int first, count;
    if (2 * span + (a_last - a0) + 1 >= n) {
      first = 0;
      count = n;
    } else {
      first = a0 - span;
      count = 2 * span + (a_last - a0) + 1;
    }
    const double kpi = g.k_over_pi;
    for (int i = 0; i < count; ++i) {
      int pn = first + i;
      pn += (pn < 0) ? n : 0;
      pn -= (pn >= n) ? n : 0;
      const double cn = table[2 * pn];
      const double sn = table[2 * pn + 1];
      const double cosd = ca * cn + sa * sn;
      const double v = rr * cosd - r;
      if (v > 0.0) {
        const double rn = sqrt(c1 - c2 * cosd);
        const double u = g.beta * rn;
        const int64_t col = pn + y.halo;
        float2 smp;
        if constexpr (INTERP == ROSAR_NEAREST) {
          const int l = (int)floor(u + 0.5) - y.l_lo;
          smp = (l >= 0 && l < y.l_count) ? load_c<DT>(ydata, l * y.ld + col) : make_float2(0.f, 0.f);
        } else {
          const double fl = floor(u);
          const float f = (float)(u - fl);
          const int l = (int)fl - y.l_lo;
          const float2 y0 = (l >= 0 && l < y.l_count) ? load_c<DT>(ydata, l * y.ld + col) : make_float2(0.f, 0.f);
          const float2 y1 = (l + 1 >= 0 && l + 1 < y.l_count) ? load_c<DT>(ydata, (l + 1) * y.ld + col)
                                                               : make_float2(0.f, 0.f);
          smp = make_float2(fmaf(f, y1.x - y0.x, y0.x), fmaf(f, y1.y - y0.y, y0.y));
        }
        const float alpha = (float)(v / rn);
        const float fr = frac_rev(kpi * rn);
        // coefficient alpha exp(-j 2 k R_n); acc += coef * smp
        const float cr = alpha * cos_rev(fr);
        const float ci = -alpha * sin_rev(fr);
        acc.x = fmaf(cr, smp.x, acc.x);
        acc.x = fmaf(-ci, smp.y, acc.x);
        acc.y = fmaf(cr, smp.y, acc.y);
        acc.y = fmaf(ci, smp.x, acc.y);
      }
    }
  }
  if (a < n) image[(int64_t)row * n + a] = make_float2(acc.x * y.inv_scale, acc.y * y.inv_scale);
}

template <int DT>
hipError_t launch_dt(const Geo& g, const View& y, int32_t interp, float2* image, const double* ws,
                     hipStream_t s) {
  const int tiles = (g.n + kBpThreads - 1) / kBpThreads;
  const int nblocks = tiles * g.n_range;
  const char* yd = reinterpret_cast<const char*>(y.data);
  if (interp == ROSAR_LINEAR)
    bp_kernel<DT, ROSAR_LINEAR><<<nblocks, kBpThreads, 0, s>>>(g, y, tiles, nblocks, ws, yd, image);
  else
    bp_kernel<DT, ROSAR_NEAREST><<<nblocks, kBpThreads, 0, s>>>(g, y, tiles, nblocks, ws, yd, image);
  return hipGetLastError();
}

}  // namespace

size_t bp_workspace_bytes(int32_t n) { return kBpHeader + (size_t)n * 2 * sizeof(double); }

hipError_t launch_bp_full(const Geo& g, const View& y, const double* angles, int32_t interp,
                          float2* image, void* ws, hipStream_t s) {
  double* w = reinterpret_cast<double*>(ws);
  bp_prep_kernel<<<1, 1024, 0, s>>>(g.n, g.phi0, g.step, angles, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (y.dtype) {
    case ROSAR_C64: return launch_dt<0>(g, y, interp, image, w, s);
    case ROSAR_C16_F16: return launch_dt<1>(g, y, interp, image, w, s);
    default: return launch_dt<2>(g, y, interp, image, w, s);
  }
}

}  // namespace rosar
