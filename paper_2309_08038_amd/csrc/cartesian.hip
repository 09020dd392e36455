// Algorithm 2 for targets on a Cartesian lattice (FFT+SAS form, eq. 43).  For the target at
// (x, y): R_t = |(x, y)|, phi_t = atan2(y, x); the weights are those of the polar grid row
// nearest to R_t (targets more than half a row spacing outside the rows get zero); the central
// phase centre is n_c = round((phi_t - phi0) / phi_Delta); tap k reads pulse (n_c + o_k) mod N
// at the bin of the slant range from that pulse to the target (eq. 2, eq. 40).  Without the
// rotation symmetry each pixel has its own tap geometry: a thread owns a pixel and evaluates it
// in float64, reading the band samples from global memory.  The angle between the target and
// pulse n_c + o is D = e - o 2 pi / N with e = phi_t - phi0 - n_c 2 pi / N, so
// cos D = cos e cos(o 2 pi / N) + sin e sin(o 2 pi / N): cos e and sin e once per target, the
// offsets' cosines and sines from an LDS table of the window (windows up to kCartTableMax
// pulses; wider ones take cos D directly).  For NEAREST a bin within 1e-9 of a rounding tie is
// recomputed from the plain cos(phi_t - phi_n).
//
// POLAR: the targets are the pixels of a polar grid of A azimuth bins that need not equal N
// (Algorithm 2's round(phi_t / phi_Delta) with phi_t = phi0 + 2 pi a / A): pixel (i, a) has
// R_t = R_i, the weights of row i, and the same per-pixel tap geometry.  A = N gives the
// plain sparse filter's image.
#include <hip/hip_runtime.h>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kCartThreads = 256;
constexpr int kCartU = 4;   // taps whose sample gathers are issued together
// back-projection: the per-pulse (cos, sin) table in LDS up to this size (N <= 3840), else
// cos(phi - theta_n) per pulse and pixel
constexpr size_t kCartPulseTableBytes = 60 * 1024;
constexpr int kCartTableMax = 4096;   // widest window whose (cos, sin) table goes to LDS (64 KB)

template <int DT, int WDT, int INTERP, bool POLAR>
__global__ __launch_bounds__(kCartThreads) void sparse_cartesian_kernel(Geo g, View y, CartGrid c, int32_t k,
                                                                        int32_t half_w, int use_table,
                                                                        const int32_t* __restrict__ offsets,
                                                                        const void* __restrict__ weights,
                                                                        float2* __restrict__ image) {
  extern __shared__ double2 s_cs[];   // [2 half_w]: (cos, sin) of o 2 pi / N, o in [-half_w, half_w)
  for (int j = threadIdx.x; use_table && j < 2 * half_w; j += kCartThreads) {
    double sn, cs;
    sincos((double)(j - half_w) * g.step, &sn, &cs);
    s_cs[j] = make_double2(cs, sn);
  }
  __syncthreads();
  const int ix = blockIdx.x * kCartThreads + threadIdx.x;
  const int iy = blockIdx.y;
  if (ix >= c.nx) return;   // no barrier below
  double rt, phi;
  int row;
  if constexpr (POLAR) {   // c.nx = A azimuth bins, c.ny = rows
    rt = g.r0 + iy * g.dr;
    phi = g.phi0 + ix * (6.283185307179586476925286766559 / c.nx);
    row = iy;
  } else {
    const double x = c.x0 + ix * c.dx, yy = c.y0 + iy * c.dy;
    rt = sqrt(x * x + yy * yy);
    phi = atan2(yy, x);
    row = (int)floor((rt - g.r0) / g.dr + 0.5);
  }
  const int nc = (int)floor((phi - g.phi0) / g.step + 0.5);
  float2 acc = make_float2(0.f, 0.f);
  if (row >= 0 && row < g.n_range) {
    const double c1 = rt * rt + g.radius * g.radius;
    const double c2 = 2.0 * rt * g.radius;
    double se, ce;
    sincos(phi - (g.phi0 + nc * g.step), &se, &ce);
    const char* yd = static_cast<const char*>(y.data);
    // Taps in groups of kCartU: the group's geometry and sample gathers first, so that its
    // loads are in flight together, then its multiply-adds in tap order (the sum order of
    // one tap at a time).
    for (int t0 = 0; t0 < k; t0 += kCartU) {
      float2 wv[kCartU], v0[kCartU], v1[kCartU];
      float fr[kCartU];
      bool use[kCartU], in0[kCartU], in1[kCartU];
#pragma unroll
      for (int q = 0; q < kCartU; ++q) {
        const int t = t0 + q;
        use[q] = in0[q] = in1[q] = false;
        wv[q] = v0[q] = v1[q] = make_float2(0.f, 0.f);
        fr[q] = 0.f;
        if (t >= k) continue;
        const int o = offsets[(int64_t)row * k + t];
        if (o < -half_w || o >= half_w) continue;   // outside the window: no contribution
        use[q] = true;
        wv[q] = load_w<WDT>(weights, (int64_t)row * k + t);
        const int nn = nc + o;
        double cd;
        if (use_table) {
          const double2 cso = s_cs[o + half_w];
          cd = fma(ce, cso.x, se * cso.y);
        } else {
          cd = cos(phi - (g.phi0 + nn * g.step));
        }
        double u = g.beta * sqrt(c1 - c2 * cd);
        if constexpr (INTERP == ROSAR_NEAREST) {
          if (near_bin_tie(u + 0.5, 1e-9)) u = g.beta * sqrt(c1 - c2 * cos(phi - (g.phi0 + nn * g.step)));
        }
        int n = nn % g.n;
        n += n < 0 ? g.n : 0;
        if constexpr (INTERP == ROSAR_NEAREST) {
          const int l = (int)floor(u + 0.5) - y.l_lo;
          in0[q] = l >= 0 && l < y.l_count;
          if (in0[q]) v0[q] = load_c<DT>(yd, (int64_t)l * y.ld + y.halo + n);
        } else {
          const double fl = floor(u);
          fr[q] = (float)(u - fl);
          const int l = (int)fl - y.l_lo;
          in0[q] = l >= 0 && l < y.l_count;
          in1[q] = l + 1 >= 0 && l + 1 < y.l_count;
          if (in0[q]) v0[q] = load_c<DT>(yd, (int64_t)l * y.ld + y.halo + n);
          if (in1[q]) v1[q] = load_c<DT>(yd, (int64_t)(l + 1) * y.ld + y.halo + n);
        }
      }
#pragma unroll
      for (int q = 0; q < kCartU; ++q) {
        if (!use[q]) continue;
        float2 s = make_float2(0.f, 0.f);
        if constexpr (INTERP == ROSAR_NEAREST) {
          if (in0[q]) s = v0[q];
        } else {
          const float f = fr[q];
          if (in0[q]) {
            s.x += (1.f - f) * v0[q].x;
            s.y += (1.f - f) * v0[q].y;
          }
          if (in1[q]) {
            s.x += f * v1[q].x;
            s.y += f * v1[q].y;
          }
        }
        cmac_conj(acc, wv[q], s);
      }
    }
  }
  image[(size_t)iy * c.nx + ix] = make_float2(acc.x * y.inv_scale, acc.y * y.inv_scale);
}

// Full-aperture back-projection for the same Cartesian targets (eq. 43 with the BPA weights,
// eqs. 2-5, 8): I = sum over visible n of alpha_n exp(-j 2 k R_n) Y(n, u(R_n)), D = phi_t - phi_n,
// visible iff R_t cos D - r > 0.  A thread owns a pixel and walks only the pulses whose nominal
// angle lies within acos(r / R_t) + max |delta| of the target's direction (delta: given angle
// minus nominal, its maximum reduced by each workgroup); the others cannot be visible.
// Geometry in float64, the carrier phase reduced in revolutions, float32 accumulation.
template <int DT, int INTERP>
__global__ __launch_bounds__(kCartThreads) void bp_cartesian_kernel(Geo g, View y, CartGrid c,
                                                                    const double* __restrict__ angles,
                                                                    int use_table, float2* __restrict__ image) {
  __shared__ double s_dmax[kCartThreads / kWave];
  // with use_table: (cos, sin) of every pulse angle theta_n (given, or phi0 + n phi_Delta), so
  // that cos(phi - theta_n) = cos phi cos theta_n + sin phi sin theta_n costs two FMAs
  extern __shared__ double2 s_pcs[];
  const double two_pi = 6.283185307179586476925286766559;
  for (int n = threadIdx.x; use_table && n < g.n; n += kCartThreads) {
    double sn, cs;
    sincos(angles ? angles[n] : g.phi0 + n * g.step, &sn, &cs);
    s_pcs[n] = make_double2(cs, sn);
  }
  if (use_table) __syncthreads();
  // largest deviation of the given pulse angles from the nominal ones (every thread takes part
  // before any leaves)
  double dmax = 0.0;
  if (angles) {
    for (int n = threadIdx.x; n < g.n; n += kCartThreads) {
      double d = angles[n] - (g.phi0 + n * g.step);
      d -= two_pi * rint(d / two_pi);
      dmax = fmax(dmax, fabs(d));
    }
    for (int off = kWave / 2; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
    if ((threadIdx.x & (kWave - 1)) == 0) s_dmax[threadIdx.x / kWave] = dmax;
    __syncthreads();
    for (int i = 0; i < kCartThreads / kWave; ++i) dmax = fmax(dmax, s_dmax[i]);
  }
  const int ix = blockIdx.x * kCartThreads + threadIdx.x;
  const int iy = blockIdx.y;
  if (ix >= c.nx) return;   // no barrier below
  const double x = c.x0 + ix * c.dx, yy = c.y0 + iy * c.dy;
  const double rt = sqrt(x * x + yy * yy);
  const double phi = atan2(yy, x);
  const double c1 = rt * rt + g.radius * g.radius;
  const double c2 = 2.0 * rt * g.radius;
  const char* yd = static_cast<const char*>(y.data);
  float2 acc = make_float2(0.f, 0.f);
  double sphi = 0.0, cphi = 1.0;
  if (use_table) sincos(phi, &sphi, &cphi);
  // target angle from pulse 0, reduced to [0, 2 pi): the span indices stay within about
  // [-N/2, 3N/2] for any phi0
  double rel = phi - g.phi0;
  rel -= two_pi * floor(rel / two_pi);
  int m0 = 0, m1 = g.n - 1;   // pulse indices m: pulse m mod N, nominally at phi0 + m phi_Delta
  if (rt <= g.radius) {
    m1 = -1;   // R cos D - r <= R - r <= 0: nothing visible
  } else {
    const double half = acos(g.radius / rt) + dmax;   // acos < pi / 2
    if (half < 0.5 * two_pi - g.step) {
      m0 = (int)floor((rel - half) / g.step);
      m1 = (int)ceil((rel + half) / g.step);
    }
  }
  for (int m = m0; m <= m1; ++m) {
    int n = m % g.n;
    n += n < 0 ? g.n : 0;
    double cd;
    if (use_table) {
      const double2 t = s_pcs[n];
      cd = fma(cphi, t.x, sphi * t.y);
    } else {
      cd = angles ? cos(phi - angles[n]) : cos(rel - m * g.step);
    }
    const double v = rt * cd - g.radius;
    if (v <= 0.0) continue;   // outside the field of view (eqs. 4-5)
    const double rn = sqrt(c1 - c2 * cd);
    const double u = g.beta * rn;
    float2 s = make_float2(0.f, 0.f);
    if constexpr (INTERP == ROSAR_NEAREST) {
      const int l = (int)floor(u + 0.5) - y.l_lo;
      if (l >= 0 && l < y.l_count) s = load_c<DT>(yd, (int64_t)l * y.ld + y.halo + n);
    } else {
      const double fl = floor(u);
      const float f = (float)(u - fl);
      const int l = (int)fl - y.l_lo;
      if (l >= 0 && l < y.l_count) {
        const float2 a = load_c<DT>(yd, (int64_t)l * y.ld + y.halo + n);
        s.x += (1.f - f) * a.x;
        s.y += (1.f - f) * a.y;
      }
      if (l + 1 >= 0 && l + 1 < y.l_count) {
        const float2 a = load_c<DT>(yd, (int64_t)(l + 1) * y.ld + y.halo + n);
        s.x += f * a.x;
        s.y += f * a.y;
      }
    }
    const double rev = rn * g.k_over_pi;   // exp(-j 2 k R_n) in revolutions
    float ss, cs;
    sincospif(-2.0f * (float)(rev - rint(rev)), &ss, &cs);
    const float al = (float)(v / rn);
    const float ex = al * cs, ey = al * ss;
    acc.x += ex * s.x - ey * s.y;
    acc.y += ex * s.y + ey * s.x;
  }
  image[(size_t)iy * c.nx + ix] = make_float2(acc.x * y.inv_scale, acc.y * y.inv_scale);
}

template <int DT>
hipError_t launch_bp_dt(const Geo& g, const View& y, const CartGrid& c, const double* angles, int32_t interp,
                        float2* image, hipStream_t s) {
  dim3 grid((c.nx + kCartThreads - 1) / kCartThreads, c.ny);
  const int use_table = (size_t)g.n * sizeof(double2) <= kCartPulseTableBytes ? 1 : 0;
  const size_t lds = use_table ? (size_t)g.n * sizeof(double2) : 0;
  if (interp == ROSAR_LINEAR)
    bp_cartesian_kernel<DT, ROSAR_LINEAR><<<grid, kCartThreads, lds, s>>>(g, y, c, angles, use_table, image);
  else
    bp_cartesian_kernel<DT, ROSAR_NEAREST><<<grid, kCartThreads, lds, s>>>(g, y, c, angles, use_table, image);
  return hipGetLastError();
}

template <int DT, int WDT, bool POLAR>
hipError_t launch_wdt(const SparseArgs& a, const CartGrid& c, hipStream_t s) {
  dim3 grid((c.nx + kCartThreads - 1) / kCartThreads, c.ny);
  const int half_w = a.window / 2;
  const int use_table = 2 * half_w <= kCartTableMax ? 1 : 0;
  const size_t lds = use_table ? (size_t)2 * half_w * sizeof(double2) : 0;
  if (a.interp == ROSAR_LINEAR)
    sparse_cartesian_kernel<DT, WDT, ROSAR_LINEAR, POLAR><<<grid, kCartThreads, lds, s>>>(
        a.g, a.y, c, a.k, half_w, use_table, a.offsets, a.weights, a.image);
  else
    sparse_cartesian_kernel<DT, WDT, ROSAR_NEAREST, POLAR><<<grid, kCartThreads, lds, s>>>(
        a.g, a.y, c, a.k, half_w, use_table, a.offsets, a.weights, a.image);
  return hipGetLastError();
}

template <int DT, bool POLAR>
hipError_t launch_dt(const SparseArgs& a, const CartGrid& c, hipStream_t s) {
  return a.w_dtype == ROSAR_C64 ? launch_wdt<DT, 0, POLAR>(a, c, s) : launch_wdt<DT, 1, POLAR>(a, c, s);
}

template <bool POLAR>
hipError_t launch_any(const SparseArgs& a, const CartGrid& c, hipStream_t s) {
  switch (a.y.dtype) {
    case ROSAR_C64: return launch_dt<0, POLAR>(a, c, s);
    case ROSAR_C16_F16: return launch_dt<1, POLAR>(a, c, s);
    default: return launch_dt<2, POLAR>(a, c, s);
  }
}

}  // namespace

hipError_t launch_sparse_cartesian(const SparseArgs& a, const CartGrid& c, hipStream_t s) {
  return launch_any<false>(a, c, s);
}

hipError_t launch_bp_cartesian(const Geo& g, const View& y, const CartGrid& c, const double* angles, int32_t interp,
                               float2* image, hipStream_t s) {
  switch (y.dtype) {
    case ROSAR_C64: return launch_bp_dt<0>(g, y, c, angles, interp, image, s);
    case ROSAR_C16_F16: return launch_bp_dt<1>(g, y, c, angles, interp, image, s);
    default: return launch_bp_dt<2>(g, y, c, angles, interp, image, s);
  }
}

hipError_t launch_sparse_polar(const SparseArgs& a, int32_t n_az, hipStream_t s) {
  const CartGrid c{n_az, a.g.n_range, 0.0, 0.0, 0.0, 0.0};
  return launch_any<true>(a, c, s);
}

}  // namespace rosar
