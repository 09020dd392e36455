// Sparse-aperture azimuth filter (Algorithm 2 with eq. 43): every polar pixel (row i,
// azimuth a) is the conjugate-weighted sum of K range-compressed samples, one per selected
// pulse a + o_t, each read at the FFT bin of that pulse's slant range (eq. 40).
//
// Plain path (no angle/phase correction).  Under the rotation symmetry the bin and weight of a
// tap depend only on (row, offset), so a whole wavefront shares them: the tap table is built
// once per wave in float64 (lane t owns tap t), then each tap's row offset is broadcast with
// v_readlane into an SGPR and its weight comes through a scalar load.  Every lane owns P
// pixels spaced one wavefront apart, so a tap costs P coalesced loads from the (L2-resident)
// range-compressed rows and 4P FMAs, with no per-lane address arithmetic.  LINEAR
// interpolation is two sub-taps with real factors (1-f, f) folded into the weight.
//
// Corrected path (per-pulse angle error dphi and phase error psi).  The slant range now varies
// per (pixel, tap) through dphi[n], so each pair evaluates the float64 geometry
// cos(D0 + dphi) = cos D0 cos dphi - sin D0 sin dphi with per-column cos/sin tables staged in
// LDS, a float64 square root, the bin, and the phase correction exp(-j 2k (R^ - R_nom) - j psi)
// on the hardware sine/cosine after a float64 range reduction.
#include "sparse_device.hpp"

namespace rosar {
namespace {

// U consecutive taps starting at tap tt of the current 64-tap chunk: loads first, then FMAs.
// MASKED: sub-taps without a sample and taps at or beyond `cnt` contribute zero.
template <int DT, int WDT, int INTERP, int P, int U, bool MASKED>
__device__ __forceinline__ void tap_group(float2 (&acc)[P], __amdgpu_buffer_rsrc_t rsrc, const uint32_t (&voff)[P],
                                          const int (&soff)[INTERP == ROSAR_LINEAR ? 2 : 1],
                                          const float (&fac)[INTERP == ROSAR_LINEAR ? 2 : 1],
                                          const void* __restrict__ weights, int64_t wbase, int tt, int cnt) {
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  float2 yv[U][NSUB][P];
  float2 wv[U][NSUB];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int ti = MASKED ? min(tt + u, cnt - 1) : tt + u;
    const float2 w = load_w<WDT>(weights, wbase + ti);
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      int so = readlane(soff[s], ti);
      float2 ws = w;
      if constexpr (INTERP == ROSAR_LINEAR) {
        const float fs = readlane(fac[s], ti);
        ws = make_float2(w.x * fs, w.y * fs);
      }
      if constexpr (MASKED) {
        const bool live = so >= 0 && tt + u < cnt;
        ws = live ? ws : make_float2(0.f, 0.f);
        so = live ? so : 0;
      }
      wv[u][s] = ws;
#pragma unroll
      for (int p = 0; p < P; ++p) yv[u][s][p] = buf_load<DT>(rsrc, voff[p], (uint32_t)so);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
      for (int p = 0; p < P; ++p) cmac_conj(acc[p], wv[u][s], yv[u][s][p]);
}

template <int DT, int WDT, int INTERP, int P, int NW>
__global__ __launch_bounds__(kWave* NW) void sparse_plain_kernel(
    Geo g, View y, int32_t k, int32_t window, int tiles_per_row, int nblocks,
    const int32_t* __restrict__ offsets, const void* __restrict__ weights,
    const char* __restrict__ ydata, float2* __restrict__ image) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int TW = kWave * P;  // pixels per wave
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  constexpr int U = (P * NSUB >= 8) ? 2 : 4;  // taps per load group
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int a_wave = tile * (TW * NW) + wave * TW;
  if (a_wave >= n) return;  // no barriers below: idle waves may leave

  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(ydata, (uint32_t)(y.l_count * y.ld * ES));
  // per-lane byte offsets of the P pixels (clamped inside the row; clamped lanes are not stored)
  uint32_t voff[P];
#pragma unroll
  for (int p = 0; p < P; ++p) voff[p] = (uint32_t)(min(a_wave + lane + kWave * p, n - 1) * ES);
  float2 acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = make_float2(0.f, 0.f);

  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  const int half_w = window / 2;
  const int64_t wrow = (int64_t)row * k;

  for (int c0 = 0; c0 < k; c0 += kWave) {
    // ---- tap table for taps c0 + lane (float64 geometry, eq. 2 and eq. 40).
    // rowel[s]: element offset of the bin row of sub-tap s, or -1 when that bin is outside the
    // band or the offset outside the window; fac[s]: real factor of the sub-tap (LINEAR:
    // 1-f and f; NEAREST: implicit 1).
    const int t = c0 + lane;
    float fac[NSUB];
    int ofs = 0, rowel[NSUB];
#pragma unroll
    for (int s = 0; s < NSUB; ++s) { fac[s] = 0.f; rowel[s] = -1; }
    if (t < k) {
      ofs = offsets[wrow + t];
      if (ofs >= -half_w && ofs < half_w) {
        const double rn = sqrt(c1 - c2 * cos(ofs * g.step));
        const double u = g.beta * rn;
        int l;
        if constexpr (INTERP == ROSAR_NEAREST) {
          l = (int)floor(u + 0.5) - y.l_lo;
        } else {
          const double fl = floor(u);
          const float f = (float)(u - fl);
          l = (int)fl - y.l_lo;
          fac[0] = 1.f - f;
          fac[NSUB - 1] = f;
        }
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
          if (l + s >= 0 && l + s < y.l_count) rowel[s] = (int)((l + s) * y.ld);
        }
      }
    }
    // whole row inside the stored halo (the usual case, halo >= window/2)
    const bool direct_lane = (ofs >= -y.halo) && (ofs < y.halo);
    const bool all_direct = __builtin_amdgcn_ballot_w64(!direct_lane && t < k) == 0;
    const int cnt = min(kWave, k - c0);
    if (all_direct) {
      // soff: byte offset of (bin row, column o + halo), -1 for an empty sub-tap
      int soff[NSUB];
#pragma unroll
      for (int s = 0; s < NSUB; ++s) soff[s] = rowel[s] >= 0 ? (rowel[s] + ofs + y.halo) * ES : -1;
      // every tap of the chunk has its samples (the usual case): unmasked groups of U taps, all
      // loads of a group issued before its FMAs, then single taps for the remainder
      const bool all_live = __builtin_amdgcn_ballot_w64(t < k && (rowel[0] < 0 || rowel[NSUB - 1] < 0)) == 0;
      int tt = 0;
      if (all_live) {
        for (; tt + U <= cnt; tt += U) tap_group<DT, WDT, INTERP, P, U, false>(acc, rsrc, voff, soff, fac, weights, wrow + c0, tt, cnt);
      }
      // masked groups: empty sub-taps and the padding past `cnt` get a zero weight and read
      // offset 0
      for (; tt < cnt; tt += U) tap_group<DT, WDT, INTERP, P, U, true>(acc, rsrc, voff, soff, fac, weights, wrow + c0, tt, cnt);
    } else {
      // some offsets reach past the halo: wrap the pulse index per pixel
      for (int tt = 0; tt < cnt; ++tt) {
        const int o = readlane(ofs, tt);
        const float2 w = load_w<WDT>(weights, wrow + c0 + tt);
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
          const int re = readlane(rowel[s], tt);
          if (re < 0) continue;
          const float fs = INTERP == ROSAR_NEAREST ? 1.f : readlane(fac[s], tt);
          const float2 ws = make_float2(w.x * fs, w.y * fs);
#pragma unroll
          for (int p = 0; p < P; ++p) {
            int a = (int)(voff[p] / ES) + o;
            a += (a < 0) ? n : 0;
            a -= (a >= n) ? n : 0;
            cmac_conj(acc[p], ws, buf_load<DT>(rsrc, (uint32_t)((a + y.halo) * ES), (uint32_t)(re * ES)));
          }
        }
      }
    }
  }
  float2* out = image + (int64_t)row * n;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int a = a_wave + lane + kWave * p;
    if (a < n) out[a] = make_float2(acc[p].x * y.inv_scale, acc[p].y * y.inv_scale);
  }
}

constexpr int kCorrThreads = 256;
constexpr int kCorrMaxCols = 2048;  // LDS table columns (tile + window)

template <int DT, int WDT, int INTERP, bool TABLE>
__global__ __launch_bounds__(kCorrThreads) void sparse_corrected_kernel(
    Geo g, View y, int32_t k, int32_t window, int tiles_per_row, int nblocks,
    const int32_t* __restrict__ offsets, const void* __restrict__ weights,
    const float* __restrict__ dphi, const float* __restrict__ dpsi,
    const char* __restrict__ ydata, float2* __restrict__ image) {
  __shared__ double s_cos[TABLE ? kCorrMaxCols : 1];
  __shared__ double s_sin[TABLE ? kCorrMaxCols : 1];
  __shared__ float s_psi[TABLE ? kCorrMaxCols : 1];
  const int lane = threadIdx.x & (kWave - 1);
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int half_w = window / 2;
  const int a0 = tile * kCorrThreads;
  const int a = a0 + threadIdx.x;
  constexpr double kInv2Pi = 0.15915494309189533577;

  if constexpr (TABLE) {
    // columns c <-> pulse (a0 - W/2 + c) mod N
    const int ncol = kCorrThreads + window;
    for (int c = threadIdx.x; c < ncol; c += kCorrThreads) {
      int pn = a0 - half_w + c;
      pn %= n;
      if (pn < 0) pn += n;
      const double d = dphi ? (double)dphi[pn] : 0.0;
      double sd, cd;
      sincos(d, &sd, &cd);
      s_cos[c] = cd;
      s_sin[c] = sd;
      s_psi[c] = dpsi ? dpsi[pn] : 0.f;
    }
    __syncthreads();
  }
  if (a0 + (threadIdx.x & ~(kWave - 1)) >= n) return;  // whole wave past the row end
  const int ac = min(a, n - 1);

  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  const int64_t wrow = (int64_t)row * k;
  float2 acc = make_float2(0.f, 0.f);

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
      const float2 w = load_w<WDT>(weights, wrow + c0 + tt);
      int pn = ac + o;
      pn += (pn < 0) ? n : 0;
      pn -= (pn >= n) ? n : 0;
      double cd, sd;
      float ps;
      if constexpr (TABLE) {
        const int c = ac - a0 + o + half_w;
        cd = s_cos[c];
        sd = s_sin[c];
        ps = s_psi[c];
      } else {
        const double d = dphi ? (double)dphi[pn] : 0.0;
        sincos(d, &sd, &cd);
        ps = dpsi ? dpsi[pn] : 0.f;
      }
      const double cosd = cD0 * cd - sD0 * sd;
      const double rh = sqrt(c1 - c2 * cosd);
      const double u = g.beta * rh;
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
      // exp(-j (2k (R^ - R_nom) + psi)), phase counted in revolutions and reduced in float64
      const float fr = frac_rev(g.k_over_pi * (rh - rN) + (double)ps * kInv2Pi);
      const float2 rot = make_float2(cos_rev(fr), -sin_rev(fr));
      cmac_conj(acc, w, cmul(smp, rot));
    }
  }
  if (a < n) image[(int64_t)row * n + a] = make_float2(acc.x * y.inv_scale, acc.y * y.inv_scale);
}

template <int DT, int WDT, int INTERP, int P, int NW>
__global__ __launch_bounds__(kWave* NW) void sparse_lds_kernel(Geo g, View y, int32_t k, int32_t window,
                                                               int tiles_per_row, int nblocks, int rows_cap,
                                                               double cos_hw, int stride, int use_dma,
                                                               const int32_t* __restrict__ offsets,
                                                               const void* __restrict__ weights,
                                                               const char* __restrict__ ydata,
                                                               float2* __restrict__ image) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_unstaged;
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  sparse::lds_tile<DT, WDT, INTERP, P, NW>(g, y, k, window, row, blk - row * tiles_per_row, rows_cap,
                                           cos_hw, stride, use_dma, offsets, weights, ydata, image, smem, s_unstaged);
}

template <int DT, int WDT, int INTERP, int P, int NW>
hipError_t launch_lds_t(const SparseArgs& a, hipStream_t s, bool* fits) {
  constexpr int T = kWave * P * NW;
  const sparse::LdsLayout L = sparse::lds_layout_capped(a.g, a.y, a.k, a.window, INTERP, T);
  *fits = L.bytes <= sparse::kLdsBudget;
  if (!*fits) return hipSuccess;
  const int tiles = (a.g.n + T - 1) / T;
  const int nblocks = tiles * a.g.n_range;
  sparse_lds_kernel<DT, WDT, INTERP, P, NW><<<nblocks, kWave * NW, L.bytes, s>>>(
      a.g, a.y, a.k, a.window, tiles, nblocks, L.rows, L.cos_hw, L.stride, L.dma, a.offsets, a.weights,
      reinterpret_cast<const char*>(a.y.data), a.image);
  return hipGetLastError();
}

template <int DT, int WDT, int INTERP, int P, int NW>
hipError_t launch_plain_t(const SparseArgs& a, hipStream_t s) {
  const int tw = kWave * P * NW;
  const int tiles = (a.g.n + tw - 1) / tw;
  const int nblocks = tiles * a.g.n_range;
  sparse_plain_kernel<DT, WDT, INTERP, P, NW><<<nblocks, kWave * NW, 0, s>>>(
      a.g, a.y, a.k, a.window, tiles, nblocks, a.offsets, a.weights,
      reinterpret_cast<const char*>(a.y.data), a.image);
  return hipGetLastError();
}

template <int DT, int WDT, int INTERP>
hipError_t launch_plain_shape(const SparseArgs& a, const Tile& t, hipStream_t s) {
#define ROSAR_SHAPE(P, NW)                                                     \
  if (t.ppl == P && t.waves == NW) {                                           \
    if (t.variant == 2) {                                                      \
      bool fits = false;                                                       \
      hipError_t e = launch_lds_t<DT, WDT, INTERP, P, NW>(a, s, &fits);        \
      if (fits) return e;                                                      \
    }                                                                          \
    return launch_plain_t<DT, WDT, INTERP, P, NW>(a, s);                       \
  }
  ROSAR_SHAPE(1, 4) ROSAR_SHAPE(2, 4) ROSAR_SHAPE(4, 4) ROSAR_SHAPE(8, 4)
  ROSAR_SHAPE(1, 2) ROSAR_SHAPE(2, 2) ROSAR_SHAPE(4, 2) ROSAR_SHAPE(8, 2)
  ROSAR_SHAPE(1, 1) ROSAR_SHAPE(2, 1) ROSAR_SHAPE(4, 1) ROSAR_SHAPE(8, 1)
  ROSAR_SHAPE(1, 8) ROSAR_SHAPE(2, 8) ROSAR_SHAPE(4, 8)
#undef ROSAR_SHAPE
  return hipErrorInvalidValue;
}

template <int DT>
hipError_t launch_plain_dt(const SparseArgs& a, const Tile& t, hipStream_t s) {
  const bool lin = a.interp == ROSAR_LINEAR;
  if (a.w_dtype == ROSAR_C64)
    return lin ? launch_plain_shape<DT, 0, ROSAR_LINEAR>(a, t, s) : launch_plain_shape<DT, 0, ROSAR_NEAREST>(a, t, s);
  return lin ? launch_plain_shape<DT, 1, ROSAR_LINEAR>(a, t, s) : launch_plain_shape<DT, 1, ROSAR_NEAREST>(a, t, s);
}

template <int DT, int WDT, int INTERP>
hipError_t launch_corr_t(const SparseArgs& a, hipStream_t s) {
  const int tiles = (a.g.n + kCorrThreads - 1) / kCorrThreads;
  const int nblocks = tiles * a.g.n_range;
  const char* yd = reinterpret_cast<const char*>(a.y.data);
  if (kCorrThreads + a.window <= kCorrMaxCols) {
    sparse_corrected_kernel<DT, WDT, INTERP, true><<<nblocks, kCorrThreads, 0, s>>>(
        a.g, a.y, a.k, a.window, tiles, nblocks, a.offsets, a.weights, a.dphi, a.dpsi, yd, a.image);
  } else {
    sparse_corrected_kernel<DT, WDT, INTERP, false><<<nblocks, kCorrThreads, 0, s>>>(
        a.g, a.y, a.k, a.window, tiles, nblocks, a.offsets, a.weights, a.dphi, a.dpsi, yd, a.image);
  }
  return hipGetLastError();
}

template <int DT>
hipError_t launch_corr_dt(const SparseArgs& a, hipStream_t s) {
  const bool lin = a.interp == ROSAR_LINEAR;
  if (a.w_dtype == ROSAR_C64)
    return lin ? launch_corr_t<DT, 0, ROSAR_LINEAR>(a, s) : launch_corr_t<DT, 0, ROSAR_NEAREST>(a, s);
  return lin ? launch_corr_t<DT, 1, ROSAR_LINEAR>(a, s) : launch_corr_t<DT, 1, ROSAR_NEAREST>(a, s);
}

}  // namespace

Tile default_tile(int32_t n, int32_t k, int32_t y_dtype) {
  (void)k;
  // LDS-staged window of 2048-pixel tiles: complex64 samples four pixels per lane over eight
  // waves, 16-bit samples eight pixels per lane over four waves (the faster shape of each on
  // the 3600- and 7200-pulse workloads); short rotations one pixel per lane
  if (n <= 1024) return Tile{2, 1, 4};
  return y_dtype == ROSAR_C64 ? Tile{2, 4, 8} : Tile{2, 8, 4};
}

bool tile_supported(const Tile& t) {
  if (t.variant < 0 || t.variant > 2) return false;
  const int p = t.ppl, w = t.waves;
  const bool p_ok = p == 1 || p == 2 || p == 4 || p == 8;
  const bool w_ok = w == 1 || w == 2 || w == 4 || w == 8;
  return p_ok && w_ok && !(p == 8 && w == 8);
}

hipError_t launch_sparse_plain(const SparseArgs& a, const Tile& t, hipStream_t s) {
  switch (a.y.dtype) {
    case ROSAR_C64: return launch_plain_dt<0>(a, t, s);
    case ROSAR_C16_F16: return launch_plain_dt<1>(a, t, s);
    default: return launch_plain_dt<2>(a, t, s);
  }
}

hipError_t launch_sparse_corrected(const SparseArgs& a, hipStream_t s) {
  switch (a.y.dtype) {
    case ROSAR_C64: return launch_corr_dt<0>(a, s);
    case ROSAR_C16_F16: return launch_corr_dt<1>(a, s);
    default: return launch_corr_dt<2>(a, s);
  }
}

}  // namespace rosar
