// Sparse-aperture azimuth filter (Algorithm 2 with eq. 43): every polar pixel (row i,
// azimuth a) is the conjugate-weighted sum of K range-compressed samples, one per selected
// pulse a + o_t, each read at the FFT bin of that pulse's slant range (eq. 40).
//
// Plain path (no angle/phase correction), two launch variants:
//  - LDS-staged (variant 2, the default; sparse::lds_tile): a workgroup stages the bin rows
//    its row's taps can touch into LDS at entry and reads every sample from there.
//  - Direct (variant 1, also the fallback when a window does not fit the LDS budget): under
//    the rotation symmetry the bin and weight of a tap depend only on (row, offset), so a
//    whole wavefront shares them: the tap table is built once per wave in float64 (lane t
//    owns tap t), then each tap's row offset is broadcast with v_readlane into an SGPR and its
//    weight comes through a scalar load.  Every lane owns P pixels spaced one wavefront apart,
//    so a tap costs P coalesced buffer loads from the (L2-resident) range-compressed rows and
//    4P FMAs, with no per-lane address arithmetic.
// LINEAR interpolation is two sub-taps with real factors (1-f, f) folded into the weight.
//
// Corrected path (per-pulse angle error dphi and phase error psi): see
// sparse_corrected_kernel.
#include <type_traits>

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
          l = sparse::tap_bin<INTERP>(u, g, rr, ofs) - y.l_lo;
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
constexpr int kCorrP = 4;                          // pixels per lane (64 apart)
constexpr int kCorrTile = kCorrThreads * kCorrP;   // pixels per workgroup
constexpr int kCorrChunk = 32;                     // taps per chunk, global gathers (one per thread of wave 0)
constexpr int kCorrChunkS = 64;                    // taps per chunk, staged path
constexpr int kCorrMaxCols = 4096;                 // largest per-pulse table held in LDS (T + W)
constexpr int kCorrStageCols = 2048;               // largest T + W whose band rows are staged in LDS
constexpr int kCorrStageRowsN = 2;                 // NEAREST: band rows staged per workgroup
constexpr int kCorrStageRowsL = 2;                 // LINEAR: (row, next row - row) pairs staged
constexpr int kColBatch = 8;                       // columns per thread whose loads are issued together
constexpr int kStageLoads = 3;                     // band rows loaded per staged column
static_assert(kCorrStageRowsN <= kStageLoads && kCorrStageRowsL + 1 <= kStageLoads, "staging loads");

// Nominal geometry and weight of one tap (no angle error), 64 bytes in LDS.
struct alignas(16) CorrTap {
  SplitBin u;       // band-relative bin beta * R_nom - l_lo (+ 1/2 for NEAREST), split
  float r2;         // R_nom^2
  float rnom;       // R_nom
  float sd, cd;     // sin, cos of D0 = 2 pi o / N
  float wa, wt;     // weight as |w| (zero for an offset outside the window) and arg(w) / 2 pi
  float q1, q2, q3; // series in e = beta d: R(D0 + d) - R_nom = d (q1 + e (q2 + e q3)) + O(d^4)
  int32_t o;        // offset (zero outside the window)
  int32_t ub;       // series path from global memory: byte offset of the clamped nominal row and column
  int32_t inwin;    // offset inside the window
  double u64;       // the float64 nominal bin (registers only)
};

// The staged series path's 32-byte entry of one tap.
struct alignas(16) CorrTapS {
  float uf;         // fraction of the nominal bin (1/2 outside the window)
  float q1, q2, q3; // series coefficients as in CorrTap
  float wa, wt;     // |w| and arg(w) / 2 pi
  int32_t o;        // offset (zero outside the window)
  int32_t ub;       // byte offset of (row u.i - lmin, column o + W/2) in the staged rows
};
constexpr size_t kTapBufBytes = std::max(kCorrChunk * sizeof(CorrTap), kCorrChunkS * sizeof(CorrTapS));
static_assert(sizeof(CorrTap) == 64 && sizeof(CorrTapS) == 32, "tap entry sizes");

// floor(x) converted to int32 in one instruction (the compiler emits a floor and a convert).
__device__ __forceinline__ int floor_to_int(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Corrected path: the angle error d_n and phase error psi_n of pulse n move the slant range of
// every (pixel, tap) pair: R^ = R(D0 + d_n), R(D) = sqrt(R^2 + r^2 - 2 R r cos D).  The
// workgroup (one row, kCorrTile pixels) computes the taps' nominal geometry in float64 into LDS
// and per-pulse values for the columns [a0 - W/2, a0 + T + W/2).  Per pair only the correction
// R^ - R_nom is evaluated, in float32, one of two ways:
//  - series: the cubic Taylor polynomial of R(D0 + d) - R(D0) in d, with float64 coefficients
//    per tap.  Its remainder is at most max|R''''| d^4 / 24, and |R''''| peaks at D = 0 with
//    c/(2 rho) + 3 c^2 / (4 rho^3) (c = 2 R r, rho = R - r).  The workgroup takes this path when
//    twice that bound at the largest |d| of its columns is below 1e-6 rad of carrier phase and
//    2^-20 bins, and when beta r |d| < 1/2 (|dR/dD| <= r, so the correction moves a bin by less
//    than one): the workloads' angle errors of a few milliradians are far inside it.  With
//    e = beta d and s = q1 + e (q2 + e q3), the bin is u + e s and the phase (k / pi) d s.
//    The pairs then reach only the rows floor(u +- beta r max|d|) of the row's taps; when those
//    span at most `stage_rows` rows, the workgroup copies them over its columns into LDS, each
//    sample already turned by exp(-j psi) of its pulse (zero outside the band), and the pairs
//    gather from LDS: NEAREST one float2 per sample, LINEAR the float4 (y_l, y_l+1 - y_l) so
//    that the interpolation is two FMAs on one 16-byte read.  Otherwise the pairs read the band in
//    global memory through buffer loads (out-of-band rows read zero), with the nominal bin
//    clamped once per tap to [-3, l_count + 2] and folded with the column into one offset;
//  - exact otherwise: R^2 - R_nom^2 = 4 R r sin(D0 + d/2) sin(d/2) and
//    R^ - R_nom = (R^2 - R_nom^2) / (R^ + R_nom), without cancellation, gathering from global
//    memory.
// The bin is the float64 nominal bin plus beta (R^ - R_nom), and the phase factor
// exp(-j (2 k (R^ - R_nom) + psi)) runs on the hardware sine/cosine in revolutions with the
// weight folded in: conj(w) exp(-j 2 pi x) = |w| exp(-j 2 pi (x + arg(w) / 2 pi)).
// TABLE = false (window too wide for the LDS tables) evaluates the per-pulse values for every
// pair from global memory, on the exact path.  `stage_rows` is the number of staged rows the
// dynamic LDS can hold (0: no staging).  Waves whose pixels all lie past the end of the
// rotation (the last tile of a row) skip the tap loops.
template <int DT, int WDT, int INTERP, bool TABLE>
__global__ __launch_bounds__(kCorrThreads) void sparse_corrected_kernel(
    Geo g, View y, int32_t k, int32_t window, int tiles_per_row, int nblocks, int stage_rows,
    const int32_t* __restrict__ offsets, const void* __restrict__ weights,
    const float* __restrict__ dphi, const float* __restrict__ dpsi,
    const char* __restrict__ ydata, float2* __restrict__ image) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr bool LIN = INTERP == ROSAR_LINEAR;
  constexpr int EB = LIN ? 16 : 8;   // bytes per staged element
  constexpr float kInv2Pi = 0.15915494309189533577f;
  // tap tables: kCorrChunk CorrTap (gathers from global memory) or kCorrChunkS CorrTapS (staged)
  __shared__ float4 s_tapbuf[kTapBufBytes / sizeof(float4)];
  CorrTap* s_tap = reinterpret_cast<CorrTap*>(s_tapbuf);
  CorrTapS* s_tapS = reinterpret_cast<CorrTapS*>(s_tapbuf);
  __shared__ float s_red[kCorrThreads / kWave];
  __shared__ int s_redi[2 * (kCorrThreads / kWave)];
  __shared__ int s_nfast;   // staged path: taps of the chunk on the fast path (listed first)
  // TABLE: global gathers: float4 per column; staged: stage_rows rows of float2 (NEAREST) or
  // float4 (LINEAR), then (beta d, (k / pi) d) per column
  extern __shared__ float4 s_dyn[];
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int half_w = window / 2;
  const int cols = kCorrTile + window;
  const int a0 = tile * kCorrTile;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int i_wave = wave * kWave * kCorrP;
  const double rr = g.r0 + row * g.dr;
  const float kpi = (float)g.k_over_pi;
  const float beta = (float)g.beta;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  const float c4 = (float)(2.0 * c2);   // 4 R r
  const double u_shift = INTERP == ROSAR_NEAREST ? 0.5 - y.l_lo : -(double)y.l_lo;
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(ydata, (uint32_t)((int64_t)y.l_count * y.ld * ES));
  const int ld_es = (int)(y.ld * ES);
  const int64_t wrow = (int64_t)row * k;

  // pulse of column c of the tables (columns wrap around the rotation)
  auto pulse_of = [&](int c) {
    int pn = a0 - half_w + c;
    if (pn < 0 || pn >= n) pn = ((pn % n) + n) % n;
    return pn;
  };
  // float64 nominal bin of offset o (eq. 2, eq. 40), with the sine and cosine of D0 and R_nom^2
  auto nominal = [&](int o, double& sd, double& cd, double& r2) {
    sincos(o * g.step, &sd, &cd);
    r2 = c1 - c2 * cd;
    return g.beta * sqrt(r2) + u_shift;
  };

  // offsets of the first taps and weights of the first tap chunk, requested before anything
  // waits on memory
  const int o_first = (int)threadIdx.x < k ? offsets[wrow + threadIdx.x] : 0;
  float2 w_first = make_float2(0.f, 0.f);
  if ((int)threadIdx.x < min(kCorrChunkS, k)) w_first = load_w<WDT>(weights, wrow + threadIdx.x);
  int o_next = o_first;
  float2 w_next = w_first;

  bool series = false, staged = false;
  float tie_err = 0.f;   // series paths, NEAREST: bound on the error of the float32 bin sum
  double cm = 0.0;       // series paths: bound on |x - u.f| of a pair, in bins
  int lmin = 0, nrows = 0;

  // float64 nominal geometry, weight and series coefficients of one tap (ub left zero)
  auto tap_geom = [&](int o, float2 w) {
    const bool inwin = o >= -half_w && o < half_w;
    double sd, cd, r2;
    const double u = nominal(o, sd, cd, r2);
    const double rn = sqrt(r2);
    CorrTap e;
    e.u = split_bin(u);
    e.r2 = (float)r2;
    e.rnom = (float)rn;
    e.sd = (float)sd;
    e.cd = (float)cd;
    e.wa = inwin ? (float)sqrt((double)w.x * w.x + (double)w.y * w.y) : 0.f;
    e.wt = atan2f(w.y, w.x) * (float)(1.0 / kTwoPiD);
    // derivatives of R(D) = sqrt(S), S = c1 - c2 cos D, at D0 (S' = c2 sin D0, S'' = c2 cos D0);
    // the quadratic and cubic coefficients are taken per power of e = beta d
    const double s1 = c2 * sd, s2 = c2 * cd;
    const double ir = 1.0 / rn, ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
    const double ib = 1.0 / g.beta;
    e.q1 = (float)(0.5 * s1 * ir);
    e.q2 = (float)(0.5 * (0.5 * s2 * ir - 0.25 * s1 * s1 * ir3) * ib);
    e.q3 = (float)((-0.5 * s1 * ir - 0.75 * s1 * s2 * ir3 + 0.375 * s1 * s1 * s1 * ir5) / 6.0 * ib * ib);
    e.o = inwin ? o : 0;
    e.ub = 0;
    e.inwin = inwin;
    e.u64 = u;
    return e;
  };
  // staged-path entry: byte offset of (row u.i - lmin, column o + W/2) in the staged rows; a
  // tap outside the window (zero weight) reads row 0 with li = 0
  auto staged_entry = [&](const CorrTap& e) {
    CorrTapS t;
    t.uf = e.inwin ? e.u.f : 0.5f;
    t.q1 = e.q1;
    t.q2 = e.q2;
    t.q3 = e.q3;
    t.wa = e.wa;
    t.wt = e.wt;
    t.o = e.o;
    t.ub = ((e.inwin ? e.u.i : lmin) - lmin) * (cols * EB) + (e.o + half_w) * EB;
    return t;
  };
  // wave 0 files the staged entries of its lanes' taps (valid: the lane holds a tap): first the
  // taps whose every pair has floor(x) = 0 (NEAREST: and no tie), so that they sample their
  // nominal row without the bin arithmetic, then the others; s_nfast counts the first
  auto file_staged = [&](const CorrTap& e, bool valid) {
    const CorrTapS t = staged_entry(e);
    const double margin = INTERP == ROSAR_NEAREST ? (double)tie_err : 0.0;
    const bool fast = valid && (double)t.uf - cm >= margin && (double)t.uf + cm < 1.0 - margin;
    const uint64_t fm = __builtin_amdgcn_ballot_w64(fast);
    const uint64_t sm = __builtin_amdgcn_ballot_w64(valid && !fast);
    const uint64_t below = (1ull << lane) - 1ull;
    const int nf = __builtin_popcountll(fm);
    if (valid) s_tapS[fast ? __builtin_popcountll(fm & below) : nf + __builtin_popcountll(sm & below)] = t;
    if (lane == 0) s_nfast = nf;
  };

  // one tap table for all taps, built by wave 0 while the column loads are in flight
  const bool fused = TABLE && stage_rows > 0 && k <= kCorrChunkS;
  CorrTap tap0{};
  // (d, psi) of every column, in the dynamic LDS past the tables built from it
  float2* dps = reinterpret_cast<float2*>(reinterpret_cast<char*>(s_dyn) + max(16, stage_rows * EB) * cols);
  if constexpr (TABLE) {
    float dmax = 0.f;
    for (int cb = threadIdx.x; cb < cols; cb += kColBatch * kCorrThreads) {
      float dv[kColBatch], pv[kColBatch];
#pragma unroll
      for (int j = 0; j < kColBatch; ++j) {
        const int c = cb + j * kCorrThreads;
        dv[j] = 0.f;
        pv[j] = 0.f;
        if (c < cols) {
          const int pn = pulse_of(c);
          if (dphi) dv[j] = dphi[pn];
          if (dpsi) pv[j] = dpsi[pn];
        }
      }
      if (fused && cb == (int)threadIdx.x && (int)threadIdx.x < k) tap0 = tap_geom(o_first, w_first);
#pragma unroll
      for (int j = 0; j < kColBatch; ++j) {
        const int c = cb + j * kCorrThreads;
        if (c < cols) {
          dps[c] = make_float2(dv[j], pv[j]);
          dmax = fmaxf(dmax, fabsf(dv[j]));
        }
      }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, off));
    if (lane == 0) s_red[wave] = dmax;
    __syncthreads();
    dmax = s_red[0];
#pragma unroll
    for (int w = 1; w < kCorrThreads / kWave; ++w) dmax = fmaxf(dmax, s_red[w]);
    const double rho = rr - g.radius;
    double cmax = 0.0;   // bound on |beta (R^ - R_nom)| of the series path, in bins
    if (rho > 0.0 && dmax == dmax) {
      const double c = 2.0 * rr * g.radius;
      const double m4 = 2.0 * (c / (2.0 * rho) + 0.75 * c * c / (rho * rho * rho));
      const double d2 = (double)dmax * (double)dmax;
      const double rem = m4 * d2 * d2 / 24.0;   // metres
      series = rem * (kTwoPiD * g.k_over_pi) <= 1e-6 && rem * g.beta <= 0x1p-20 &&
               g.beta * g.radius * (double)dmax < 0.5 && g.k_over_pi * g.radius * (double)dmax < 64.0;
      cmax = g.beta * g.radius * (double)dmax + 0x1p-20;
      // the sum's error bound as in corr_bin, with |correction| <= cmax
      tie_err = (float)(0x1p-18 + cmax * 0x1p-12);
    }
    if (series && stage_rows > 0) {
      // rows the pairs can reach: floor(u +- cmax) over the in-window taps, with a margin for
      // the float32 evaluation of the sum
      cm = cmax * (1.0 + 0x1p-10) + 0x1p-16;
      int lo = INT_MAX, hi = INT_MIN;
      if (fused) {
        if ((int)threadIdx.x < k && tap0.inwin) {
          lo = (int)floor(tap0.u64 - cm);
          hi = (int)floor(tap0.u64 + cm);
        }
      } else {
        for (int t = threadIdx.x; t < k; t += kCorrThreads) {
          const int o = t == (int)threadIdx.x ? o_first : offsets[wrow + t];
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
      for (int w = 1; w < kCorrThreads / kWave; ++w) {
        lo = min(lo, s_redi[2 * w]);
        hi = max(hi, s_redi[2 * w + 1]);
      }
      if (hi < lo) lo = hi = 0;   // no tap inside the window
      lmin = lo;
      nrows = hi - lo + 1;
      staged = nrows <= stage_rows;
    }
    if (staged) {
      if (fused && wave == 0) file_staged(tap0, (int)threadIdx.x < k);
      // band rows lmin .. lmin + nrows - 1 (LINEAR: and the next) over the columns, turned by
      // exp(-j psi); the (beta d, (k / pi) d) table takes the place of (d, psi), column by
      // column
      float2* ek = dps;
      const int nload = nrows + (LIN ? 1 : 0);   // at most kStageLoads
      for (int cb = threadIdx.x; cb < cols; cb += kColBatch * kCorrThreads) {
        float2 v[kColBatch][kStageLoads];
#pragma unroll
        for (int j = 0; j < kColBatch; ++j) {
          const int c = cb + j * kCorrThreads;
          const uint32_t colb = c < cols ? (uint32_t)((pulse_of(c) + y.halo) * ES) : 0u;
#pragma unroll
          for (int r = 0; r < kStageLoads; ++r) {
            const int l = lmin + r;
            v[j][r] = make_float2(0.f, 0.f);
            if (c < cols && r < nload && l >= 0 && l < y.l_count)
              v[j][r] = buf_load<DT>(rsrc, (uint32_t)__mul24(l, ld_es) + colb, 0u);
          }
        }
#pragma unroll
        for (int j = 0; j < kColBatch; ++j) {
          const int c = cb + j * kCorrThreads;
          if (c >= cols) continue;
          const float2 dp = dps[c];
          float sp = 0.f, cp = 1.f;
          if (dpsi) {
            // exp(-j psi) on the hardware sine/cosine in revolutions, like the pairs' phase
            float pr = dp.y * kInv2Pi;
            pr -= rintf(pr);
            sp = sin_rev(pr);
            cp = cos_rev(pr);
          }
          ek[c] = make_float2(beta * dp.x, kpi * dp.x);
#pragma unroll
          for (int r = 0; r < kStageLoads; ++r)
            v[j][r] = make_float2(fmaf(v[j][r].x, cp, v[j][r].y * sp), fmaf(v[j][r].y, cp, -v[j][r].x * sp));
#pragma unroll
          for (int r = 0; r < kStageLoads - (LIN ? 1 : 0); ++r) {
            if (r >= nrows) break;
            if constexpr (LIN) {
              reinterpret_cast<float4*>(s_dyn)[r * cols + c] =
                  make_float4(v[j][r].x, v[j][r].y, v[j][r + 1].x - v[j][r].x, v[j][r + 1].y - v[j][r].y);
            } else {
              reinterpret_cast<float2*>(s_dyn)[r * cols + c] = v[j][r];
            }
          }
        }
      }
    } else {
      for (int c = threadIdx.x; c < cols; c += kCorrThreads) {
        const float2 dp = dps[c];
        const float d = dp.x;
        float pr = dp.y * kInv2Pi;
        pr -= rintf(pr);
        if (series) {
          s_dyn[c] = make_float4(pr, beta * d, kpi * d, 0.f);
        } else {
          float sh = 0.f, ch = 1.f;
          if (dphi) sincosf(0.5f * d, &sh, &ch);
          s_dyn[c] = make_float4(pr, d, sh, ch);
        }
      }
    }
  }

  const bool wave_live = a0 + i_wave < n;   // some pixel of this wave lies in the rotation
  int acol[kCorrP];        // pixel column, clamped into the rotation for padding lanes
  uint32_t acb[kCorrP];    // its byte offset in a band row
  float2 acc[kCorrP];
#pragma unroll
  for (int p = 0; p < kCorrP; ++p) {
    acol[p] = min(a0 + i_wave + lane + kWave * p, n - 1);
    acb[p] = (uint32_t)acol[p] * ES;
    acc[p] = make_float2(0.f, 0.f);
  }

  // tap table of taps [c0, c0 + cnt), one per thread of wave 0, from the offsets and weights
  // loaded ahead; then the next chunk's (of `chunk` taps) are requested, to arrive during this
  // chunk's pairs
  auto build_taps = [&](int c0, int cnt, int chunk, bool ser, bool stg) {
    if (stg) {
      if (wave == 0) {
        CorrTap e{};
        if ((int)threadIdx.x < cnt) e = tap_geom(o_next, w_next);
        file_staged(e, (int)threadIdx.x < cnt);
      }
    } else if ((int)threadIdx.x < cnt) {
      CorrTap e = tap_geom(o_next, w_next);
      if (ser) {
        // byte offset of (row u.i, column o + halo) in the band, the row clamped so that every
        // sampled row stays out of the band when the nominal one is
        e.u.i = min(max(e.u.i, -3), y.l_count + 2);
        e.ub = (int32_t)((uint32_t)e.u.i * (uint32_t)ld_es + (uint32_t)((e.o + y.halo) * ES));
      }
      s_tap[threadIdx.x] = e;
    }
    const int c1 = c0 + chunk;
    if ((int)threadIdx.x < min(chunk, k - c1)) {
      o_next = offsets[wrow + c1 + threadIdx.x];
      w_next = load_w<WDT>(weights, wrow + c1 + threadIdx.x);
    }
  };

  // exp term and accumulation shared by every path: acc += |w| exp(-j 2 pi rev) smp, where rev
  // already holds arg(w) / 2 pi
  auto accumulate = [&](float2& ac, float wa, float rev, float2 smp) {
    const float a = wa * cos_rev(rev), b = wa * sin_rev(rev);
    ac.x = fmaf(smp.x, a, fmaf(smp.y, b, ac.x));
    ac.y = fmaf(smp.y, a, fmaf(-smp.x, b, ac.y));
  };

  // NEAREST tie: the plain float64 bin at the angle (o 2 pi) / N + delta_n of the oracle's
  // definition, sampled from the band in global memory
  auto tie_sample = [&](int p, int o, int& pn) {
    pn = acol[p] + o;
    pn += (pn < 0) ? n : 0;
    pn -= (pn >= n) ? n : 0;
    const double d = (double)o * g.step + (dphi ? (double)dphi[pn] : 0.0);
    int l = (int)floor(plain_bin_half(rr, g.radius, d, g.beta)) - y.l_lo;
    l = min(max(l, -1), y.l_count);
    return buf_load<DT>(rsrc, (uint32_t)(__mul24(l, ld_es) + (pn + y.halo) * ES), 0u);
  };

  if (staged) {
    // series path over the staged rows
    const char* band = reinterpret_cast<const char*>(s_dyn);
    const float2* ek = dps;
    const int rowb = cols * EB;
    const int laneb = (i_wave + lane) * EB;
    auto pairs = [&](int cnt) {
      const int nfast = __builtin_amdgcn_readfirstlane(wave_live ? s_nfast : 0);
      // taps whose pairs all sample their nominal row: x = u.f + e s lies in [0, 1)
      for (int t = 0; t < nfast; ++t) {
        const CorrTapS tp = s_tapS[t];
        const char* bt = band + (tp.ub + laneb);
#pragma unroll
        for (int p = 0; p < kCorrP; ++p) {
          const float2 q = ek[i_wave + lane + kWave * p + tp.o + half_w];
          const float s = fmaf(q.x, fmaf(q.x, tp.q3, tp.q2), tp.q1);
          const char* at = bt + kWave * EB * p;
          float2 smp;
          if constexpr (INTERP == ROSAR_NEAREST) {
            smp = *reinterpret_cast<const float2*>(at);
          } else {
            const float x = fmaf(q.x, s, tp.uf);
            const float4 v = *reinterpret_cast<const float4*>(at);
            smp = make_float2(fmaf(x, v.z, v.x), fmaf(x, v.w, v.y));
          }
          accumulate(acc[p], tp.wa, fmaf(q.y, s, tp.wt), smp);
        }
      }
      for (int t = nfast; t < (wave_live ? cnt : 0); ++t) {
        const CorrTapS tp = s_tapS[t];
        const char* bt = band + (tp.ub + laneb);
        float2 smp[kCorrP];
        float rev[kCorrP];
        int ties = 0;   // NEAREST: bit p set when pixel p's bin sum lies near a rounding boundary
#pragma unroll
        for (int p = 0; p < kCorrP; ++p) {
          const float2 q = ek[i_wave + lane + kWave * p + tp.o + half_w];
          const float s = fmaf(q.x, fmaf(q.x, tp.q3, tp.q2), tp.q1);
          const float x = fmaf(q.x, s, tp.uf);
          rev[p] = fmaf(q.y, s, tp.wt);
          const float fr = __builtin_amdgcn_fractf(x);
          const char* at = bt + __mul24(floor_to_int(x), rowb) + kWave * EB * p;
          if constexpr (INTERP == ROSAR_NEAREST) {
            smp[p] = *reinterpret_cast<const float2*>(at);
            ties |= (fr < tie_err || fr > 1.f - tie_err) ? (1 << p) : 0;
          } else {
            const float4 v = *reinterpret_cast<const float4*>(at);
            smp[p] = make_float2(fmaf(fr, v.z, v.x), fmaf(fr, v.w, v.y));
          }
        }
        if constexpr (INTERP == ROSAR_NEAREST) {
          if (__builtin_expect(__builtin_amdgcn_ballot_w64(ties != 0) != 0, 0)) {
#pragma unroll
            for (int p = 0; p < kCorrP; ++p) {
              if (ties & (1 << p)) {
                // the tie's sample comes from global memory, not yet turned by exp(-j psi)
                int pn;
                smp[p] = tie_sample(p, tp.o, pn);
                float pr = dpsi ? dpsi[pn] * kInv2Pi : 0.f;
                rev[p] += pr - rintf(pr);
              }
            }
          }
        }
#pragma unroll
        for (int p = 0; p < kCorrP; ++p) accumulate(acc[p], tp.wa, rev[p], smp[p]);
      }
    };
    if (fused) {
      __syncthreads();
      pairs(k);
    } else {
      __syncthreads();
      for (int c0 = 0; c0 < k; c0 += kCorrChunkS) {
        const int cnt = min(kCorrChunkS, k - c0);
        build_taps(c0, cnt, kCorrChunkS, true, true);
        __syncthreads();
        pairs(cnt);
        __syncthreads();
      }
    }
  } else {
    // gathers from global memory, with the series (SERIES = true) or the exact correction;
    // DIRECT: the halo holds every column a + o (no wrap)
    auto taps = [&](auto series_tag, auto direct_tag) {
      constexpr bool SERIES = decltype(series_tag)::value;
      constexpr bool DIRECT = decltype(direct_tag)::value;
      for (int c0 = 0; c0 < k; c0 += kCorrChunk) {
        const int cnt = min(kCorrChunk, k - c0);
        build_taps(c0, cnt, kCorrChunk, SERIES, false);
        __syncthreads();
        for (int t = 0; t < (wave_live ? cnt : 0); ++t) {
          const CorrTap tp = s_tap[t];
#pragma unroll
          for (int p = 0; p < kCorrP; ++p) {
            float x, rev, err = tie_err;
            if constexpr (SERIES) {
              const float4 q = s_dyn[i_wave + lane + kWave * p + tp.o + half_w];
              const float s = fmaf(q.y, fmaf(q.y, tp.q3, tp.q2), tp.q1);
              x = fmaf(q.y, s, tp.u.f);
              rev = fmaf(q.z, s, q.x);
            } else {
              float sh = 0.f, ch = 1.f, pr;
              if constexpr (TABLE) {
                const float4 q = s_dyn[i_wave + lane + kWave * p + tp.o + half_w];
                pr = q.x;
                sh = q.z;
                ch = q.w;
              } else {
                int pn = acol[p] + tp.o;
                pn += (pn < 0) ? n : 0;
                pn -= (pn >= n) ? n : 0;
                if (dphi) sincosf(0.5f * dphi[pn], &sh, &ch);
                pr = dpsi ? dpsi[pn] * kInv2Pi : 0.f;
              }
              const float s_mid = fmaf(tp.sd, ch, tp.cd * sh);   // sin(D0 + d/2)
              const float dd = c4 * s_mid * sh;                    // R^2 - R_nom^2
              const float r2 = fmaxf(tp.r2 + dd, 1e-30f);
              const float rn = r2 * __builtin_amdgcn_rsqf(r2);
              const float diff = dd * __builtin_amdgcn_rcpf(rn + tp.rnom);   // R^ - R_nom
              const float corr = beta * diff;
              x = tp.u.f + corr;
              err = 0x1p-18f + fabsf(corr) * 0x1p-12f;
              rev = fmaf(kpi, diff, pr);
              rev -= floorf(rev);
            }
            const float fr = __builtin_amdgcn_fractf(x);
            const int li = floor_to_int(x);
            uint32_t off0;
            if constexpr (SERIES && DIRECT) {
              off0 = (uint32_t)__mul24(li, ld_es) + (acb[p] + (uint32_t)tp.ub);
            } else {
              int col = acol[p] + tp.o;
              if constexpr (!DIRECT) {
                col += (col < 0) ? n : 0;
                col -= (col >= n) ? n : 0;
              }
              int l = tp.u.i + li;
              if constexpr (!SERIES) l = min(max(l, INTERP == ROSAR_NEAREST ? -1 : -2), y.l_count);
              off0 = (uint32_t)(__mul24(l, ld_es) + (col + y.halo) * ES);
            }
            float2 smp;
            if constexpr (INTERP == ROSAR_NEAREST) {
              smp = buf_load<DT>(rsrc, off0, 0u);
              if (__builtin_expect(fr < err || fr > 1.f - err, 0)) {
                int pn;
                smp = tie_sample(p, tp.o, pn);
              }
            } else {
              const float2 y0 = buf_load<DT>(rsrc, off0, 0u);
              const float2 y1 = buf_load<DT>(rsrc, off0 + (uint32_t)ld_es, 0u);
              smp = make_float2(fmaf(fr, y1.x - y0.x, y0.x), fmaf(fr, y1.y - y0.y, y0.y));
            }
            accumulate(acc[p], tp.wa, rev + tp.wt, smp);
          }
        }
        __syncthreads();
      }
    };
    const bool direct = y.halo >= half_w;
    if (series) {
      if (direct)
        taps(std::true_type{}, std::true_type{});
      else
        taps(std::true_type{}, std::false_type{});
    } else {
      if (direct)
        taps(std::false_type{}, std::true_type{});
      else
        taps(std::false_type{}, std::false_type{});
    }
  }

  float2* out = image + (int64_t)row * n;
#pragma unroll
  for (int p = 0; p < kCorrP; ++p) {
    const int a = a0 + i_wave + lane + kWave * p;
    if (a < n) out[a] = make_float2(acc[p].x * y.inv_scale, acc[p].y * y.inv_scale);
  }
}

// PRE: the rows' tap tables come precomputed from `tabs` (sparse-filter plans).
template <int DT, int WDT, int INTERP, int P, int NW, bool PRE>
__global__ __launch_bounds__(kWave* NW) void sparse_lds_kernel(Geo g, View y, int32_t k, int32_t window,
                                                               int tiles_per_row, int nblocks, int rows_cap,
                                                               double cos_hw, int stride, int use_dma,
                                                               const int32_t* __restrict__ offsets,
                                                               const void* __restrict__ weights,
                                                               const char* __restrict__ ydata,
                                                               float2* __restrict__ image,
                                                               const char* __restrict__ tabs) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_unstaged;
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  sparse::lds_tile<DT, WDT, INTERP, P, NW, PRE>(g, y, k, window, row, blk - row * tiles_per_row, rows_cap, cos_hw,
                                                stride, use_dma, offsets, weights, ydata, image, smem, s_unstaged,
                                                tabs);
}

template <int DT, int WDT, int INTERP, int P, int NW>
hipError_t launch_lds_t(const SparseArgs& a, hipStream_t s, bool* fits) {
  constexpr int T = kWave * P * NW;
  const sparse::LdsLayout L = sparse::lds_layout_capped(a.g, a.y, a.k, a.window, INTERP, T);
  *fits = L.bytes <= sparse::kLdsBudget;
  if (!*fits) return hipSuccess;
  const int tiles = (a.g.n + T - 1) / T;
  const int nblocks = tiles * a.g.n_range;
  sparse_lds_kernel<DT, WDT, INTERP, P, NW, false><<<nblocks, kWave * NW, L.bytes, s>>>(
      a.g, a.y, a.k, a.window, tiles, nblocks, L.rows, L.cos_hw, L.stride, L.dma, a.offsets, a.weights,
      reinterpret_cast<const char*>(a.y.data), a.image, nullptr);
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
  const int tiles = (a.g.n + kCorrTile - 1) / kCorrTile;
  const int nblocks = tiles * a.g.n_range;
  const char* yd = reinterpret_cast<const char*>(a.y.data);
  const int cols = kCorrTile + a.window;
  if (cols <= kCorrMaxCols) {
    // dynamic LDS: the float4 column table or the staged band rows, then a float2 per column
    const bool lin = INTERP == ROSAR_LINEAR;
    const int stage = cols <= kCorrStageCols ? (lin ? kCorrStageRowsL : kCorrStageRowsN) : 0;
    const size_t lds = (size_t)std::max(16, stage * (lin ? 16 : 8)) * cols + (size_t)cols * sizeof(float2);
    sparse_corrected_kernel<DT, WDT, INTERP, true><<<nblocks, kCorrThreads, lds, s>>>(
        a.g, a.y, a.k, a.window, tiles, nblocks, stage, a.offsets, a.weights, a.dphi, a.dpsi, yd, a.image);
  } else {
    sparse_corrected_kernel<DT, WDT, INTERP, false><<<nblocks, kCorrThreads, 0, s>>>(
        a.g, a.y, a.k, a.window, tiles, nblocks, 0, a.offsets, a.weights, a.dphi, a.dpsi, yd, a.image);
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

// ---------------------------------------------------------------- sparse-filter plans
#define ROSAR_PLAN_SHAPES(X) X(4, 8) X(8, 4) X(4, 4) X(2, 8) X(2, 4) X(8, 2)

template <int DT, int WDT, int INTERP, int P, int NW>
hipError_t launch_planned_t(const SparseArgs& a, const PlanLayout& pl, const char* tabs, hipStream_t s) {
  constexpr int T = kWave * P * NW;
  const int tiles = (a.g.n + T - 1) / T;
  const int nblocks = tiles * a.g.n_range;
  sparse_lds_kernel<DT, WDT, INTERP, P, NW, true><<<nblocks, kWave * NW, pl.lds_bytes, s>>>(
      a.g, a.y, a.k, a.window, tiles, nblocks, pl.rows_cap, pl.cos_hw, pl.stride, 1, a.offsets, a.weights,
      reinterpret_cast<const char*>(a.y.data), a.image, tabs);
  return hipGetLastError();
}

template <int DT, int WDT, int INTERP>
hipError_t launch_planned_shape(const SparseArgs& a, const PlanLayout& pl, const char* tabs, hipStream_t s) {
#define ROSAR_PSHAPE(P, NW) \
  if (pl.ppl == P && pl.waves == NW) return launch_planned_t<DT, WDT, INTERP, P, NW>(a, pl, tabs, s);
  ROSAR_PLAN_SHAPES(ROSAR_PSHAPE)
#undef ROSAR_PSHAPE
  return hipErrorInvalidValue;
}

template <int DT>
hipError_t launch_planned_dt(const SparseArgs& a, const PlanLayout& pl, const char* tabs, hipStream_t s) {
  const bool lin = a.interp == ROSAR_LINEAR;
  if (a.w_dtype == ROSAR_C64)
    return lin ? launch_planned_shape<DT, 0, ROSAR_LINEAR>(a, pl, tabs, s)
               : launch_planned_shape<DT, 0, ROSAR_NEAREST>(a, pl, tabs, s);
  return lin ? launch_planned_shape<DT, 1, ROSAR_LINEAR>(a, pl, tabs, s)
             : launch_planned_shape<DT, 1, ROSAR_NEAREST>(a, pl, tabs, s);
}

template <int DT, int WDT, int INTERP>
hipError_t launch_tables_t(const SparseArgs& a, const PlanLayout& pl, char* tabs, hipStream_t s) {
  sparse::tap_table_kernel<DT, WDT, INTERP><<<a.g.n_range, 256, 0, s>>>(
      a.g, a.y, a.k, a.window, pl.rows_cap, pl.cos_hw, pl.stride, pl.shift, a.offsets, a.weights, tabs);
  return hipGetLastError();
}

template <int DT>
hipError_t launch_tables_dt(const SparseArgs& a, const PlanLayout& pl, char* tabs, hipStream_t s) {
  const bool lin = a.interp == ROSAR_LINEAR;
  if (a.w_dtype == ROSAR_C64)
    return lin ? launch_tables_t<DT, 0, ROSAR_LINEAR>(a, pl, tabs, s) : launch_tables_t<DT, 0, ROSAR_NEAREST>(a, pl, tabs, s);
  return lin ? launch_tables_t<DT, 1, ROSAR_LINEAR>(a, pl, tabs, s) : launch_tables_t<DT, 1, ROSAR_NEAREST>(a, pl, tabs, s);
}

}  // namespace

bool plan_shape_supported(int ppl, int waves) {
#define ROSAR_PCHECK(P, NW) if (ppl == P && waves == NW) return true;
  ROSAR_PLAN_SHAPES(ROSAR_PCHECK)
#undef ROSAR_PCHECK
  return false;
}

bool sparse_plan_layout(const SparseArgs& a, int ppl, int waves, PlanLayout* out) {
  const int T = kWave * ppl * waves;
  const sparse::LdsLayout L = sparse::lds_layout_capped(a.g, a.y, a.k, a.window, a.interp, T);
  if (!L.dma || L.bytes > sparse::kLdsBudget) return false;
  const int es = a.y.dtype == ROSAR_C64 ? 8 : 4;
  const int cpl = 16 / es;
  const int half_w = a.window / 2;
  const int nsub = a.interp == ROSAR_LINEAR ? 2 : 1;
  out->ppl = ppl;
  out->waves = waves;
  out->rows_cap = L.rows;
  out->stride = L.stride;
  out->cos_hw = L.cos_hw;
  out->shift = ((a.y.halo - half_w) & (cpl - 1)) + half_w;   // tiles start at multiples of cpl
  out->lds_bytes = L.bytes + 16;
  out->row_bytes = sparse::row_table_bytes(a.k * nsub);
  return true;
}

hipError_t launch_tap_tables(const SparseArgs& a, const PlanLayout& pl, char* tabs, hipStream_t s) {
  switch (a.y.dtype) {
    case ROSAR_C64: return launch_tables_dt<0>(a, pl, tabs, s);
    case ROSAR_C16_F16: return launch_tables_dt<1>(a, pl, tabs, s);
    default: return launch_tables_dt<2>(a, pl, tabs, s);
  }
}

hipError_t launch_sparse_planned(const SparseArgs& a, const PlanLayout& pl, const char* tabs, hipStream_t s) {
  switch (a.y.dtype) {
    case ROSAR_C64: return launch_planned_dt<0>(a, pl, tabs, s);
    case ROSAR_C16_F16: return launch_planned_dt<1>(a, pl, tabs, s);
    default: return launch_planned_dt<2>(a, pl, tabs, s);
  }
}

Tile default_tile(int32_t n, int32_t y_dtype) {
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
