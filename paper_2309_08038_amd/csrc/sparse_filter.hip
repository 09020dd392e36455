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
#include <climits>

#include "rosar_device.hpp"

namespace rosar {
namespace {

// Raw buffer resource over `bytes` bytes (gfx9 family word 3).  Loads address
// base + voffset + soffset; every offset the kernels form stays inside the buffer.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <int DT>
__device__ __forceinline__ float2 buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (DT == 0) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    return DT == 1 ? unpack_f16x2(v) : unpack_bf16x2(v);
  }
}

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

// ---------------------------------------------------------------------------------------
// LDS-staged plain path.  A workgroup owns T = 64*P*NW consecutive pixels of one row.  Its
// threads first build the row's tap table in LDS (tap t by thread t, float64 bins) and reduce
// the span of bin rows and offsets the taps touch; the workgroup then copies those rows over
// the columns [a0 + o_min, a0 + T + o_max) into LDS once (pulse index wrapped modulo N while
// copying), and every tap becomes one broadcast read of its table entry, one address add and
// P conflict-free LDS reads.  Entries whose bin row did not fit the staged rows (the host
// sizes the staging from an upper bound, so this is only a guard) are applied afterwards from
// global memory.  FP16/BF16 samples use v_dot2_f32_{f16,bf16}: two instructions per complex
// multiply-accumulate with float32 accumulation.
struct alignas(16) TapEntry {
  int lds_off;     // byte offset of the sample column in the staged rows (0 when not staged)
  int glob_row;    // element offset of the bin row in Y_T for a sampled entry whose row was
                   // not staged; -1 otherwise
  uint32_t w1, w2; // DT 0: re/im of the weight as float bits; DT 1/2: packed pairs (zero when
                   // not staged: such entries are applied from global memory by the guard loop)
};

template <int DT>
__device__ __forceinline__ void pack_weight(float2 w, uint32_t& w1, uint32_t& w2) {
  if constexpr (DT == 0) {
    w1 = __float_as_uint(w.x);
    w2 = __float_as_uint(w.y);
  } else if constexpr (DT == 1) {
    __half2 a = __floats2half2_rn(w.x, w.y);    // (wr, wi):  yr wr + yi wi = Re(conj(w) y)
    __half2 b = __floats2half2_rn(-w.y, w.x);   // (-wi, wr): yi wr - yr wi = Im(conj(w) y)
    w1 = __builtin_bit_cast(uint32_t, a);
    w2 = __builtin_bit_cast(uint32_t, b);
  } else {
    w1 = (uint32_t)f32_to_bf16_rne(w.x) | ((uint32_t)f32_to_bf16_rne(w.y) << 16);
    w2 = (uint32_t)f32_to_bf16_rne(-w.y) | ((uint32_t)f32_to_bf16_rne(w.x) << 16);
  }
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef short bf16x2v __attribute__((ext_vector_type(2)));

// acc += conj(w) * y with the weight in packed form and the sample as stored (raw bits)
template <int DT>
__device__ __forceinline__ void mac_packed(float2& acc, uint32_t w1, uint32_t w2, uint32_t ylo, uint32_t yhi) {
  if constexpr (DT == 0) {
    const float wr = __uint_as_float(w1), wi = __uint_as_float(w2);
    const float yr = __uint_as_float(ylo), yi = __uint_as_float(yhi);
    acc.x = fmaf(wr, yr, acc.x);
    acc.x = fmaf(wi, yi, acc.x);
    acc.y = fmaf(wr, yi, acc.y);
    acc.y = fmaf(-wi, yr, acc.y);
  } else if constexpr (DT == 1) {
    const half2v y = __builtin_bit_cast(half2v, ylo);
    acc.x = __builtin_amdgcn_fdot2(y, __builtin_bit_cast(half2v, w1), acc.x, false);
    acc.y = __builtin_amdgcn_fdot2(y, __builtin_bit_cast(half2v, w2), acc.y, false);
  } else {
    const bf16x2v y = __builtin_bit_cast(bf16x2v, ylo);
    acc.x = __builtin_amdgcn_fdot2_f32_bf16(y, __builtin_bit_cast(bf16x2v, w1), acc.x, false);
    acc.y = __builtin_amdgcn_fdot2_f32_bf16(y, __builtin_bit_cast(bf16x2v, w2), acc.y, false);
  }
}

template <int DT>
__device__ __forceinline__ void lds_sample(const char* smem, uint32_t byte_off, uint32_t& lo, uint32_t& hi) {
  if constexpr (DT == 0) {
    const uint2 v = *reinterpret_cast<const uint2*>(smem + byte_off);
    lo = v.x;
    hi = v.y;
  } else {
    lo = *reinterpret_cast<const uint32_t*>(smem + byte_off);
    hi = 0;
  }
}

// Staged-entry loop for the first PA of the P pixel chunks of a lane (PA < P on a row's last,
// partial wave).  Groups of U entries: table reads and samples first, then the FMAs.
template <int DT, int P, int PA>
__device__ __forceinline__ void staged_taps(float2 (&acc)[P], const TapEntry* table, const char* stage,
                                            uint32_t lane_base, int ne) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int U = 4;
  int e = 0;
  for (; e + U <= ne; e += U) {
    TapEntry te[U];
    uint32_t ylo[U][PA], yhi[U][PA];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      te[u] = table[e + u];
      const uint32_t base = lane_base + (uint32_t)te[u].lds_off;
#pragma unroll
      for (int p = 0; p < PA; ++p) lds_sample<DT>(stage, base + p * kWave * ES, ylo[u][p], yhi[u][p]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int p = 0; p < PA; ++p) mac_packed<DT>(acc[p], te[u].w1, te[u].w2, ylo[u][p], yhi[u][p]);
  }
  for (; e < ne; ++e) {
    const TapEntry te = table[e];
    const uint32_t base = lane_base + (uint32_t)te.lds_off;
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      uint32_t lo, hi;
      lds_sample<DT>(stage, base + p * kWave * ES, lo, hi);
      mac_packed<DT>(acc[p], te.w1, te.w2, lo, hi);
    }
  }
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

// Bin of a slant range: NEAREST rounds (eq. 40), LINEAR takes the lower neighbour.
template <int INTERP>
__device__ __forceinline__ int bin_of(double u) {
  return INTERP == ROSAR_NEAREST ? (int)floor(u + 0.5) : (int)floor(u);
}

template <int DT, int WDT, int INTERP, int P, int NW>
__global__ __launch_bounds__(kWave* NW) void sparse_lds_kernel(
    Geo g, View y, int32_t k, int32_t window, int tiles_per_row, int nblocks, int rows_cap, int stride,
    int use_dma, const int32_t* __restrict__ offsets, const void* __restrict__ weights,
    const char* __restrict__ ydata, float2* __restrict__ image) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  constexpr int NT = kWave * NW;
  constexpr int T = kWave * P * NW;
  constexpr int CPL = 16 / ES;            // columns per lane of one 16-byte direct-to-LDS load
  constexpr int CHUNK = kWave * CPL;      // columns per wave-wide direct-to-LDS load
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_unstaged;
  const int ne = k * NSUB;
  TapEntry* table = reinterpret_cast<TapEntry*>(smem);
  uint2* side = reinterpret_cast<uint2*>(smem + ne * (int)sizeof(TapEntry));
  char* stage = smem + ((ne * ((int)sizeof(TapEntry) + 8) + 15) & ~15);

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int a0 = tile * T;
  const int half_w = window / 2;
  const int64_t wrow = (int64_t)row * k;
  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;

  // ---- staged window: bin rows [lfirst, lfirst + nrows) from the geometry alone (the nearest
  // slant range of any tap is |R - r|, at offset 0), columns of pulses [a0 - W/2, a0 + T + W/2)
  const int lfirst = max(bin_of<INTERP>(g.beta * fabs(rr - g.radius)) - y.l_lo, 0);
  const int nrows = max(min(rows_cap, y.l_count - lfirst), 0);
  int col0;   // stored column of staged column 0
  if (use_dma) {
    // direct-to-LDS 16-byte loads from an even stored column (the halo covers the window)
    col0 = (a0 - half_w + y.halo) & ~(CPL - 1);
    const int nchunk = stride / CHUNK;
    const int64_t last = (int64_t)y.l_count * y.ld - CPL;   // clamp: columns past the stored
    for (int j = wave; j < nrows * nchunk; j += NW) {        // rotation feed padded pixels only
      const int r = j / nchunk;
      const int ch = j - r * nchunk;
      int64_t el = (int64_t)(lfirst + r) * y.ld + col0 + ch * CHUNK + lane * CPL;
      el = min(el, last);
      __builtin_amdgcn_global_load_lds((gbl_void_t*)(ydata + el * ES),
                                       (lds_void_t*)(stage + (r * stride + ch * CHUNK) * ES), 16, 0, 0);
    }
  } else {
    // element-wise copy with the pulse index wrapped modulo N
    col0 = a0 - half_w + y.halo;
    using TE = typename Elem<DT>::T;
    constexpr int SU = 8;
    const int cols = T + window;
    const int total = nrows * cols;
    for (int i0 = threadIdx.x; i0 < total; i0 += NT * SU) {
      TE v[SU];
      int dst[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = i0 + u * NT;
        dst[u] = -1;
        if (i < total) {
          const int r = i / cols;
          const int c = i - r * cols;
          int pn = a0 - half_w + c;
          pn %= n;
          pn += pn < 0 ? n : 0;
          v[u] = *reinterpret_cast<const TE*>(ydata + ((int64_t)(lfirst + r) * y.ld + pn + y.halo) * ES);
          dst[u] = (r * stride + c) * ES;
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (dst[u] >= 0) *reinterpret_cast<TE*>(stage + dst[u]) = v[u];
    }
  }
  // LDS column of pixel a0 + i at offset o: i + o + shift
  const int shift = (a0 - half_w + y.halo) - col0 + half_w;

  // ---- tap table (tap t by thread t): float64 bins (eq. 2 / eq. 40), packed weights
  if (threadIdx.x == 0) s_unstaged = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += NT) {
    const int o = offsets[wrow + t];
    const float2 w = load_w<WDT>(weights, wrow + t);
    const bool inwin = o >= -half_w && o < half_w;
    int l = 0;
    float f = 0.f;
    if (inwin) {
      const double u = g.beta * sqrt(c1 - c2 * cos(o * g.step));
      l = bin_of<INTERP>(u) - y.l_lo;
      if constexpr (INTERP == ROSAR_LINEAR) f = (float)(u - floor(u));
    }
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      const int ls = l + s;
      const bool ok = inwin && ls >= 0 && ls < y.l_count;
      const bool staged = ok && ls >= lfirst && ls < lfirst + nrows;
      const float fs = INTERP == ROSAR_NEAREST ? 1.f : (s == 0 ? 1.f - f : f);
      uint32_t w1, w2;
      pack_weight<DT>(ok ? make_float2(w.x * fs, w.y * fs) : make_float2(0.f, 0.f), w1, w2);
      TapEntry e;
      e.lds_off = staged ? ((ls - lfirst) * stride + o + shift) * ES : 0;
      e.glob_row = (ok && !staged) ? (int)(ls * y.ld) : -1;
      e.w1 = staged ? w1 : 0u;
      e.w2 = staged ? w2 : 0u;
      table[t * NSUB + s] = e;
      side[t * NSUB + s] = make_uint2(w1, w2);
      if (ok && !staged) s_unstaged = 1;
    }
  }
  if (use_dma) __builtin_amdgcn_s_waitcnt(0);  // direct-to-LDS loads complete
  __syncthreads();

  const int a_wave = a0 + wave * kWave * P;
  if (a_wave >= n) return;  // no barriers below
  const uint32_t lane_base = (uint32_t)((wave * kWave * P + lane) * ES);
  float2 acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = make_float2(0.f, 0.f);

  // pixel chunks of 64 this wave really has (the last wave of a row may be partial)
  const int pa = min(P, (n - a_wave + kWave - 1) / kWave);
  const int ne_staged = nrows > 0 ? ne : 0;
  if (pa == P) {
    staged_taps<DT, P, P>(acc, table, stage, lane_base, ne_staged);
  } else {
    switch (pa) {
      case 1: staged_taps<DT, P, 1>(acc, table, stage, lane_base, ne_staged); break;
      case 2: if constexpr (P > 2) staged_taps<DT, P, 2>(acc, table, stage, lane_base, ne_staged); break;
      case 3: if constexpr (P > 3) staged_taps<DT, P, 3>(acc, table, stage, lane_base, ne_staged); break;
      case 4: if constexpr (P > 4) staged_taps<DT, P, 4>(acc, table, stage, lane_base, ne_staged); break;
      case 5: if constexpr (P > 5) staged_taps<DT, P, 5>(acc, table, stage, lane_base, ne_staged); break;
      case 6: if constexpr (P > 6) staged_taps<DT, P, 6>(acc, table, stage, lane_base, ne_staged); break;
      default: if constexpr (P > 7) staged_taps<DT, P, 7>(acc, table, stage, lane_base, ne_staged); break;
    }
  }
  if (s_unstaged) {
    // guard: sampled entries outside the staged rows, straight from global memory
    for (int e2 = 0; e2 < ne; ++e2) {
      const TapEntry te = table[e2];
      if (__builtin_amdgcn_readfirstlane(te.glob_row) < 0) continue;
      const int o = offsets[wrow + e2 / NSUB];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        int a = min(a_wave + lane + kWave * p, n - 1) + o;
        a += (a < 0) ? n : 0;
        a -= (a >= n) ? n : 0;
        using TE = typename Elem<DT>::T;
        const TE v = *reinterpret_cast<const TE*>(ydata + ((int64_t)te.glob_row + a + y.halo) * ES);
        uint32_t lo, hi;
        if constexpr (DT == 0) {
          lo = __float_as_uint(v.x);
          hi = __float_as_uint(v.y);
        } else {
          lo = v;
          hi = 0;
        }
        mac_packed<DT>(acc[p], side[e2].x, side[e2].y, lo, hi);
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

// ---------------------------------------------------------------------------------------
// LDS-staged plain path with pixel pairs.  Same staging as sparse_lds_kernel, plus a second copy
// of the staged rows shifted by one column, so that every tap can read the two adjacent pixels
// of a lane with one aligned LDS access (ds_read_b128 for complex float32, ds_read_b64 for the
// 16-bit types): a tap whose column offset from the tile start is odd reads the shifted copy.
// Lane l of wave w owns pixel pairs a0 + 64*P*w + 128*q + 2*l + {0, 1}, q < P/2.  The last wave
// of a row runs only the pairs that exist (no padded tile work).
template <int DT>
struct Pair;
template <> struct Pair<0> { using T = uint4; };
template <> struct Pair<1> { using T = uint2; };
template <> struct Pair<2> { using T = uint2; };

template <int DT>
__device__ __forceinline__ void mac_pair(float2& a0, float2& a1, uint32_t w1, uint32_t w2,
                                         typename Pair<DT>::T v) {
  if constexpr (DT == 0) {
    mac_packed<0>(a0, w1, w2, v.x, v.y);
    mac_packed<0>(a1, w1, w2, v.z, v.w);
  } else {
    mac_packed<DT>(a0, w1, w2, v.x, 0u);
    mac_packed<DT>(a1, w1, w2, v.y, 0u);
  }
}

// Tap loop over the staged entries for QA pixel pairs per lane.
template <int DT, int QA>
__device__ __forceinline__ void pair_taps(float2 (&acc)[16], const TapEntry* table, const char* stage,
                                          uint32_t lane_base, int ne) {
  constexpr int PB = 2 * Elem<DT>::bytes;   // bytes of a pixel pair
  using PT = typename Pair<DT>::T;
  constexpr int U = QA >= 4 ? 2 : 4;
  int e = 0;
  for (; e + U <= ne; e += U) {
    TapEntry te[U];
    PT v[U][QA];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      te[u] = table[e + u];
      const char* b = stage + lane_base + te[u].lds_off;
#pragma unroll
      for (int q = 0; q < QA; ++q) v[u][q] = *reinterpret_cast<const PT*>(b + q * kWave * PB);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < QA; ++q) mac_pair<DT>(acc[2 * q], acc[2 * q + 1], te[u].w1, te[u].w2, v[u][q]);
  }
  for (; e < ne; ++e) {
    const TapEntry te = table[e];
    const char* b = stage + lane_base + te.lds_off;
#pragma unroll
    for (int q = 0; q < QA; ++q)
      mac_pair<DT>(acc[2 * q], acc[2 * q + 1], te.w1, te.w2, *reinterpret_cast<const PT*>(b + q * kWave * PB));
  }
}

template <int DT, int WDT, int INTERP, int Q, int NW>
__global__ __launch_bounds__(kWave* NW) void sparse_pair_kernel(
    Geo g, View y, int32_t k, int32_t window, int tiles_per_row, int nblocks, int rows_cap, int stride,
    const int32_t* __restrict__ offsets, const void* __restrict__ weights,
    const char* __restrict__ ydata, float2* __restrict__ image) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  constexpr int NT = kWave * NW;
  constexpr int P = 2 * Q;
  constexpr int T = kWave * P * NW;
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_span[5];  // lmin, lmax, omin, omax, any entry unstaged
  const int ne = k * NSUB;
  TapEntry* table = reinterpret_cast<TapEntry*>(smem);
  uint2* side = reinterpret_cast<uint2*>(smem + ne * (int)sizeof(TapEntry));
  char* stage = smem + ((ne * ((int)sizeof(TapEntry) + 8) + 15) & ~15);
  // copy 0 at `stage`, copy 1 (shifted one column) right after: rows_cap * stride elements each
  const int copy_bytes = rows_cap * stride * ES;

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int blk = xcd_logical_block(blockIdx.x, nblocks);
  const int row = blk / tiles_per_row;
  const int tile = blk - row * tiles_per_row;
  const int n = g.n;
  const int a0 = tile * T;
  const int half_w = window / 2;
  const int64_t wrow = (int64_t)row * k;
  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;

  if (threadIdx.x == 0) {
    s_span[0] = INT_MAX;
    s_span[1] = INT_MIN;
    s_span[2] = INT_MAX;
    s_span[3] = INT_MIN;
    s_span[4] = 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k; t += NT) {
    const int o = offsets[wrow + t];
    const float2 w = load_w<WDT>(weights, wrow + t);
    int l = -1;
    float f = 0.f;
    const bool inwin = o >= -half_w && o < half_w;
    if (inwin) {
      const double u = g.beta * sqrt(c1 - c2 * cos(o * g.step));
      if constexpr (INTERP == ROSAR_NEAREST) {
        l = (int)floor(u + 0.5) - y.l_lo;
      } else {
        const double fl = floor(u);
        f = (float)(u - fl);
        l = (int)fl - y.l_lo;
      }
    }
    bool any = false;
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      const int ls = l + s;
      const bool ok = inwin && ls >= 0 && ls < y.l_count;
      const float fs = INTERP == ROSAR_NEAREST ? 1.f : (s == 0 ? 1.f - f : f);
      TapEntry e;
      e.lds_off = ok ? ls : -1;
      e.glob_row = ok ? (int)(ls * y.ld) : -1;
      pack_weight<DT>(ok ? make_float2(w.x * fs, w.y * fs) : make_float2(0.f, 0.f), e.w1, e.w2);
      table[t * NSUB + s] = e;
      if (ok) {
        atomicMin(&s_span[0], ls);
        atomicMax(&s_span[1], ls);
        any = true;
      }
    }
    if (any) {
      atomicMin(&s_span[2], o);
      atomicMax(&s_span[3], o);
    }
  }
  __syncthreads();
  const int lmin = s_span[0];
  const int nrows = s_span[1] >= lmin ? min(s_span[1] - lmin + 1, rows_cap) : 0;
  const int omin = s_span[2];
  const int span = s_span[3] >= omin ? s_span[3] - omin : 0;
  for (int e = threadIdx.x; e < ne; e += NT) {
    TapEntry& te = table[e];
    const int l = te.lds_off;
    const int c = offsets[wrow + e / NSUB] - omin;
    const bool staged = l >= 0 && l - lmin < nrows;
    side[e] = make_uint2(te.w1, te.w2);
    // even column: copy 0 at c; odd column: copy 1 (shifted by one) at c - 1
    te.lds_off = staged ? ((c & 1) * copy_bytes + ((l - lmin) * stride + (c & ~1)) * ES) : 0;
    if (!staged) {
      te.w1 = 0u;
      te.w2 = 0u;
      if (l >= 0) s_span[4] = 1;
    }
    if (staged || l < 0) te.glob_row = -1;
  }
  // stage copy 0 (columns [a0 + omin, a0 + omin + T + span + 1)) and copy 1 = copy 0 shifted by one
  const int cols = T + span + 2;
  {
    using TE = typename Elem<DT>::T;
    constexpr int SU = 8;
    const int total = nrows * cols;
    for (int i0 = threadIdx.x; i0 < total; i0 += NT * SU) {
      TE v[SU];
      int r_[SU], c_[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = i0 + u * NT;
        r_[u] = -1;
        if (i < total) {
          const int r = i / cols;
          const int c = i - r * cols;
          int pn = a0 + omin + c;
          pn += pn < 0 ? n : 0;
          pn -= pn >= n ? n : 0;
          if (pn >= n) pn %= n;
          v[u] = *reinterpret_cast<const TE*>(ydata + ((int64_t)(lmin + r) * y.ld + pn + y.halo) * ES);
          r_[u] = r;
          c_[u] = c;
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        if (r_[u] >= 0) {
          const int base = r_[u] * stride;
          *reinterpret_cast<TE*>(stage + (base + c_[u]) * ES) = v[u];
          if (c_[u] >= 1) *reinterpret_cast<TE*>(stage + copy_bytes + (base + c_[u] - 1) * ES) = v[u];
        }
      }
    }
  }
  __syncthreads();

  const int a_wave = a0 + wave * kWave * P;
  if (a_wave >= n) return;  // no barriers below
  float2 acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = make_float2(0.f, 0.f);
  const uint32_t lane_base = (uint32_t)((wave * kWave * P + 2 * lane) * ES);
  const int ne_staged = nrows > 0 ? ne : 0;
  // pairs this wave really has (the last wave of a row may be partial)
  const int qa = min(Q, (n - a_wave + 2 * kWave - 1) / (2 * kWave));
  switch (qa) {
    case 1: pair_taps<DT, 1>(acc, table, stage, lane_base, ne_staged); break;
    case 2: if constexpr (Q >= 2) pair_taps<DT, 2>(acc, table, stage, lane_base, ne_staged); break;
    case 3: if constexpr (Q >= 3) pair_taps<DT, 3>(acc, table, stage, lane_base, ne_staged); break;
    default: if constexpr (Q >= 4) pair_taps<DT, Q>(acc, table, stage, lane_base, ne_staged); break;
  }
  if (s_span[4]) {
    // guard: sampled entries whose row was not staged, straight from global memory
    for (int e2 = 0; e2 < ne; ++e2) {
      const TapEntry te = table[e2];
      if (__builtin_amdgcn_readfirstlane(te.glob_row) < 0) continue;
      const int o = offsets[wrow + e2 / NSUB];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        int a = min(a_wave + 128 * (p / 2) + 2 * lane + (p & 1), n - 1) + o;
        a += (a < 0) ? n : 0;
        a -= (a >= n) ? n : 0;
        using TE = typename Elem<DT>::T;
        const TE v = *reinterpret_cast<const TE*>(ydata + ((int64_t)te.glob_row + a + y.halo) * ES);
        uint32_t lo, hi;
        if constexpr (DT == 0) {
          lo = __float_as_uint(v.x);
          hi = __float_as_uint(v.y);
        } else {
          lo = v;
          hi = 0;
        }
        mac_packed<DT>(acc[p], side[e2].x, side[e2].y, lo, hi);
      }
    }
  }
  float2* out = image + (int64_t)row * n;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int a = a_wave + 128 * (p / 2) + 2 * lane + (p & 1);
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

constexpr size_t kLdsBudget = 96 * 1024;

// Upper bound on the FFT rows the taps of one range row touch: the slant range of a tap grows
// with |offset| over the window (|D| <= pi), so the rows lie between those of offsets 0 and W/2.
int staged_rows_bound(const SparseArgs& a) {
  const double r = a.g.radius;
  const double cw = cos((a.window / 2) * a.g.step);
  int best = 1;
  for (int i = 0; i < a.g.n_range; ++i) {
    const double rr = a.g.r0 + i * a.g.dr;
    const double umin = a.g.beta * fabs(rr - r);
    const double umax = a.g.beta * sqrt(rr * rr + r * r - 2.0 * rr * r * cw);
    int cnt = a.interp == ROSAR_NEAREST ? (int)(floor(umax + 0.5) - floor(umin + 0.5)) + 1
                                        : (int)(floor(umax) - floor(umin)) + 2;
    best = max(best, cnt);
  }
  return min(best, a.y.l_count);
}

template <int DT, int WDT, int INTERP, int P, int NW>
hipError_t launch_lds_t(const SparseArgs& a, hipStream_t s, bool* fits) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int T = kWave * P * NW;
  constexpr int CHUNK = kWave * (16 / ES);
  const int nsub = INTERP == ROSAR_LINEAR ? 2 : 1;
  const int rows = staged_rows_bound(a);
  // direct-to-LDS staging needs the halo to cover the window and 16-byte aligned rows
  const bool dma = a.y.halo >= a.window / 2 && ((a.y.ld * ES) % 16) == 0 &&
                   (reinterpret_cast<uintptr_t>(a.y.data) % 16) == 0;
  const int cols = T + a.window + (16 / ES);
  const int stride = dma ? (cols + CHUNK - 1) / CHUNK * CHUNK : cols;
  const size_t table = ((size_t)a.k * nsub * (sizeof(TapEntry) + 8) + 15) & ~(size_t)15;
  const size_t bytes = table + (size_t)rows * stride * ES;
  *fits = bytes <= kLdsBudget;
  if (!*fits) return hipSuccess;
  const int tiles = (a.g.n + T - 1) / T;
  const int nblocks = tiles * a.g.n_range;
  sparse_lds_kernel<DT, WDT, INTERP, P, NW><<<nblocks, kWave * NW, bytes, s>>>(
      a.g, a.y, a.k, a.window, tiles, nblocks, rows, stride, dma ? 1 : 0, a.offsets, a.weights,
      reinterpret_cast<const char*>(a.y.data), a.image);
  return hipGetLastError();
}

template <int DT, int WDT, int INTERP, int Q, int NW>
hipError_t launch_pair_t(const SparseArgs& a, hipStream_t s, bool* fits) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int T = kWave * 2 * Q * NW;
  const int nsub = INTERP == ROSAR_LINEAR ? 2 : 1;
  const int rows = staged_rows_bound(a);
  const int stride = (T + a.window + 2 + 1) & ~1;   // even: pair reads stay 2-element aligned
  const size_t table = ((size_t)a.k * nsub * (sizeof(TapEntry) + 8) + 15) & ~(size_t)15;
  const size_t bytes = table + 2 * (size_t)rows * stride * ES;
  *fits = bytes <= kLdsBudget;
  if (!*fits) return hipSuccess;
  const int tiles = (a.g.n + T - 1) / T;
  const int nblocks = tiles * a.g.n_range;
  sparse_pair_kernel<DT, WDT, INTERP, Q, NW><<<nblocks, kWave * NW, bytes, s>>>(
      a.g, a.y, a.k, a.window, tiles, nblocks, rows, stride, a.offsets, a.weights,
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
    if (t.variant == 3 && P >= 2) {                                            \
      bool fits = false;                                                       \
      hipError_t e = launch_pair_t<DT, WDT, INTERP, (P >= 2 ? P / 2 : 1), NW>(a, s, &fits); \
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
  (void)y_dtype;
  // LDS-staged window, eight pixels per lane, four waves: 2048-pixel tiles (short rotations:
  // one pixel per lane)
  Tile t{2, 8, 4};
  if (n <= 1024) t = Tile{2, 1, 4};
  return t;
}

bool tile_supported(const Tile& t) {
  if (t.variant < 0 || t.variant > 3) return false;
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
