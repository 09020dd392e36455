// LDS-staged sparse-aperture filter tile (Algorithm 2 with eq. 43), shared by the
// single-rotation kernel and the persistent batched kernel.
//
// A workgroup owns T = 64*P*NW consecutive pixels of one range row.  The window it reads (the
// bin rows its taps touch, over pulses [a0 - W/2, a0 + T + W/2)) follows from the geometry
// alone -- the nearest slant range of any tap is |R - r| at offset 0 and the host bounds the
// row span -- so it is copied into LDS with direct-to-LDS 16-byte loads issued at entry, while
// the threads build the row's tap table (tap t by thread t: float64 bin of eq. 2 / eq. 40,
// weight packed for the storage type).  Each tap is then one broadcast table read, one address
// add and P conflict-free LDS reads per lane; FP16/BF16 samples use v_dot2_f32_{f16,bf16}
// (two instructions per complex multiply-accumulate, float32 accumulation).  Taps whose bin row
// is not staged (only if the bound was capped) are applied from global memory afterwards.
#pragma once

#include <climits>

#include "rosar_device.hpp"

namespace rosar {
namespace sparse {

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

typedef unsigned u32x2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const volatile u32x2v lds_u32x2;
typedef __attribute__((address_space(3))) const volatile u32x4v lds_u32x4;
typedef __attribute__((address_space(3))) const volatile uint32_t lds_u32;
typedef __attribute__((address_space(3))) const char lds_char;

// One sample of a lane from the staged rows.  The reads are volatile so that the compiler keeps
// each one a single ds_read_b64 / ds_read_b32: fused into ds_read2st64 pairs (the P reads of a
// tap are 64 samples apart) the loop measured about 25 % slower on gfx950.
template <int DT>
__device__ __forceinline__ void lds_sample(const char* smem, uint32_t byte_off, uint32_t& lo, uint32_t& hi) {
  if constexpr (DT == 0) {
    const u32x2v v = *(lds_u32x2*)((lds_char*)smem + byte_off);
    lo = v.x;
    hi = v.y;
  } else {
    lo = *(lds_u32*)((lds_char*)smem + byte_off);
    hi = 0;
  }
}

// One tap-table entry as a single 16-byte broadcast LDS read (the compiler would otherwise
// split it into the fields the loop uses, two instructions).
__device__ __forceinline__ TapEntry lds_entry(const TapEntry* table, int e) {
  const u32x4v v = *(lds_u32x4*)((lds_char*)reinterpret_cast<const char*>(table) + e * 16);
  TapEntry t;
  t.lds_off = (int)v.x;
  t.glob_row = (int)v.y;
  t.w1 = v.z;
  t.w2 = v.w;
  return t;
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
      te[u] = lds_entry(table, e + u);
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
    const TapEntry te = lds_entry(table, e);
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

// Bin of tap offset o of range row rr (eq. 2, eq. 40) from the float64 u = beta R(o 2 pi / N)
// the caller evaluated: NEAREST near a rounding boundary is settled by the plain evaluation at
// angle (o 2 pi) / N.  LINEAR is continuous across its bin boundaries and takes floor(u).
template <int INTERP>
__device__ __forceinline__ int tap_bin(double u, const Geo& g, double rr, int o) {
  if constexpr (INTERP == ROSAR_NEAREST) {
    const double uh = u + 0.5;
    if (near_bin_tie(uh, kBinErr64))
      return (int)floor(plain_bin_half(rr, g.radius, (double)o * g.step, g.beta));
    return (int)floor(uh);
  } else {
    return (int)floor(u);
  }
}

// Bin rows [lfirst, lfirst + nrows) of the staged window of one range row, from the geometry
// alone: the slant range of a tap grows with |offset| (|R - r| at offset 0, at most that of
// offset W/2, whose cosine is cos_hw).  Uniform across the workgroup.
struct RowSpan {
  int lfirst, nrows;
};

template <int INTERP>
__device__ __forceinline__ RowSpan row_span(const Geo& g, const View& y, int row, int rows_cap, double cos_hw) {
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  const double rr = g.r0 + row * g.dr;
  const double u_near = g.beta * fabs(rr - g.radius);
  const double u_far = g.beta * sqrt(rr * rr + g.radius * g.radius - 2.0 * rr * g.radius * cos_hw);
  RowSpan sp;
  sp.lfirst = max(bin_of<INTERP>(u_near) - y.l_lo, 0);
  const int lspan = bin_of<INTERP>(u_far) - y.l_lo + NSUB - sp.lfirst;
  sp.nrows = max(min(min(rows_cap, lspan), y.l_count - sp.lfirst), 0);
  return sp;
}

// First stored column of the staged window of the tile starting at pixel a0 (direct-to-LDS
// staging starts at an aligned column), and the LDS column of pixel a0 + i at offset o:
// i + o + shift.
template <int DT>
__device__ __forceinline__ int stage_col0(const View& y, int a0, int half_w, int use_dma) {
  constexpr int CPL = 16 / Elem<DT>::bytes;
  const int c = a0 - half_w + y.halo;
  return use_dma ? (c & ~(CPL - 1)) : c;
}

// Issue the direct-to-LDS 16-byte loads of the staged rows (all NW waves; chunk (r, c) of the
// staged rows is wave (r * nchunk + c) mod NW's, all indices uniform).  The last chunk of a row
// is partial: its lanes past the row end stay idle.  Columns past the stored rotation (clamped)
// feed padded pixels only.  Completion: s_waitcnt vmcnt, then a barrier.
template <int DT, int NW>
__device__ __forceinline__ void stage_dma(const View& y, const char* __restrict__ ydata, char* stage, RowSpan sp,
                                          int col0, int stride, int wave, int lane) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int CPL = 16 / ES;
  constexpr int CHUNK = kWave * CPL;
  const int nchunk = (stride + CHUNK - 1) / CHUNK;
  const int64_t last = (int64_t)y.l_count * y.ld - CPL;
  const int lane_col = lane * CPL;
  int r = 0, ch = wave;
  while (ch >= nchunk) { ch -= nchunk; ++r; }
  while (r < sp.nrows) {
    const int c = ch * CHUNK;
    const int64_t el0 = (int64_t)(sp.lfirst + r) * y.ld + col0 + c;
    if (c + lane_col < stride) {
      int64_t el = el0 + lane_col;
      if (el0 + CHUNK - CPL > last) el = min(el, last);
      __builtin_amdgcn_global_load_lds((gbl_void_t*)(ydata + el * ES),
                                       (lds_void_t*)(stage + (r * stride + c) * ES), 16, 0, 0);
    }
    ch += NW;
    while (ch >= nchunk) { ch -= nchunk; ++r; }
  }
}

// Element-wise staging with the pulse index wrapped modulo N (used when the halo does not cover
// the window or rows are not 16-byte aligned).  Synchronous: the data is in LDS after a barrier.
template <int DT, int NW>
__device__ __forceinline__ void stage_copy(const View& y, const char* __restrict__ ydata, char* stage, RowSpan sp,
                                           int n, int a0, int half_w, int cols, int stride) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int NT = kWave * NW;
  using TE = typename Elem<DT>::T;
  constexpr int SU = 8;
  const int total = sp.nrows * cols;
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
        v[u] = *reinterpret_cast<const TE*>(ydata + ((int64_t)(sp.lfirst + r) * y.ld + pn + y.halo) * ES);
        dst[u] = (r * stride + c) * ES;
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u)
      if (dst[u] >= 0) *reinterpret_cast<TE*>(stage + dst[u]) = v[u];
  }
}

// Tap table of one range row, taps t = t0, t0 + tstep, ... (float64 bins of eq. 2 / eq. 40,
// weights packed for the storage type).  Entries whose bin row is outside the staged span are
// marked for the guard loop; returns true (for this thread) if it wrote such an entry.
template <int DT, int WDT, int INTERP>
__device__ __forceinline__ bool build_taps(const Geo& g, const View& y, int k, int half_w, int row, RowSpan sp,
                                           int stride, int shift, const int32_t* __restrict__ offsets,
                                           const void* __restrict__ weights, TapEntry* table, uint2* side, int t0,
                                           int tstep) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  const int64_t wrow = (int64_t)row * k;
  const double rr = g.r0 + row * g.dr;
  const double c1 = rr * rr + g.radius * g.radius;
  const double c2 = 2.0 * rr * g.radius;
  bool unstaged = false;
  for (int t = t0; t < k; t += tstep) {
    const int o = offsets[wrow + t];
    const float2 w = load_w<WDT>(weights, wrow + t);
    const bool inwin = o >= -half_w && o < half_w;
    int l = 0;
    float f = 0.f;
    if (inwin) {
      const double u = g.beta * sqrt(c1 - c2 * cos(o * g.step));
      l = tap_bin<INTERP>(u, g, rr, o) - y.l_lo;
      if constexpr (INTERP == ROSAR_LINEAR) f = (float)(u - floor(u));
    }
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      const int ls = l + s;
      const bool ok = inwin && ls >= 0 && ls < y.l_count;
      const bool staged = ok && ls >= sp.lfirst && ls < sp.lfirst + sp.nrows;
      const float fs = INTERP == ROSAR_NEAREST ? 1.f : (s == 0 ? 1.f - f : f);
      uint32_t w1, w2;
      pack_weight<DT>(ok ? make_float2(w.x * fs, w.y * fs) : make_float2(0.f, 0.f), w1, w2);
      TapEntry e;
      e.lds_off = staged ? ((ls - sp.lfirst) * stride + o + shift) * ES : 0;
      e.glob_row = (ok && !staged) ? (int)(ls * y.ld) : -1;
      e.w1 = staged ? w1 : 0u;
      e.w2 = staged ? w2 : 0u;
      table[t * NSUB + s] = e;
      side[t * NSUB + s] = make_uint2(w1, w2);
      unstaged |= ok && !staged;
    }
  }
  return unstaged;
}

// The P pixel chunks of one wave (pixels a_wave + lane + 64 p) into acc: staged entries from
// LDS, then the guard loop for entries outside the staged rows (if any).  a_wave < n.
template <int DT, int INTERP, int P>
__device__ __forceinline__ void wave_pixels(float2 (&acc)[P], const Geo& g, const View& y, int k, int row,
                                            int a_wave, int lane, const TapEntry* table, const uint2* side,
                                            const char* stage, uint32_t lane_base, int ne_staged, bool unstaged,
                                            const int32_t* __restrict__ offsets, const char* __restrict__ ydata) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  const int n = g.n;
  const int ne = k * NSUB;
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = make_float2(0.f, 0.f);

  // pixel chunks of 64 this wave really has (the last wave of a row may be partial)
  const int pa = min(P, (n - a_wave + kWave - 1) / kWave);
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
  if (unstaged) {
    // guard: sampled entries outside the staged rows, straight from global memory
    const int64_t wrow = (int64_t)row * k;
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
}

template <int P>
__device__ __forceinline__ void store_pixels(const float2 (&acc)[P], float inv_scale, int n, int row, int a_wave,
                                             int lane, float2* __restrict__ image) {
  float2* out = image + (int64_t)row * n;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int a = a_wave + lane + kWave * p;
    if (a < n) out[a] = make_float2(acc[p].x * inv_scale, acc[p].y * inv_scale);
  }
}

// Byte offsets of the tap table, its side copy and the staged rows in one LDS buffer.
__host__ __device__ constexpr int table_bytes(int ne) { return ne * (int)sizeof(TapEntry); }
__host__ __device__ constexpr int stage_offset(int ne) { return (ne * ((int)sizeof(TapEntry) + 8) + 15) & ~15; }

// Precomputed tap tables (sparse-filter plans).  One block per range row, in the byte layout the
// tile function stages: a 16-byte header (first staged bin row, staged row count, any entry
// outside the staged rows), the tap table and its side copy of the weights.  The entries are
// those build_taps makes inside the tile function, so both paths compute the same image.
__host__ __device__ constexpr int row_table_bytes(int ne) { return 16 + stage_offset(ne); }

template <int DT, int WDT, int INTERP>
__global__ __launch_bounds__(256) void tap_table_kernel(Geo g, View y, int32_t k, int32_t window, int rows_cap,
                                                        double cos_hw, int stride, int shift,
                                                        const int32_t* __restrict__ offsets,
                                                        const void* __restrict__ weights, char* __restrict__ tabs) {
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  const int row = blockIdx.x;
  const int ne = k * NSUB;
  char* blk = tabs + (size_t)row * row_table_bytes(ne);
  const RowSpan sp = row_span<INTERP>(g, y, row, rows_cap, cos_hw);
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  if (build_taps<DT, WDT, INTERP>(g, y, k, window / 2, row, sp, stride, shift, offsets, weights,
                                  reinterpret_cast<TapEntry*>(blk + 16),
                                  reinterpret_cast<uint2*>(blk + 16 + table_bytes(ne)), threadIdx.x, blockDim.x))
    s_any = 1;
  __syncthreads();
  if (threadIdx.x == 0) *reinterpret_cast<int4*>(blk) = make_int4(sp.lfirst, sp.nrows, s_any, 0);
}

// One workgroup's tile: `row` x pixels [tile * T, tile * T + T) of a rotation.  All threads of
// the workgroup call it; `smem` is the dynamic LDS (lds_bytes of the layout), `s_unstaged` a
// workgroup-shared int.  Staging is issued at entry, while the threads build the row's tap
// table (tap t by thread t) -- or, with PRE, copy the row's precomputed table block from `tabs`
// (tap_table_kernel; then `smem` holds 16 more bytes, the block header, in front).  Ends with
// every thread past its last LDS access, but callers that reuse `smem` for another tile must
// place a barrier in between.
template <int DT, int WDT, int INTERP, int P, int NW, bool PRE = false>
__device__ __forceinline__ void lds_tile(const Geo& g, const View& y, int32_t k, int32_t window, int row,
                                         int tile, int rows_cap, double cos_hw, int stride, int use_dma,
                                         const int32_t* __restrict__ offsets, const void* __restrict__ weights,
                                         const char* __restrict__ ydata, float2* __restrict__ image, char* smem,
                                         int& s_unstaged, const char* __restrict__ tabs = nullptr) {
  constexpr int ES = Elem<DT>::bytes;
  constexpr int NSUB = INTERP == ROSAR_LINEAR ? 2 : 1;
  constexpr int NT = kWave * NW;
  constexpr int T = kWave * P * NW;
  const int ne = k * NSUB;
  char* const hdr = smem;
  if constexpr (PRE) smem += 16;
  TapEntry* table = reinterpret_cast<TapEntry*>(smem);
  uint2* side = reinterpret_cast<uint2*>(smem + table_bytes(ne));
  char* stage = smem + stage_offset(ne);

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
  const int n = g.n;
  const int a0 = tile * T;
  const int half_w = window / 2;
  const RowSpan sp = row_span<INTERP>(g, y, row, rows_cap, cos_hw);
  const int col0 = stage_col0<DT>(y, a0, half_w, use_dma);
  if (use_dma) stage_dma<DT, NW>(y, ydata, stage, sp, col0, stride, wave, lane);
  else stage_copy<DT, NW>(y, ydata, stage, sp, n, a0, half_w, T + window, stride);
  const int shift = (a0 - half_w + y.halo) - col0 + half_w;

  if constexpr (PRE) {
    // the row's table block (header, entries, weights) straight into LDS, 16 bytes a lane
    const char* src = tabs + (size_t)row * row_table_bytes(ne);
    const int n16 = row_table_bytes(ne) / 16;
    for (int c = wave * kWave; c < n16; c += NT) {
      if (c + lane < n16)
        __builtin_amdgcn_global_load_lds((gbl_void_t*)(src + (size_t)(c + lane) * 16), (lds_void_t*)(hdr + c * 16),
                                         16, 0, 0);
    }
    (void)offsets;
    (void)weights;
    (void)shift;
    __builtin_amdgcn_s_waitcnt(0);  // direct-to-LDS loads complete
    __syncthreads();
    if (threadIdx.x == 0) s_unstaged = reinterpret_cast<const int*>(hdr)[2];
    __syncthreads();
  } else {
    if (threadIdx.x == 0) s_unstaged = 0;
    __syncthreads();
    if (build_taps<DT, WDT, INTERP>(g, y, k, half_w, row, sp, stride, shift, offsets, weights, table, side,
                                    threadIdx.x, NT))
      s_unstaged = 1;
    if (use_dma) __builtin_amdgcn_s_waitcnt(0);  // direct-to-LDS loads complete
    __syncthreads();
  }

  const int a_wave = a0 + wave * kWave * P;
  if (a_wave >= n) return;  // whole wave past the row end (no barrier below)
  const uint32_t lane_base = (uint32_t)((wave * kWave * P + lane) * ES);
  float2 acc[P];
  wave_pixels<DT, INTERP, P>(acc, g, y, k, row, a_wave, lane, table, side, stage, lane_base, sp.nrows > 0 ? ne : 0,
                             s_unstaged != 0, offsets, ydata);
  store_pixels<P>(acc, y.inv_scale, n, row, a_wave, lane, image);
}

// ---------------------------------------------------------------------------------- host side
constexpr size_t kLdsBudget = 78 * 1024;   // two workgroups per CU (160 KB of LDS), with room for static LDS

// Upper bound on the FFT rows the taps of one range row touch: the slant range of a tap grows
// with |offset| over the window (|D| <= pi), so the rows lie between those of offsets 0 and W/2.
inline int staged_rows_bound(const Geo& g, int n_range, int window, int interp, int l_count) {
  const double r = g.radius;
  const double cw = cos((window / 2) * g.step);
  int best = 1;
  for (int i = 0; i < n_range; ++i) {
    const double rr = g.r0 + i * g.dr;
    const double umin = g.beta * fabs(rr - r);
    const double umax = g.beta * sqrt(rr * rr + r * r - 2.0 * rr * r * cw);
    int cnt = interp == ROSAR_NEAREST ? (int)(floor(umax + 0.5) - floor(umin + 0.5)) + 1
                                      : (int)(floor(umax) - floor(umin)) + 2;
    best = cnt > best ? cnt : best;
  }
  return best < l_count ? best : l_count;
}

struct LdsLayout {
  int rows, stride, dma;
  size_t bytes;
  double cos_hw;   // cos((W/2) * 2 pi / N): bounds the slant range of a tap in the window
};

// LDS layout of lds_tile for tiles of `tile_px` pixels (direct-to-LDS staging needs the halo to
// cover the window and 16-byte aligned rows).
inline LdsLayout lds_layout(const Geo& g, const View& y, int k, int window, int interp, int tile_px,
                            int rows_cap_limit) {
  const int es = y.dtype == ROSAR_C64 ? 8 : 4;
  const int cpl = 16 / es;
  const int nsub = interp == ROSAR_LINEAR ? 2 : 1;
  LdsLayout L{};
  L.rows = staged_rows_bound(g, g.n_range, window, interp, y.l_count);
  if (rows_cap_limit > 0 && L.rows > rows_cap_limit) L.rows = rows_cap_limit;
  L.dma = y.halo >= window / 2 && ((y.ld * es) % 16) == 0 && (reinterpret_cast<uintptr_t>(y.data) % 16) == 0;
  const int cols = tile_px + window + cpl;
  L.stride = L.dma ? (cols + cpl - 1) / cpl * cpl : cols;   // rows stay 16-byte aligned
  const size_t table = ((size_t)k * nsub * (sizeof(TapEntry) + 8) + 15) & ~(size_t)15;
  L.bytes = table + (size_t)L.rows * L.stride * es;
  L.cos_hw = cos((window / 2) * g.step);
  return L;
}

// lds_layout with the staged rows capped so that the workgroup fits the LDS budget (taps of
// rows past the cap go through the guard path).  bytes > kLdsBudget only if one row does not fit.
inline LdsLayout lds_layout_capped(const Geo& g, const View& y, int k, int window, int interp, int tile_px) {
  LdsLayout full = lds_layout(g, y, k, window, interp, tile_px, 0);
  const int es = y.dtype == ROSAR_C64 ? 8 : 4;
  const size_t per_row = (size_t)full.stride * es;
  const size_t table = full.bytes - (size_t)full.rows * per_row;
  int cap = full.rows;
  while (cap > 1 && table + (size_t)cap * per_row > kLdsBudget) --cap;
  return cap == full.rows ? full : lds_layout(g, y, k, window, interp, tile_px, cap);
}

}  // namespace sparse
}  // namespace rosar
