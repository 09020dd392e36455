// Windowed range FFT of a group of pulses (Sec. III-D, eq. 38), shared by the single-rotation
// range-compression kernel and the batched kernel.
//
// One wavefront transforms one pulse at a time with a Stockham autosort FFT (radix 8, then 4
// or 2 for the remaining factor) in LDS; twiddles come from an LDS table of
// exp(-j 2 pi t / L).  The first pass reads the raw samples straight from HBM (zero padding
// past M) and applies the window from LDS.  A workgroup of NW waves handles NW*PPW pulses, then
// writes the transposed band with NW*PPW consecutive pulses per row segment, plus the circular
// halo copies of the first/last `halo` pulses.  Each wave owns its pulses' LDS rows, so the
// passes order their LDS accesses with wave-level fences; the workgroup synchronises only
// around the twiddle/window tables and before the transposed store.
#pragma once

#include "rosar_device.hpp"

namespace rosar {
namespace fft {


// Orders the LDS accesses of one wavefront (each wave owns its pulses' rows in LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS layout of one pulse row: element i sits at i + i/32, so the strided Stockham writes (and
// reads) of a pass spread over the banks instead of piling onto a few; the row pitch is odd so
// that the transposed store, which reads one element from each of several rows, does not
// conflict either.
__device__ __forceinline__ constexpr int lds_idx(int i) { return i + (i >> 5); }
constexpr int row_pitch(int l) { return l + l / 32 + 1; }

constexpr int radix_of(int x) { return (x % 8 == 0) ? 8 : ((x % 4 == 0) ? 4 : 2); }
constexpr int pass_count(int l) {
  int p = 0;
  while (l > 1) { l /= radix_of(l); ++p; }
  return p;
}
constexpr int pass_radix(int l, int pass) {
  for (int i = 0; i < pass; ++i) l /= radix_of(l);
  return radix_of(l);
}
constexpr int pass_ns(int l, int pass) {
  int ns = 1;
  for (int i = 0; i < pass; ++i) { int r = radix_of(l); ns *= r; l /= r; }
  return ns;
}

// Forward DFT of length R in registers: X[q] = sum_r v[r] exp(-j 2 pi r q / R).
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = make_float2(t.x + b.x, t.y + b.y);
  b = make_float2(t.x - b.x, t.y - b.y);
}

__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = make_float2(a0.x + a2.x, a0.y + a2.y);
  float2 t1 = make_float2(a0.x - a2.x, a0.y - a2.y);
  float2 t2 = make_float2(a1.x + a3.x, a1.y + a3.y);
  float2 t3 = make_float2(a1.x - a3.x, a1.y - a3.y);
  a0 = make_float2(t0.x + t2.x, t0.y + t2.y);
  a2 = make_float2(t0.x - t2.x, t0.y - t2.y);
  a1 = make_float2(t1.x + t3.y, t1.y - t3.x);   // t1 - j t3
  a3 = make_float2(t1.x - t3.y, t1.y + t3.x);   // t1 + j t3
}

template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else {
    // radix 8 = two length-4 DFTs (even/odd inputs) combined with exp(-j 2 pi q / 8)
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const float c = 0.70710678118654752440f;
    float2 w1 = make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));    // (1-j)/sqrt2 * o1
    float2 w2 = make_float2(o2.y, -o2.x);                              // -j * o2
    float2 w3 = make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));   // (-1-j)/sqrt2 * o3
    v[0] = make_float2(e0.x + o0.x, e0.y + o0.y);
    v[4] = make_float2(e0.x - o0.x, e0.y - o0.y);
    v[1] = make_float2(e1.x + w1.x, e1.y + w1.y);
    v[5] = make_float2(e1.x - w1.x, e1.y - w1.y);
    v[2] = make_float2(e2.x + w2.x, e2.y + w2.y);
    v[6] = make_float2(e2.x - w2.x, e2.y - w2.y);
    v[3] = make_float2(e3.x + w3.x, e3.y + w3.y);
    v[7] = make_float2(e3.x - w3.x, e3.y - w3.y);
  }
}

constexpr int pass_bpl(int l, int pass) { return (l / pass_radix(l, pass) + kWave - 1) / kWave; }

template <int L, int PASS>
struct PassShape {
  static constexpr int R = pass_radix(L, PASS);
  static constexpr int NS = pass_ns(L, PASS);
  static constexpr int NB = L / R;                          // butterflies per pulse
  static constexpr int BPL = (NB + kWave - 1) / kWave;      // butterflies per lane
};

// Operands of one Stockham pass of radix R (after NS points have been combined) for the PPW
// pulses of a wave: from the pulse rows of `buf` in LDS, or for the first pass the raw samples
// from global memory (zero padding past M, zero for pulses past N; the window is applied
// separately, see apply_window).
template <int L, int PPW, int PASS>
__device__ __forceinline__ void pass_load(float2 (&v)[PPW][pass_bpl(L, PASS)][pass_radix(L, PASS)],
                                          const float2* buf, int wave, int lane, const RcArgs& a, int n0) {
  using S = PassShape<L, PASS>;
  constexpr int LP = row_pitch(L);
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int wp = wave * PPW + p;
    const int n = n0 + wp;
#pragma unroll
    for (int b = 0; b < S::BPL; ++b) {
      const int j = lane + kWave * b;
#pragma unroll
      for (int r = 0; r < S::R; ++r) {
        const int idx = j + r * S::NB;
        float2 x = make_float2(0.f, 0.f);
        if constexpr (PASS == 0) {
          if (j < S::NB && n < a.n && idx < a.m) x = a.raw[(int64_t)n * a.m + idx];
        } else {
          if (j < S::NB) x = buf[wp * LP + lds_idx(idx)];
        }
        v[p][b][r] = x;
      }
    }
  }
}

// First-pass operands times the window staged in LDS (samples past M are zero already).
template <int L, int PPW>
__device__ __forceinline__ void apply_window(float2 (&v)[PPW][pass_bpl(L, 0)][pass_radix(L, 0)],
                                             const float* win, int lane, int m) {
  using S = PassShape<L, 0>;
#pragma unroll
  for (int p = 0; p < PPW; ++p)
#pragma unroll
    for (int b = 0; b < S::BPL; ++b)
#pragma unroll
      for (int r = 0; r < S::R; ++r) {
        const int idx = lane + kWave * b + r * S::NB;
        const float h = idx < m ? win[idx] : 0.f;
        v[p][b][r].x *= h;
        v[p][b][r].y *= h;
      }
}

// Twiddles, radix-R DFT and the Stockham write of one pass (in place on the pulse rows).
template <int L, int PPW, int PASS>
__device__ __forceinline__ void pass_compute(float2 (&v)[PPW][pass_bpl(L, PASS)][pass_radix(L, PASS)],
                                             float2* buf, const float2* tw, int wave, int lane) {
  using S = PassShape<L, PASS>;
  constexpr int R = S::R, NS = S::NS, NB = S::NB;
  constexpr int LP = row_pitch(L);
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int wp = wave * PPW + p;
#pragma unroll
    for (int b = 0; b < S::BPL; ++b) {
      const int j = lane + kWave * b;
      if (j < NB) {
        const int k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) v[p][b][r] = cmul(v[p][b][r], tw[k * r * (L / (NS * R))]);
        }
        dft<R>(v[p][b]);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) buf[wp * LP + lds_idx(base + q * NS)] = v[p][b][q];
      }
    }
  }
  wave_sync();
}

// Passes PASS.. of the FFT, each reading the previous pass's rows from LDS.
template <int L, int PPW, int PASS>
__device__ __forceinline__ void fft_rest(float2* buf, const float2* tw, int wave, int lane, const RcArgs& a) {
  if constexpr (PASS < pass_count(L)) {
    using S = PassShape<L, PASS>;
    float2 v[PPW][S::BPL][S::R];
    pass_load<L, PPW, PASS>(v, buf, wave, lane, a, 0);
    wave_sync();
    pass_compute<L, PPW, PASS>(v, buf, tw, wave, lane);
    fft_rest<L, PPW, PASS + 1>(buf, tw, wave, lane, a);
  }
}


// Two band elements of consecutive pulses (idx even) as one 16-byte (complex64) or 8-byte
// (16-bit pairs) store.
template <int DT>
__device__ __forceinline__ void store_c2(void* base, int64_t idx, float2 v0, float2 v1) {
  if constexpr (DT == 0) {
    reinterpret_cast<float4*>(base)[idx >> 1] = make_float4(v0.x, v0.y, v1.x, v1.y);
  } else if constexpr (DT == 1) {
    const __half2 h0 = __floats2half2_rn(v0.x, v0.y), h1 = __floats2half2_rn(v1.x, v1.y);
    uint2 u;
    __builtin_memcpy(&u.x, &h0, sizeof(uint32_t));
    __builtin_memcpy(&u.y, &h1, sizeof(uint32_t));
    reinterpret_cast<uint2*>(base)[idx >> 1] = u;
  } else {
    uint2 u;
    u.x = f32_to_bf16_rne(v0.x) | (f32_to_bf16_rne(v0.y) << 16);
    u.y = f32_to_bf16_rne(v1.x) | (f32_to_bf16_rne(v1.y) << 16);
    reinterpret_cast<uint2*>(base)[idx >> 1] = u;
  }
}

// Transposed band store for even N, halo and row pitch (and an aligned band): each thread owns
// pulses (2h, 2h + 1) of the block and writes them as one store per row, so a wave covers
// 2 * kWave / PW rows with PW consecutive pulses each.  The LDS reads of two sweeps are issued
// before their stores.  Pulse pairs never straddle N or a halo boundary, since all three are even.
template <int L, int PPW, int DT, int NW>
__device__ __forceinline__ void store_band_pairs(const RcArgs& a, int n0, const float2* buf) {
  constexpr int PW = NW * PPW, LP = row_pitch(L), NT = NW * kWave;
  constexpr int HP = PW / 2;          // threads per row segment
  constexpr int RS = NT / HP;         // rows per sweep of the workgroup
  constexpr int U = 2;                // sweeps whose reads go out together
  static_assert(PW % 2 == 0, "pulse pairs");
  const int tid = threadIdx.x;
  const int pp = 2 * (tid % HP), r0 = tid / HP;
  const int n = n0 + pp;
  if (n >= a.n) return;
  const bool h_lo = n < a.halo, h_hi = n >= a.n - a.halo;
  const float2* s0 = buf + pp * LP;
  const float2* s1 = s0 + LP;
  for (int base = r0; base < a.l_count; base += RS * U) {
    float2 v0[U], v1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int lr = base + u * RS;
      const bool in = lr < a.l_count;
      v0[u] = in ? s0[lds_idx(a.l_lo + lr)] : make_float2(0.f, 0.f);
      v1[u] = in ? s1[lds_idx(a.l_lo + lr)] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int lr = base + u * RS;
      if (lr < a.l_count) {
        float2 w0 = v0[u], w1 = v1[u];
        w0.x *= a.scale;
        w0.y *= a.scale;
        w1.x *= a.scale;
        w1.y *= a.scale;
        const int64_t at = (int64_t)lr * a.ld + n + a.halo;
        store_c2<DT>(a.out, at, w0, w1);
        if (h_lo) store_c2<DT>(a.out, at + a.n, w0, w1);
        if (h_hi) store_c2<DT>(a.out, at - a.n, w0, w1);
      }
    }
  }
}

// LDS float2 needed by rc_block<L, PPW, NW>: twiddle table, NW*PPW padded pulse rows and the
// window (L floats).
constexpr int rc_lds_elems(int l, int ppw, int nw) { return l + nw * ppw * row_pitch(l) + l / 2; }

// Range-compress pulses [n0, n0 + NW*PPW) of one rotation: FFT each (wave w owns pulses
// n0 + w*PPW ...), then store the band transposed with NW*PPW consecutive pulses per row
// segment.  The first pass's raw samples are requested before the workgroup builds the
// twiddle table and stages the window, so their latency overlaps that work.  `lds` holds
// rc_lds_elems(L, PPW, NW) float2.  All threads of the workgroup call it.
template <int L, int PPW, int DT, int NW>
__device__ __forceinline__ void rc_block(const RcArgs& a, int n0, float2* lds) {
  constexpr int PW = NW * PPW;
  constexpr int LP = row_pitch(L);
  constexpr int NT = NW * kWave;
  float2* tw = lds;
  float2* buf = lds + L;
  float* win = reinterpret_cast<float*>(lds + L + PW * LP);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  using S0 = PassShape<L, 0>;
  float2 v[PPW][S0::BPL][S0::R];
  if (S0::NB % kWave == 0 && a.m >= L && n0 + (wave + 1) * PPW <= a.n) {
    // whole pulses, every lane in range: plain loads at constant offsets, no per-element guard
    const float2* src = a.raw + (int64_t)(n0 + wave * PPW) * a.m + lane;
#pragma unroll
    for (int p = 0; p < PPW; ++p)
#pragma unroll
      for (int b = 0; b < S0::BPL; ++b)
#pragma unroll
        for (int r = 0; r < S0::R; ++r) v[p][b][r] = src[(int64_t)p * a.m + kWave * b + r * S0::NB];
  } else {
    pass_load<L, PPW, 0>(v, buf, wave, lane, a, n0);
  }
  for (int t = tid; t < L; t += NT) {
    float s, c;
    sincospif(-2.0f * (float)t / (float)L, &s, &c);
    tw[t] = make_float2(c, s);
    win[t] = t < a.m ? (a.window ? a.window[t] : 1.f) : 0.f;
  }
  __syncthreads();
  apply_window<L, PPW>(v, win, lane, a.m);
  pass_compute<L, PPW, 0>(v, buf, tw, wave, lane);
  fft_rest<L, PPW, 1>(buf, tw, wave, lane, a);
  __syncthreads();

  if (((a.ld | a.halo | a.n) & 1) == 0 && ((uintptr_t)a.out & (DT == 0 ? 15 : 7)) == 0) {
    store_band_pairs<L, PPW, DT, NW>(a, n0, buf);
    return;
  }
  // transposed store of the band: PW consecutive pulses form one contiguous row segment
  const int total = a.l_count * PW;
  for (int i = tid; i < total; i += NT) {
    const int pp = i % PW;
    const int lr = i / PW;
    const int n = n0 + pp;
    if (n >= a.n) continue;
    float2 v2 = buf[pp * LP + lds_idx(a.l_lo + lr)];
    v2.x *= a.scale;
    v2.y *= a.scale;
    const int64_t row = (int64_t)lr * a.ld;
    store_c<DT>(a.out, row + n + a.halo, v2);
    if (n < a.halo) store_c<DT>(a.out, row + n + a.halo + a.n, v2);
    if (n >= a.n - a.halo) store_c<DT>(a.out, row + n + a.halo - a.n, v2);
  }
}

}  // namespace fft
}  // namespace rosar
