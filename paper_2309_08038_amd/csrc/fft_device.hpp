// Windowed range FFT of a group of pulses (Sec. III-D, eq. 38), shared by the single-rotation
// range-compression kernel and the persistent batched kernel.
//
// One wavefront transforms one pulse at a time with a Stockham autosort FFT (radix 8, then 4
// or 2 for the remaining factor) in LDS; twiddles come from an LDS table of
// exp(-j 2 pi t / L).  The first pass reads raw samples straight from HBM with the window and
// zero padding applied.  A workgroup of NW waves handles NW*PPW pulses, then writes the
// transposed band with NW*PPW consecutive pulses per row segment, plus the circular halo
// copies of the first/last `halo` pulses.  Each wave owns its pulses' LDS rows, so the passes
// order their LDS accesses with wave-level fences; the workgroup synchronises only around the
// twiddle table and before the transposed store.
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

// One Stockham pass of radix R after `NS` points have been combined; in place on each pulse
// row of `buf` (read phase, barrier, write phase, barrier).  The first pass (NS == 1) loads
// the windowed, zero-padded raw samples from global memory instead of LDS.
template <int L, int PPW, int PASS>
__device__ __forceinline__ void fft_pass(float2* buf, const float2* tw, int wave, int lane,
                                         const RcArgs& a, int n0) {
  constexpr int R = pass_radix(L, PASS);
  constexpr int NS = pass_ns(L, PASS);
  constexpr int NB = L / R;
  constexpr int BPL = (NB + kWave - 1) / kWave;
  constexpr int LP = L + 1;
  float2 v[PPW][BPL][R];
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int wp = wave * PPW + p;
    const int n = n0 + wp;
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
      const int j = lane + kWave * b;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = j + r * NB;
        float2 x = make_float2(0.f, 0.f);
        if constexpr (PASS == 0) {
          if (j < NB && n < a.n && idx < a.m) {
            x = a.raw[(int64_t)n * a.m + idx];
            if (a.window) { float h = a.window[idx]; x.x *= h; x.y *= h; }
          }
        } else {
          if (j < NB) x = buf[wp * LP + idx];
        }
        v[p][b][r] = x;
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int p = 0; p < PPW; ++p) {
    const int wp = wave * PPW + p;
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
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
        for (int q = 0; q < R; ++q) buf[wp * LP + base + q * NS] = v[p][b][q];
      }
    }
  }
  wave_sync();
}

template <int L, int PPW, int PASS>
__device__ __forceinline__ void fft_all(float2* buf, const float2* tw, int wave, int lane,
                                        const RcArgs& a, int n0) {
  if constexpr (PASS < pass_count(L)) {
    fft_pass<L, PPW, PASS>(buf, tw, wave, lane, a, n0);
    fft_all<L, PPW, PASS + 1>(buf, tw, wave, lane, a, n0);
  }
}


// LDS float2 needed by rc_block<L, PPW, NW>: twiddle table + NW*PPW padded pulse rows.
constexpr int rc_lds_elems(int l, int ppw, int nw) { return l + nw * ppw * (l + 1); }

// Range-compress pulses [n0, n0 + NW*PPW) of one rotation: FFT each (wave w owns pulses
// n0 + w*PPW ...), then store the band transposed with NW*PPW consecutive pulses per row
// segment.  `lds` holds rc_lds_elems(L, PPW, NW) float2.  All threads of the workgroup call it.
template <int L, int PPW, int DT, int NW>
__device__ __forceinline__ void rc_block(const RcArgs& a, int n0, float2* lds) {
  constexpr int PW = NW * PPW;
  constexpr int LP = L + 1;
  constexpr int NT = NW * kWave;
  float2* tw = lds;
  float2* buf = lds + L;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  for (int t = tid; t < L; t += NT) {
    float s, c;
    sincospif(-2.0f * (float)t / (float)L, &s, &c);
    tw[t] = make_float2(c, s);
  }
  __syncthreads();
  fft_all<L, PPW, 0>(buf, tw, wave, lane, a, n0);
  __syncthreads();

  // transposed store of the band: PW consecutive pulses form one contiguous row segment
  const int total = a.l_count * PW;
  for (int i = tid; i < total; i += NT) {
    const int pp = i % PW;
    const int lr = i / PW;
    const int n = n0 + pp;
    if (n >= a.n) continue;
    float2 v = buf[pp * LP + a.l_lo + lr];
    v.x *= a.scale;
    v.y *= a.scale;
    const int64_t row = (int64_t)lr * a.ld;
    store_c<DT>(a.out, row + n + a.halo, v);
    if (n < a.halo) store_c<DT>(a.out, row + n + a.halo + a.n, v);
    if (n >= a.n - a.halo) store_c<DT>(a.out, row + n + a.halo - a.n, v);
  }
}

}  // namespace fft
}  // namespace rosar
