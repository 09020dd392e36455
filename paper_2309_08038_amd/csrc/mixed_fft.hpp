// Workgroup-wide complex FFT of one row held in LDS, any length N = 2^a 3^b 5^c up to
// kFftMaxN: Stockham autosort passes of radix 8, 4, 2, 5 and 3.  Each pass reads its
// butterflies' inputs into registers, synchronises, and writes the outputs back into the same
// LDS buffer, so one N-element buffer suffices.  A twiddle exp(-j 2 pi t / N) is the product of
// two entries of small LDS tables, lo[t mod 64] = exp(-j 2 pi (t mod 64) / N) and
// hi[t / 64] = exp(-j 2 pi 64 (t / 64) / N), both evaluated in float64 on the host: 1.5 KB of
// LDS instead of an N-entry table, and no global-memory latency inside a pass.
//
// DIR = -1: X[m] = sum_n x[n] exp(-j 2 pi n m / N) (forward); DIR = +1: the same with +j
// (unnormalised inverse).
#pragma once

#include "rosar_device.hpp"

namespace rosar {
namespace mfft {

constexpr int kFftThreads = 512;
constexpr int kFftMaxN = 8192;

// Radix sequence of one length (host-built; the product of radix[0..n_pass) is n).
using Factors = FftFactors;

constexpr int kTwLo = 64;
constexpr int kTwHi = kFftMaxN / kTwLo;

// The twiddle tables in LDS (global layout: kTwLo lo entries, then ceil(N / 64) hi entries).
struct Twiddles {
  float2 lo[kTwLo];
  float2 hi[kTwHi];
};

__host__ __device__ constexpr int twiddle_count(int n) { return kTwLo + (n + kTwLo - 1) / kTwLo; }

// Copies the tables into LDS; the caller synchronises before the first pass.
__device__ __forceinline__ void load_twiddles(Twiddles& t, const float2* __restrict__ tw, int n, int tid) {
  const int cnt = twiddle_count(n);
  for (int i = tid; i < cnt; i += kFftThreads) {
    if (i < kTwLo) t.lo[i] = tw[i];
    else t.hi[i - kTwLo] = tw[i];
  }
}

// The same tables evaluated in the kernel (float32 sincospi of the exact ratio t / N), for
// callers without a host-built table.
__device__ __forceinline__ void make_twiddles(Twiddles& t, int n, int tid) {
  const int cnt = twiddle_count(n);
  for (int i = tid; i < cnt; i += kFftThreads) {
    const int tt = i < kTwLo ? i : (i - kTwLo) * kTwLo;
    float sn, cs;
    sincospif(-2.0f * (float)tt / (float)n, &sn, &cs);
    if (i < kTwLo) t.lo[i] = make_float2(cs, sn);
    else t.hi[i - kTwLo] = make_float2(cs, sn);
  }
}

// j * z for DIR = +1, -j * z for DIR = -1.
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 z) {
  return DIR > 0 ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// In-register DFT of R points with exp(DIR j 2 pi / R) as the root of unity.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = rot90<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
  } else if constexpr (R == 8) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, DIR>(e);
    dft<4, DIR>(o);
    constexpr float h = 0.70710678118654752440f;
    // o[q] * exp(DIR j 2 pi q / 8)
    o[1] = cscale(cadd(o[1], rot90<DIR>(o[1])), h);
    o[2] = rot90<DIR>(o[2]);
    o[3] = cscale(csub(rot90<DIR>(o[3]), o[3]), h);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = cadd(e[q], o[q]);
      v[q + 4] = csub(e[q], o[q]);
    }
  } else if constexpr (R == 3) {
    constexpr float s3 = 0.86602540378443864676f;   // sin(2 pi / 3)
    const float2 s = cadd(v[1], v[2]);
    const float2 d = rot90<DIR>(cscale(csub(v[1], v[2]), s3));
    const float2 h = csub(v[0], cscale(s, 0.5f));
    v[0] = cadd(v[0], s);
    v[1] = cadd(h, d);
    v[2] = csub(h, d);
  } else if constexpr (R == 5) {
    constexpr float c1 = 0.30901699437494742410f;    // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742410f;   // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357212f;    // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247312917f;    // sin(4 pi / 5)
    const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const float2 a = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    const float2 b = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    const float2 p = rot90<DIR>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
    const float2 q = rot90<DIR>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a, p);
    v[4] = csub(a, p);
    v[2] = cadd(b, q);
    v[3] = csub(b, q);
  }
}

// One Stockham pass of radix R over sub-transforms of length ns (ns * R divides n).  Butterfly
// j reads buf[j + i n/R], applies the twiddles exp(DIR j 2 pi i k / (ns R)) with k = j mod ns,
// and writes buf[(j - k) R + k + i ns].  All threads of the block call it.
template <int R, int DIR>
__device__ __forceinline__ void fft_pass(float2* buf, int n, int ns, const Twiddles& tw, int tid) {
  constexpr int MAXB = (kFftMaxN / R + kFftThreads - 1) / kFftThreads;
  const int nb = n / R;
  const int tstep = n / (ns * R);
  // j / ns as a multiply-high for ns >= 2 (magic = ceil(2^32 / ns) < 2^32): exact for
  // j, ns <= 8192 since j * (magic * ns - 2^32) < 2^32.  ns == 1 gives k = 0.
  const uint32_t magic = ns > 1 ? (uint32_t)((0x100000000ull + (uint64_t)ns - 1) / (uint64_t)ns) : 0u;
  float2 v[MAXB][R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = tid + b * kFftThreads;
    if (j < nb) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[b][i] = buf[j + i * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = tid + b * kFftThreads;
    if (j < nb) {
      const int k = ns > 1 ? j - (int)__umulhi((uint32_t)j, magic) * ns : 0;
      if (k != 0) {
#pragma unroll
        for (int i = 1; i < R; ++i) {
          const int t = i * k * tstep;
          float2 w = cmul(tw.hi[t >> 6], tw.lo[t & (kTwLo - 1)]);
          if (DIR > 0) w.y = -w.y;
          v[b][i] = cmul(v[b][i], w);
        }
      }
      dft<R, DIR>(v[b]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int i = 0; i < R; ++i) buf[base + i * ns] = v[b][i];
    }
  }
  __syncthreads();
}

// The whole transform; `buf` holds the row on entry and the result on exit (block-uniform
// arguments; the caller synchronises before, the last pass synchronises after).
template <int DIR>
__device__ __forceinline__ void block_fft(float2* buf, const Factors& f, const Twiddles& tw, int tid) {
  int ns = 1;
  for (int p = 0; p < f.n_pass; ++p) {
    switch (f.radix[p]) {
      case 8: fft_pass<8, DIR>(buf, f.n, ns, tw, tid); break;
      case 4: fft_pass<4, DIR>(buf, f.n, ns, tw, tid); break;
      case 2: fft_pass<2, DIR>(buf, f.n, ns, tw, tid); break;
      case 5: fft_pass<5, DIR>(buf, f.n, ns, tw, tid); break;
      default: fft_pass<3, DIR>(buf, f.n, ns, tw, tid); break;
    }
    ns *= f.radix[p];
  }
}

}  // namespace mfft
}  // namespace rosar
