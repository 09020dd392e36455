// Adjoint of the sparse-aperture filter (Algorithm 2 with eq. 43, no angle or phase errors) with
// respect to the range-compressed band.  The filter is linear in the band:
//   I[r, a] = sum_k conj(w[r, k]) c Y[l_k, (a + o_k) mod N]
// (c = 1 for NEAREST, 1 - f or f on the two bins of a LINEAR tap), so for a real loss with
// g = dL/dRe(I) + j dL/dIm(I)
//   grad_Y[l, n] = sum over taps (r, k) reading bin row l of w[r, k] c g[r, (n - o_k) mod N].
// Per band row this is a gather: only the range rows whose taps reach bin row l contribute, and a
// range row's taps reach at most 32 consecutive bin rows.  The tap lists (float64 bins, the same
// expression as the forward filter's tables) are written to the caller's workspace first; then
// one workgroup per (band row, pulse tile) marks the contributing range rows in an LDS bitmask
// and walks them in increasing order, so the sum order is fixed and results are reproducible.
#include <hip/hip_runtime.h>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kAdjThreads = 256;
constexpr int kAdjP = 4;   // pulses per thread
constexpr int kAdjTile = kAdjThreads * kAdjP;

__global__ __launch_bounds__(kAdjThreads) void adjoint_band_kernel(int n, int n_range, int tiles,
                                                                   const char* __restrict__ tabs, int row_bytes,
                                                                   const float2* __restrict__ grad_image,
                                                                   float2* __restrict__ grad_band) {
  extern __shared__ uint32_t s_rows[];   // ceil(n_range / 32) words
  const int l = blockIdx.x / tiles;
  const int n0 = (blockIdx.x % tiles) * kAdjTile;
  const int tid = threadIdx.x;
  const int words = (n_range + 31) / 32;
  for (int i = tid; i < words; i += kAdjThreads) s_rows[i] = 0u;
  __syncthreads();
  for (int r = tid; r < n_range; r += kAdjThreads) {
    const int4 h = *reinterpret_cast<const int4*>(tabs + (size_t)r * row_bytes);
    const int rel = l - h.x;
    if (rel >= 0 && rel < 32 && ((unsigned)h.y >> rel) & 1u) atomicOr(&s_rows[r >> 5], 1u << (r & 31));
  }
  __syncthreads();

  float2 acc[kAdjP];
#pragma unroll
  for (int p = 0; p < kAdjP; ++p) acc[p] = make_float2(0.f, 0.f);
  for (int wi = 0; wi < words; ++wi) {
    for (unsigned m = s_rows[wi]; m; m &= m - 1u) {
      const int r = wi * 32 + __builtin_ctz(m);
      const int4* blk = reinterpret_cast<const int4*>(tabs + (size_t)r * row_bytes);
      const int4 h = blk[0];
      const int rel = l - h.x;
      const float2* grow = grad_image + (size_t)r * n;
      for (int e = 0; e < h.z; ++e) {
        const int4 t = blk[1 + e];
        if (t.y != rel) continue;
        // the table holds conj(w) c (the forward coefficient); the adjoint applies w c
        const float cx = __int_as_float(t.z), cy = -__int_as_float(t.w);
#pragma unroll
        for (int p = 0; p < kAdjP; ++p) {
          const int np = n0 + tid + p * kAdjThreads;
          if (np < n) {
            int a = np - t.x;
            a += a < 0 ? n : 0;
            const float2 gv = grow[a];
            acc[p].x = fmaf(cx, gv.x, fmaf(-cy, gv.y, acc[p].x));
            acc[p].y = fmaf(cx, gv.y, fmaf(cy, gv.x, acc[p].y));
          }
        }
      }
    }
  }
  float2* out = grad_band + (size_t)l * n;
#pragma unroll
  for (int p = 0; p < kAdjP; ++p) {
    const int np = n0 + tid + p * kAdjThreads;
    if (np < n) out[np] = acc[p];
  }
}

}  // namespace

size_t adjoint_band_workspace_bytes(const FcLayout& L, int32_t n_range) {
  return (size_t)L.row_bytes * (size_t)n_range + 256;
}

hipError_t launch_adjoint_band(const SparseArgs& a, const FcLayout& L, const float2* grad_image, float2* grad_band,
                               void* ws, hipStream_t s) {
  char* tabs = static_cast<char*>(ws);
  int* bad = reinterpret_cast<int*>(tabs + (size_t)L.row_bytes * a.g.n_range);   // set only past the host bound
  hipError_t e = launch_fc_tables(a, L, tabs, bad, s);
  if (e != hipSuccess) return e;
  const int tiles = (a.g.n + kAdjTile - 1) / kAdjTile;
  const size_t lds = (size_t)((a.g.n_range + 31) / 32) * sizeof(uint32_t);
  adjoint_band_kernel<<<a.y.l_count * tiles, kAdjThreads, lds, s>>>(a.g.n, a.g.n_range, tiles, tabs, L.row_bytes,
                                                                    grad_image, grad_band);
  return hipGetLastError();
}

}  // namespace rosar
