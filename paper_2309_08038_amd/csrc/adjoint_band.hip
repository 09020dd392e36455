// Adjoint of the sparse-aperture filter (Algorithm 2 with eq. 43, no angle or phase errors) with
// respect to the range-compressed band.  The filter is linear in the band:
//   I[r, a] = sum_k conj(w[r, k]) c Y[l_k, (a + o_k) mod N]
// (c = 1 for NEAREST, 1 - f or f on the two bins of a LINEAR tap), so for a real loss with
// g = dL/dRe(I) + j dL/dIm(I)
//   grad_Y[l, n] = sum over taps (r, k) reading bin row l of w[r, k] c g[r, (n - o_k) mod N].
// Per band row this is a gather: only the range rows whose taps reach bin row l contribute, and a
// range row's taps reach at most 32 consecutive bin rows.  The tap lists (float64 bins, the same
// expression as the forward filter's tables) are written to the caller's workspace first; then
// one workgroup per (band row, pulse tile) finds the contributing range rows and walks them in
// increasing order (the staged form lists them in LDS with an ordered ballot, the direct form
// marks them in an LDS bitmask), so the sum order is fixed and results are reproducible.
// The staged form copies, batch by batch, the gradient rows of the contributing range rows over
// the columns the tile's taps reach ([n0 - W/2, n0 + T + W/2], modulo N) into LDS; the direct
// form (kept for windows too wide for one staged row) reads them from global memory.  Both add
// the same terms in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>

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

constexpr int kAdjMaxRows = 8;            // staged gradient rows per batch
constexpr size_t kAdjLdsBudget = 40 * 1024;
constexpr int kAdjWaves = kAdjThreads / kWave;
constexpr int kAdjU = 4;                  // taps whose stage reads are issued together
constexpr int kAdjRowsPer = 4;            // row headers per thread requested together
constexpr int kAdjTilesPer = 1;           // pulse tiles of one band row per workgroup (4: 190 us, too few workgroups)

__host__ __device__ constexpr int rows_words(int n_range) { return ((n_range + 31) / 32 + 3) & ~3; }
__host__ __device__ constexpr int list_words(int n_range) { return (n_range + 3) & ~3; }

// Staged form.  Dynamic LDS: the list of contributing rows (list_words words, each
// (row << 5) | bin offset, in increasing row order), then cap * ne compacted taps {LDS offset of
// the tap's first sample, coef.x, coef.y, 0}, then cap staged gradient rows.
__global__ __launch_bounds__(kAdjThreads) void adjoint_band_staged_kernel(int n, int n_range, int tiles, int groups,
                                                                          int half_w,
                                                                          int cap, int ne, const char* __restrict__ tabs,
                                                                          int row_bytes,
                                                                          const float2* __restrict__ grad_image,
                                                                          float2* __restrict__ grad_band) {
  extern __shared__ int4 s_dyn[];   // int4: the tap table's 16-byte LDS reads need 16-byte alignment
  __shared__ int s_wcnt[kAdjWaves];
  __shared__ int s_ntaps;
  const int l = blockIdx.x / groups;
  const int tile0 = (blockIdx.x % groups) * kAdjTilesPer;   // this workgroup's tiles: tile0 + [0, kAdjTilesPer)
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int width = kAdjTile + 2 * half_w + 1;   // staged columns of a tile: n0 - half_w + [0, width)
  int* rows = reinterpret_cast<int*>(s_dyn);
  int4* taps = s_dyn + list_words(n_range) / 4;
  float2* stage = reinterpret_cast<float2*>(taps + cap * ne);

  // The contributing range rows (a tap on band row l), listed in increasing order: the headers
  // of kAdjRowsPer * kAdjThreads rows are requested together, then a ballot per wave and
  // chunk, the waves' counts added in wave order.  Every thread tracks the same running count.
  int nrows = 0;
  for (int base = 0; base < n_range; base += kAdjRowsPer * kAdjThreads) {
    int4 h[kAdjRowsPer];
#pragma unroll
    for (int q = 0; q < kAdjRowsPer; ++q) {
      const int r = base + q * kAdjThreads + tid;
      h[q] = r < n_range ? *reinterpret_cast<const int4*>(tabs + (size_t)r * row_bytes) : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < kAdjRowsPer; ++q) {
      const int r = base + q * kAdjThreads + tid;
      const int rel = l - h[q].x;
      const bool match = r < n_range && rel >= 0 && rel < 32 && (((unsigned)h[q].y >> rel) & 1u);
      const uint64_t bal = __ballot(match);
      if (lane == 0) s_wcnt[wave] = __popcll(bal);
      __syncthreads();
      int off = nrows, tot = 0;
#pragma unroll
      for (int w2 = 0; w2 < kAdjWaves; ++w2) {
        const int c = s_wcnt[w2];
        off += w2 < wave ? c : 0;
        tot += c;
      }
      if (match) rows[off + __popcll(bal & ((1ull << lane) - 1ull))] = (r << 5) | rel;
      nrows += tot;
      __syncthreads();   // s_wcnt is rewritten by the next chunk
    }
  }

  float2 acc[kAdjTilesPer][kAdjP];
#pragma unroll
  for (int tt = 0; tt < kAdjTilesPer; ++tt)
#pragma unroll
    for (int p = 0; p < kAdjP; ++p) acc[tt][p] = make_float2(0.f, 0.f);
  for (int b0 = 0; b0 < nrows; b0 += cap) {
    // the batch rows[b0, b0 + cnt)
    const int cnt = min(cap, nrows - b0);
    if (tid == 0) s_ntaps = 0;
    __syncthreads();
    // compact the batch's taps on band row l, in (row, entry) order: a ballot per wave, the
    // waves' counts added in wave order
    const int total = cnt * ne;
    for (int base = 0; base < total; base += kAdjThreads) {
      const int idx = base + tid;
      int4 t = make_int4(0, -1, 0, 0);
      int slot = 0, rel = -2;
      if (idx < total) {
        slot = idx / ne;
        const int re = rows[b0 + slot];
        rel = re & 31;
        t = reinterpret_cast<const int4*>(tabs + (size_t)(re >> 5) * row_bytes)[1 + idx - slot * ne];
      }
      const bool match = idx < total && t.y == rel;
      const uint64_t bal = __ballot(match);
      const int before = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) s_wcnt[wave] = __popcll(bal);
      __syncthreads();
      int off = s_ntaps;
      for (int w2 = 0; w2 < wave; ++w2) off += s_wcnt[w2];
      if (match) {
        const int o = t.x < half_w ? t.x : t.x - n;   // tap offset in [-W/2, W/2)
        // the table holds conj(w) c; the adjoint applies w c
        taps[off + before] = make_int4(slot * width + half_w - o, t.z, __float_as_int(-__int_as_float(t.w)), 0);
      }
      __syncthreads();
      if (tid == 0) {
        int sum = 0;
        for (int w2 = 0; w2 < kAdjWaves; ++w2) sum += s_wcnt[w2];
        s_ntaps += sum;
      }
      __syncthreads();
    }
    const int ntaps = s_ntaps;
    // the batch's taps applied to each tile: stage the rows' gradient columns, then accumulate
#pragma unroll
    for (int tt = 0; tt < kAdjTilesPer; ++tt) {
      const int tile = tile0 + tt;
      if (tile >= tiles) break;   // block-uniform
      const int n0 = tile * kAdjTile;
      for (int slot = 0; slot < cnt; ++slot) {
        const float2* grow = grad_image + (size_t)(rows[b0 + slot] >> 5) * n;
        for (int i = tid; i < width; i += kAdjThreads) stage[slot * width + i] = grow[(n0 - half_w + i + n) % n];
      }
      __syncthreads();
      // Taps in groups of kAdjU: a group's samples are requested before its multiply-adds.
      // Pulses past N accumulate values that are never stored; their stage reads stay inside
      // the slot (t.x + tid + p * kAdjThreads < (slot + 1) * width for any offset in the window).
      int e = 0;
      for (; e + kAdjU <= ntaps; e += kAdjU) {
        int4 t[kAdjU];
        float2 gv[kAdjU][kAdjP];
#pragma unroll
        for (int u = 0; u < kAdjU; ++u) {
          t[u] = taps[e + u];
#pragma unroll
          for (int p = 0; p < kAdjP; ++p) gv[u][p] = stage[t[u].x + tid + p * kAdjThreads];
        }
#pragma unroll
        for (int u = 0; u < kAdjU; ++u) {
          const float cx = __int_as_float(t[u].y), cy = __int_as_float(t[u].z);
#pragma unroll
          for (int p = 0; p < kAdjP; ++p) {
            acc[tt][p].x = fmaf(cx, gv[u][p].x, fmaf(-cy, gv[u][p].y, acc[tt][p].x));
            acc[tt][p].y = fmaf(cx, gv[u][p].y, fmaf(cy, gv[u][p].x, acc[tt][p].y));
          }
        }
      }
      for (; e < ntaps; ++e) {
        const int4 t = taps[e];
        const float cx = __int_as_float(t.y), cy = __int_as_float(t.z);
#pragma unroll
        for (int p = 0; p < kAdjP; ++p) {
          const float2 gv = stage[t.x + tid + p * kAdjThreads];
          acc[tt][p].x = fmaf(cx, gv.x, fmaf(-cy, gv.y, acc[tt][p].x));
          acc[tt][p].y = fmaf(cx, gv.y, fmaf(cy, gv.x, acc[tt][p].y));
        }
      }
      __syncthreads();   // the next tile or batch overwrites the stage (and the taps and list)
    }
  }
  float2* out = grad_band + (size_t)l * n;
#pragma unroll
  for (int tt = 0; tt < kAdjTilesPer; ++tt) {
#pragma unroll
    for (int p = 0; p < kAdjP; ++p) {
      const int np = (tile0 + tt) * kAdjTile + tid + p * kAdjThreads;
      if (tile0 + tt < tiles && np < n) out[np] = acc[tt][p];
    }
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
  hipError_t e = launch_fc_tables(a, L, tabs, bad, nullptr, s);
  if (e != hipSuccess) return e;
  const int tiles = (a.g.n + kAdjTile - 1) / kAdjTile;
  const int half_w = a.window / 2;
  const size_t mask_bytes = (size_t)rows_words(a.g.n_range) * sizeof(uint32_t);
  const size_t per_row = (size_t)(kAdjTile + 2 * half_w + 1) * sizeof(float2) + (size_t)L.ne * sizeof(int4);
  const size_t list_bytes = (size_t)list_words(a.g.n_range) * sizeof(int);
  const int cap = list_bytes >= kAdjLdsBudget ? 0 : (int)std::min<size_t>(kAdjMaxRows, (kAdjLdsBudget - list_bytes) / per_row);
  if (cap >= 1) {
    const int groups = (tiles + kAdjTilesPer - 1) / kAdjTilesPer;
    adjoint_band_staged_kernel<<<a.y.l_count * groups, kAdjThreads, list_bytes + (size_t)cap * per_row, s>>>(
        a.g.n, a.g.n_range, tiles, groups, half_w, cap, L.ne, tabs, L.row_bytes, grad_image, grad_band);
  } else {
    adjoint_band_kernel<<<a.y.l_count * tiles, kAdjThreads, mask_bytes, s>>>(a.g.n, a.g.n_range, tiles, tabs,
                                                                             L.row_bytes, grad_image, grad_band);
  }
  return hipGetLastError();
}

}  // namespace rosar
