// Offline robust sparse-array synthesis: Algorithm 1 (FPP-SCA) for every range bin of a polar
// grid, one workgroup per bin, all iterations in one launch.
//
// Per bin R (Sec. III-A/B): the candidates are the phase centres that see a target at the
// bin's azimuth (eqs. 4-5), offsets o in [-h, h] with R cos(o 2 pi / N) > r; the steering
// vector of a direction phi (from the target's azimuth) has elements
// a_k(phi) = cos(theta'_k) exp(+j 2 k R(phi - D_k)), D_k = o_k 2 pi / N (eq. 16); the main lobe
// is phi = 0 and the side-lobe directions are spaced by the sampled angle interval over
// [D_min, -phi_MW] and [phi_MW, D_max].  Starting from w_(0) = 1/sqrt(n), U'_(0) = |w_(0)^H a_m|,
// every iteration solves the convex sub-problem of eq. 36 (l1 norm + lambda_b (b + b1 + b2)
// under the linearised C1, C2, C4 of eqs. 33-35, C3, C5, b, b1, b2 >= 0) around the previous
// iterate, by the barrier method: damped Newton steps on tau f0 + phi(x) with a backtracking
// line search, tau multiplied by mu after each centring until m / tau < eps.  |w_k| <= t_k is a
// second-order cone with the barrier -log(t_k^2 - |w_k|^2).
//
// Newton system: the epigraph variables t couple only with their own (Re w_k, Im w_k), so they
// are eliminated per cone (a 2 x 2 Schur update); the reduced system over
// y = [Re w, Im w, U', b, b1, b2] (ny = 2n + 4) is assembled in float64 in global memory,
// factored by a blocked Cholesky (32-column panels, the trailing updates on the matrix cores)
// and solved by forward and backward substitution.  The side-lobe terms are a rank-3S update G G^T: the columns of G
// (2n x 3S, written once per Newton step) are sqrt(2/(-f_s)) times the real forms of a_s and
// j a_s and 2/|f_s| times that of a_s (a_s^H w); G G^T runs on the float64 matrix cores
// (16 x 16 x 4 MFMA), 64 x 64 output blocks per pass, 32 columns of G staged in LDS at a time
// while the next 32 are loaded.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rosar_device.hpp"

namespace rosar {
namespace {

constexpr int kSasThreads = 256;
constexpr int kSasWaves = kSasThreads / kWave;
constexpr int kMB = 64;            // G G^T output block (rows and columns) per pass
constexpr int kKC = 32;            // columns of G staged in LDS per step (eight MFMA k-steps)
constexpr int kCP = 32;            // Cholesky panel width

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Rows of G (2n, padded to whole output blocks) and columns (3S, padded to whole stages).
__host__ __device__ inline int g_rows(int n) { return (2 * n + kMB - 1) / kMB * kMB; }
__host__ __device__ inline int g_cols(int s) { return (3 * s + kKC - 1) / kKC * kKC; }

struct SasBuffers {
  double2* a_s;     // [s_max][n_max]
  double2* a_m;     // [n_max]
  double2* g;       // [n_max]  a_m (a_m^H w_i)
  double2* wi;      // [n_max]  linearisation point
  double2* z;       // [s_max]  a_s^H w
  double* fs;       // [s_max]  C2 values
  double* x;        // [3 n_max + 4]
  double* xt;       // [3 n_max + 4] line-search trial point
  double* dx;       // [3 n_max + 4]
  double* grad;     // [3 n_max + 4]
  double* rhs;      // [2 n_max + 4]
  double* H;        // [ny_max][ny_max]
  double2* cs;      // [s_max]  (sqrt(2/(-f_s)), 2/|f_s|)
  double* G;        // [g_cols(s_max)][g_rows(n_max)]  side-lobe factor, column-major
};

__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

__host__ __device__ inline size_t bin_bytes(int n_max, int s_max) {
  const size_t nv = 3 * (size_t)n_max + 4, ny = 2 * (size_t)n_max + 4;
  return align256((size_t)s_max * n_max * 16) + 3 * align256((size_t)n_max * 16) + align256((size_t)s_max * 16) +
         align256((size_t)s_max * 8) + 4 * align256(nv * 8) + align256(ny * 8) + align256(ny * ny * 8) +
         align256((size_t)s_max * 16) + align256((size_t)g_cols(s_max) * g_rows(n_max) * 8);
}

__device__ inline SasBuffers carve(char* base, int n_max, int s_max) {
  const size_t nv = 3 * (size_t)n_max + 4, ny = 2 * (size_t)n_max + 4;
  SasBuffers b;
  char* p = base;
  auto take = [&p](size_t bytes) {
    char* q = p;
    p += align256(bytes);
    return q;
  };
  b.a_s = reinterpret_cast<double2*>(take((size_t)s_max * n_max * 16));
  b.a_m = reinterpret_cast<double2*>(take((size_t)n_max * 16));
  b.g = reinterpret_cast<double2*>(take((size_t)n_max * 16));
  b.wi = reinterpret_cast<double2*>(take((size_t)n_max * 16));
  b.z = reinterpret_cast<double2*>(take((size_t)s_max * 16));
  b.fs = reinterpret_cast<double*>(take((size_t)s_max * 8));
  b.x = reinterpret_cast<double*>(take(nv * 8));
  b.xt = reinterpret_cast<double*>(take(nv * 8));
  b.dx = reinterpret_cast<double*>(take(nv * 8));
  b.grad = reinterpret_cast<double*>(take(nv * 8));
  b.rhs = reinterpret_cast<double*>(take(ny * 8));
  b.H = reinterpret_cast<double*>(take(ny * ny * 8));
  b.cs = reinterpret_cast<double2*>(take((size_t)s_max * 16));
  b.G = reinterpret_cast<double*>(take((size_t)g_cols(s_max) * g_rows(n_max) * 8));
  return b;
}

// ---------------------------------------------------------------- workgroup reductions
// Deterministic: per-thread partials combined by wave shuffles, then the waves in order.
__device__ inline double block_sum(double v, double* red) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kSasWaves; ++w) s += red[w];
  return s;
}

__device__ inline double block_max(double v, double* red) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < kSasWaves; ++w) s = fmax(s, red[w]);
  return s;
}

__device__ inline double2 cmul_conj_a(double2 a, double2 w) {   // conj(a) * w
  return make_double2(a.x * w.x + a.y * w.y, a.x * w.y - a.y * w.x);
}

// z_s = a_s^H w for every side-lobe row: one wave per row, lanes over the candidates.
__device__ void side_products(const SasBuffers& B, const double* x, int n, int n_max, int s_cnt) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int s = wave; s < s_cnt; s += kSasWaves) {
    const double2* row = B.a_s + (size_t)s * n_max;
    double zr = 0.0, zi = 0.0;
    for (int k = lane; k < n; k += kWave) {
      const double2 p = cmul_conj_a(row[k], make_double2(x[k], x[n + k]));
      zr += p.x;
      zi += p.y;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
      zr += __shfl_xor(zr, off);
      zi += __shfl_xor(zi, off);
    }
    if (lane == 0) B.z[s] = make_double2(zr, zi);
  }
  __syncthreads();
}

struct SubConst {
  double c1, alpha, beta, c4, delta, umin, lam;
};

// tau f0 + phi(x) of eq. 36's barrier problem at x (z of x computed first), or +inf outside the
// domain.  Also leaves f_s in B.fs.  All threads return the same value.
__device__ double barrier_value(const SasBuffers& B, const double* x, int n, int n_max, int s_cnt, const SubConst& c,
                                double tau, double* red) {
  side_products(B, x, n, n_max, s_cnt);
  const double u = x[3 * n], b = x[3 * n + 1], b1 = x[3 * n + 2], b2 = x[3 * n + 3];
  double acc = 0.0, bad = 0.0;
  // cones and the sums over w
  double sum_t = 0.0, ww = 0.0, gw = 0.0, wiw = 0.0;
  for (int k = threadIdx.x; k < n; k += kSasThreads) {
    const double wr = x[k], wim = x[n + k], t = x[2 * n + k];
    const double uu = t * t - (wr * wr + wim * wim);
    if (!(uu > 0.0) || !(t > 0.0)) bad = 1.0;
    else acc -= log(uu);
    sum_t += t;
    ww += wr * wr + wim * wim;
    const double2 gk = B.g[k], wk = B.wi[k];
    gw += gk.x * wr + gk.y * wim;        // Re(g^H w)
    wiw += wk.x * wr + wk.y * wim;       // Re(w_i^H w)
  }
  for (int s = threadIdx.x; s < s_cnt; s += kSasThreads) {
    const double2 z = B.z[s];
    const double f = z.x * z.x + z.y * z.y + c.alpha * u + c.beta - b2;
    B.fs[s] = f;
    if (!(f < 0.0)) bad = 1.0;
    else acc -= log(-f);
  }
  bad = block_max(bad, red);
  acc = block_sum(acc, red);
  sum_t = block_sum(sum_t, red);
  ww = block_sum(ww, red);
  gw = block_sum(gw, red);
  wiw = block_sum(wiw, red);
  const double f1 = (u + c.delta) * (u + c.delta) + c.c1 - 2.0 * gw - b1;
  const double f3 = ww - 1.0 - b;
  const double f4 = c.c4 - b - 2.0 * wiw;
  const double f5 = c.umin - u;
  if (bad > 0.0 || !(f1 < 0.0) || !(f3 < 0.0) || !(f4 < 0.0) || !(f5 < 0.0) || !(b > 0.0) || !(b1 > 0.0) ||
      !(b2 > 0.0))
    return INFINITY;
  return tau * (sum_t + c.lam * (b + b1 + b2)) + acc - log(-f1) - log(-f3) - log(-f4) - log(-f5) - log(b) - log(b1) -
         log(b2);
}

// Gradient of tau f0 + phi at x (B.fs, B.z of x must be current) into B.grad, and the reduced
// Hessian over y = [Re w, Im w, U', b, b1, b2] (lower triangle) into B.H.  The t-gradient and
// the cone's t-couplings are folded in by the per-cone Schur update; B.rhs gets -(reduced
// gradient).
__device__ void assemble(const SasBuffers& B, const double* x, int n, int n_max, int s_cnt, const SubConst& c,
                         double tau, double* red, double* lds) {
  const int ny = 2 * n + 4;
  const int iu = 2 * n, ib = 2 * n + 1, ib1 = 2 * n + 2, ib2 = 2 * n + 3;   // reduced indices
  const double u = x[3 * n], b = x[3 * n + 1], b1 = x[3 * n + 2], b2 = x[3 * n + 3];
  // scalar constraint values
  double ww = 0.0, gw = 0.0, wiw = 0.0;
  for (int k = threadIdx.x; k < n; k += kSasThreads) {
    const double wr = x[k], wim = x[n + k];
    ww += wr * wr + wim * wim;
    gw += B.g[k].x * wr + B.g[k].y * wim;
    wiw += B.wi[k].x * wr + B.wi[k].y * wim;
  }
  ww = block_sum(ww, red);
  gw = block_sum(gw, red);
  wiw = block_sum(wiw, red);
  const double f1 = (u + c.delta) * (u + c.delta) + c.c1 - 2.0 * gw - b1;
  const double f3 = ww - 1.0 - b;
  const double f4 = c.c4 - b - 2.0 * wiw;
  const double f5 = c.umin - u;
  // side-lobe sums for the border rows: sum 1/(-f), alpha-weighted, and 1/f^2
  double s_inv = 0.0, s_inv2 = 0.0;
  for (int s = threadIdx.x; s < s_cnt; s += kSasThreads) {
    const double f = B.fs[s];
    s_inv += 1.0 / (-f);
    s_inv2 += 1.0 / (f * f);
  }
  s_inv = block_sum(s_inv, red);
  s_inv2 = block_sum(s_inv2, red);

  // ---- gradient (full vector, t included)
  // w: cones 2w/u; C1 -2 g/(-f1); C2 sum_s 2 a_s z_s / (-f_s); C3 2 w/(-f3); C4 -2 w_i/(-f4)
  for (int k = threadIdx.x; k < n; k += kSasThreads) {
    const double wr = x[k], wim = x[n + k], t = x[2 * n + k];
    const double uu = t * t - (wr * wr + wim * wim);
    double gr = 2.0 * wr / uu - 2.0 * B.g[k].x / (-f1) + 2.0 * wr / (-f3) - 2.0 * B.wi[k].x / (-f4);
    double gi = 2.0 * wim / uu - 2.0 * B.g[k].y / (-f1) + 2.0 * wim / (-f3) - 2.0 * B.wi[k].y / (-f4);
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < s_cnt; ++s) {
      const double2 a = B.a_s[(size_t)s * n_max + k];
      const double2 z = B.z[s];
      const double cf = 2.0 / (-B.fs[s]);
      // a z
      sr += cf * (a.x * z.x - a.y * z.y);
      si += cf * (a.x * z.y + a.y * z.x);
    }
    B.grad[k] = gr + sr;
    B.grad[n + k] = gi + si;
    B.grad[2 * n + k] = tau - 2.0 * t / uu;
  }
  if (threadIdx.x == 0) {
    B.grad[3 * n] = 2.0 * (u + c.delta) / (-f1) + c.alpha * s_inv - 1.0 / (-f5);
    B.grad[3 * n + 1] = tau * c.lam - 1.0 / (-f3) - 1.0 / (-f4) - 1.0 / b;
    B.grad[3 * n + 2] = tau * c.lam - 1.0 / (-f1) - 1.0 / b1;
    B.grad[3 * n + 3] = tau * c.lam - s_inv - 1.0 / b2;
  }
  __syncthreads();

  // ---- Hessian, w-w block: sum_s [c_s (P P^T + Q Q^T) + d_s V V^T] = G G^T
  // (P = (Re a, Im a), Q = (-Im a, Re a), V = (Re(a z), Im(a z)), c = 2/(-f), d = 4/f^2)
  const int nw = 2 * n;
  for (int si = threadIdx.x; si < s_cnt; si += kSasThreads) {
    const double f = B.fs[si];
    B.cs[si] = make_double2(sqrt(2.0 / (-f)), 2.0 / fabs(f));
  }
  __syncthreads();
  const int gr = g_rows(n_max), gc = g_cols(s_cnt);
  for (int c = 0; c < gc; ++c) {
    const int si = c / 3, t = c - 3 * si;
    for (int row = threadIdx.x; row < gr; row += kSasThreads) {
      double v = 0.0;
      if (row < nw && si < s_cnt) {
        const int k = row < n ? row : row - n;
        const double2 a = B.a_s[(size_t)si * n_max + k];
        const double2 sc = B.cs[si];
        if (t == 0) {
          v = sc.x * (row < n ? a.x : a.y);
        } else if (t == 1) {
          v = sc.x * (row < n ? -a.y : a.x);
        } else {
          const double2 z = B.z[si];
          v = sc.y * (row < n ? a.x * z.x - a.y * z.y : a.x * z.y + a.y * z.x);
        }
      }
      B.G[(size_t)c * gr + row] = v;
    }
  }
  __syncthreads();
  {
    // G G^T on the matrix cores: per 64 x 64 block of the lower triangle, wave w owns block
    // rows [16 w, 16 w + 16) and four 16-column tiles.  v_mfma_f64_16x16x4f64 lane l takes
    // A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16] in register r.
    double* sI = lds;                 // [kKC][kMB] block rows' columns of G
    double* sJ = lds + kKC * kMB;     // [kKC][kMB] block columns'
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int nb = (nw + kMB - 1) / kMB;
    constexpr int kPer = 2 * kKC * kMB / kSasThreads;   // staged entries per thread
    for (int bi = 0; bi < nb; ++bi) {
      for (int bj = 0; bj <= bi; ++bj) {
        dbl4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
        double pre[kPer];
        auto fetch = [&](int k0) {
#pragma unroll
          for (int m = 0; m < kPer; ++m) {
            const int e = threadIdx.x + kSasThreads * m;
            const int side = e / (kKC * kMB), rem = e % (kKC * kMB);
            const int c = rem / kMB, r = rem % kMB;
            pre[m] = B.G[(size_t)(k0 + c) * gr + (side ? bj : bi) * kMB + r];
          }
        };
        fetch(0);
        for (int k0 = 0; k0 < gc; k0 += kKC) {
          __syncthreads();
#pragma unroll
          for (int m = 0; m < kPer; ++m) {
            const int e = threadIdx.x + kSasThreads * m;
            const int side = e / (kKC * kMB), rem = e % (kKC * kMB);
            (side ? sJ : sI)[rem] = pre[m];
          }
          __syncthreads();
          if (k0 + kKC < gc) fetch(k0 + kKC);
#pragma unroll
          for (int kk = 0; kk < kKC; kk += 4) {
            const double a = sI[(kk + lane / 16) * kMB + wave * 16 + lane % 16];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const double b = sJ[(kk + lane / 16) * kMB + t * 16 + lane % 16];
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = bi * kMB + wave * 16 + lane / 16 + 4 * r;
            const int j = bj * kMB + t * 16 + lane % 16;
            if (i < nw && j <= i) B.H[(size_t)i * ny + j] = acc[t][r];
          }
      }
    }
  }
  __syncthreads();
  // rank-1 terms of C1, C3, C4 and the C3 diagonal, the cones' reduced 2 x 2 blocks
  const double i1 = 1.0 / (f1 * f1), i3 = 1.0 / (f3 * f3), i4 = 1.0 / (f4 * f4);
  for (int e = threadIdx.x; e < nw * nw; e += kSasThreads) {
    const int i = e / nw, j = e % nw;
    if (j > i) continue;
    const int ki = i < n ? i : i - n, kj = j < n ? j : j - n;
    // gradients in w of f1, f3, f4 at components i, j
    const double g1i = -2.0 * (i < n ? B.g[ki].x : B.g[ki].y), g1j = -2.0 * (j < n ? B.g[kj].x : B.g[kj].y);
    const double g3i = 2.0 * x[i], g3j = 2.0 * x[j];
    const double g4i = -2.0 * (i < n ? B.wi[ki].x : B.wi[ki].y), g4j = -2.0 * (j < n ? B.wi[kj].x : B.wi[kj].y);
    double h = B.H[(size_t)i * ny + j] + g1i * g1j * i1 + g3i * g3j * i3 + g4i * g4j * i4;
    if (i == j) h += 2.0 / (-f3);
    if (ki == kj) {
      // cone k: reduced block diag(2,2)/u + 4 w w^T / u^2 - (h_wt h_wt^T) / h_tt
      const int k = ki;
      const double wr = x[k], wim = x[n + k], t = x[2 * n + k];
      const double uu = t * t - (wr * wr + wim * wim);
      const double wa = i < n ? wr : wim, wb = j < n ? wr : wim;
      const double htt = -2.0 / uu + 4.0 * t * t / (uu * uu);
      const double hat = -4.0 * wa * t / (uu * uu), hbt = -4.0 * wb * t / (uu * uu);
      h += (i == j ? 2.0 / uu : 0.0) + 4.0 * wa * wb / (uu * uu) - hat * hbt / htt;
    }
    B.H[(size_t)i * ny + j] = h;
  }
  // border rows: U', b, b1, b2 against w, and among themselves
  for (int j = threadIdx.x; j < nw; j += kSasThreads) {
    const int kj = j < n ? j : j - n;
    double hu = 0.0, hb2 = 0.0;
    for (int s = 0; s < s_cnt; ++s) {
      const double2 a = B.a_s[(size_t)s * n_max + kj];
      const double2 z = B.z[s];
      const double v = j < n ? a.x * z.x - a.y * z.y : a.x * z.y + a.y * z.x;
      const double f = B.fs[s];
      hu += 2.0 * v * c.alpha / (f * f);
      hb2 += -2.0 * v / (f * f);
    }
    const double g1 = -2.0 * (j < n ? B.g[kj].x : B.g[kj].y);
    const double g3 = 2.0 * x[j];
    const double g4 = -2.0 * (j < n ? B.wi[kj].x : B.wi[kj].y);
    B.H[(size_t)iu * ny + j] = hu + g1 * 2.0 * (u + c.delta) * i1;
    B.H[(size_t)ib * ny + j] = -g3 * i3 - g4 * i4;
    B.H[(size_t)ib1 * ny + j] = -g1 * i1;
    B.H[(size_t)ib2 * ny + j] = hb2;
  }
  if (threadIdx.x == 0) {
    double s_a2 = c.alpha * c.alpha * s_inv2;
    B.H[(size_t)iu * ny + iu] = 4.0 * (u + c.delta) * (u + c.delta) * i1 + 2.0 / (-f1) + s_a2 + 1.0 / (f5 * f5);
    B.H[(size_t)ib * ny + iu] = 0.0;
    B.H[(size_t)ib1 * ny + iu] = -2.0 * (u + c.delta) * i1;
    B.H[(size_t)ib2 * ny + iu] = -c.alpha * s_inv2;
    B.H[(size_t)ib * ny + ib] = i3 + i4 + 1.0 / (b * b);
    B.H[(size_t)ib1 * ny + ib] = 0.0;
    B.H[(size_t)ib2 * ny + ib] = 0.0;
    B.H[(size_t)ib1 * ny + ib1] = i1 + 1.0 / (b1 * b1);
    B.H[(size_t)ib2 * ny + ib1] = 0.0;
    B.H[(size_t)ib2 * ny + ib2] = s_inv2 + 1.0 / (b2 * b2);
  }
  // reduced right-hand side -(g_y - h_yt g_t / h_tt)
  for (int i = threadIdx.x; i < ny; i += kSasThreads) {
    double gy;
    if (i < nw) {
      const int k = i < n ? i : i - n;
      const double wr = x[k], wim = x[n + k], t = x[2 * n + k];
      const double uu = t * t - (wr * wr + wim * wim);
      const double wa = i < n ? wr : wim;
      const double htt = -2.0 / uu + 4.0 * t * t / (uu * uu);
      const double hat = -4.0 * wa * t / (uu * uu);
      gy = B.grad[i] - hat * B.grad[2 * n + k] / htt;
    } else {
      gy = B.grad[3 * n + (i - nw)];
    }
    B.rhs[i] = -gy;
  }
  __syncthreads();
}

// In-place Cholesky of the lower triangle of H (ny x ny, row stride ny), right-looking with
// kCP-column panels: the diagonal block is factored in LDS column by column by the whole
// workgroup, the panel below by forward substitution (one row per thread, held in LDS), and the trailing
// update A22 -= L21 L21^T runs on the float64 matrix cores over 64 x 64 blocks of the lower
// triangle (the panel's 32 columns of the block rows and columns staged in LDS).  Returns false
// (all threads) if a pivot is not positive.
__device__ bool cholesky(double* H, int ny, double* lds, double* red) {
  (void)red;
  constexpr int LP = kCP + 1;              // padded row of the diagonal block
  constexpr int SL = kMB + 1;              // padded column of the staged panels
  double* L11 = lds;                       // [kCP][LP]
  double* dinv = L11 + kCP * LP;           // [kCP] 1 / L11[j][j]
  double* sI = dinv + kCP;                 // [kCP][SL] panel columns of the block rows
  double* sJ = sI + kCP * SL;              // [kCP][SL] panel columns of the block columns
  double* vL = sJ + kCP * SL;              // [kSasThreads][LP] one panel row per thread
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int k0 = 0; k0 < ny; k0 += kCP) {
    const int kb = min(kCP, ny - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < kCP * kCP; e += kSasThreads) {
      const int i = e / kCP, j = e % kCP;
      L11[i * LP + j] = (i < kb && j <= i) ? H[(size_t)(k0 + i) * ny + k0 + j] : 0.0;
    }
    __syncthreads();
    // the diagonal block, column by column (every thread reads the same pivots, so the
    // positivity test is uniform)
    for (int j = 0; j < kb; ++j) {
      const double d = L11[j * LP + j];
      if (!(d > 0.0)) return false;
      const double ljj = sqrt(d);
      __syncthreads();   // every thread has read the pivot
      for (int i = j + 1 + (int)threadIdx.x; i < kb; i += kSasThreads) L11[i * LP + j] /= ljj;
      if (threadIdx.x == 0) {
        L11[j * LP + j] = ljj;
        dinv[j] = 1.0 / ljj;
      }
      __syncthreads();
      const int rem = kb - j - 1;
      for (int e = threadIdx.x; e < rem * rem; e += kSasThreads) {
        const int i = j + 1 + e / rem, m = j + 1 + e % rem;
        if (m <= i) L11[i * LP + m] -= L11[i * LP + j] * L11[m * LP + j];
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < kb * kb; e += kSasThreads) {
      const int i = e / kb, j = e % kb;
      if (j <= i) H[(size_t)(k0 + i) * ny + k0 + j] = L11[i * LP + j];
    }
    // panel below: L21 = A21 L11^{-T}, one row per thread, the row held in LDS
    const int rows = ny - k0 - kb;
    double* vr = vL + threadIdx.x * LP;
    for (int r = threadIdx.x; r < rows; r += kSasThreads) {
      double* hrow = H + (size_t)(k0 + kb + r) * ny + k0;
      for (int j = 0; j < kb; ++j) vr[j] = hrow[j];
      for (int j = 0; j < kb; ++j) {
        double sum = vr[j];
        for (int q = 0; q < j; ++q) sum -= vr[q] * L11[j * LP + q];
        vr[j] = sum * dinv[j];
      }
      for (int j = 0; j < kb; ++j) hrow[j] = vr[j];
    }
    __syncthreads();
    // trailing update A22 -= L21 L21^T on the matrix cores (lane layout as in the assembly)
    const int base = k0 + kb;
    const int nb = (rows + kMB - 1) / kMB;
    for (int bi = 0; bi < nb; ++bi) {
      for (int bj = 0; bj <= bi; ++bj) {
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * kMB * kCP; e += kSasThreads) {
          const int side = e / (kMB * kCP), rem = e % (kMB * kCP);
          const int r = rem / kCP, c = rem % kCP;
          const int row = (side ? bj : bi) * kMB + r;
          const double v = (row < rows && c < kb) ? H[(size_t)(base + row) * ny + k0 + c] : 0.0;
          (side ? sJ : sI)[c * SL + r] = v;
        }
        __syncthreads();
        dbl4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = bi * kMB + wave * 16 + lane / 16 + 4 * q;
            const int j = bj * kMB + t * 16 + lane % 16;
            acc[t][q] = (i < rows && j <= i) ? H[(size_t)(base + i) * ny + base + j] : 0.0;
          }
#pragma unroll
        for (int kk = 0; kk < kCP; kk += 4) {
          const double a = -sI[(kk + lane / 16) * SL + wave * 16 + lane % 16];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double b = sJ[(kk + lane / 16) * SL + t * 16 + lane % 16];
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = bi * kMB + wave * 16 + lane / 16 + 4 * q;
            const int j = bj * kMB + t * 16 + lane % 16;
            if (i < rows && j <= i) H[(size_t)(base + i) * ny + base + j] = acc[t][q];
          }
      }
    }
  }
  __syncthreads();
  return true;
}

// Solves L L^T y = rhs in place (L in the lower triangle of H).
__device__ void chol_solve(const double* H, int ny, double* rhs) {
  for (int k = 0; k < ny; ++k) {
    __syncthreads();
    const double yk = rhs[k] / H[(size_t)k * ny + k];
    __syncthreads();
    if (threadIdx.x == 0) rhs[k] = yk;
    for (int i = k + 1 + threadIdx.x; i < ny; i += kSasThreads) rhs[i] -= H[(size_t)i * ny + k] * yk;
  }
  for (int k = ny - 1; k >= 0; --k) {
    __syncthreads();
    const double xk = rhs[k] / H[(size_t)k * ny + k];
    __syncthreads();
    if (threadIdx.x == 0) rhs[k] = xk;
    for (int i = threadIdx.x; i < k; i += kSasThreads) rhs[i] -= H[(size_t)k * ny + i] * xk;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSasThreads) void sas_design_kernel(Geo g, SasDesignParams p, const double* __restrict__ delta_r,
                                                                 int n_max, int s_max, size_t stride, char* __restrict__ ws,
                                                                 int32_t window, int32_t* __restrict__ offsets,
                                                                 float2* __restrict__ weights, int32_t* __restrict__ count,
                                                                 double* __restrict__ hist) {
  __shared__ double red[kSasWaves];
  constexpr int kAsmLds = 2 * kKC * kMB;
  constexpr int kCholLds = kCP * (kCP + 1) + kCP + 2 * kCP * (kMB + 1) + kSasThreads * (kCP + 1);
  __shared__ double lds[kAsmLds > kCholLds ? kAsmLds : kCholLds];
  const int bin = blockIdx.x;
  const SasBuffers B = carve(ws + (size_t)bin * stride, n_max, s_max);
  const double rr = g.r0 + bin * g.dr;
  const double r = g.radius;
  const int nn = g.n;
  // candidates o in [-h, h]: R cos(o 2 pi / N) - r > 0 (eqs. 4-5)
  int h = 0;
  while (h + 1 <= nn / 2 && rr * cos((double)(h + 1) * kTwoPiD / (double)nn) - r > 0.0) ++h;
  const bool any = rr * cos(0.0) - r > 0.0;
  const int n = any ? 2 * h + 1 : 0;
  double* hist_bin = hist ? hist + (size_t)bin * p.iters * 6 : nullptr;
  // side-lobe directions: [D_min, -phi_MW] and [phi_MW, D_max] at the sampled interval
  const double d_min = (double)(-h) * kTwoPiD / (double)nn, d_max = (double)h * kTwoPiD / (double)nn;
  const int n_left = max((int)floor((-p.phi_mw - d_min) / p.d_angle) + 1, 0);
  const int n_right = max((int)floor((d_max - p.phi_mw) / p.d_angle) + 1, 0);
  const int s_cnt = n_left + n_right;
  if (n == 0 || n > n_max || s_cnt > s_max) {
    // no phase centre sees the row (R <= r): no taps and an all-zero history
    for (int k = threadIdx.x; k < window; k += kSasThreads) {
      offsets[(size_t)bin * window + k] = 0;
      weights[(size_t)bin * window + k] = make_float2(0.f, 0.f);
    }
    if (hist_bin)
      for (int e = threadIdx.x; e < p.iters * 6; e += kSasThreads) hist_bin[e] = 0.0;
    if (threadIdx.x == 0) count[bin] = 0;
    return;
  }
  const double step = kTwoPiD / (double)nn;
  // steering vectors (eq. 16): a_k(phi) = alpha exp(+j 2 k R(phi - D_k))
  for (int e = threadIdx.x; e < (s_cnt + 1) * n; e += kSasThreads) {
    const int s = e / n, k = e % n;
    double phi;
    if (s == s_cnt) phi = 0.0;
    else if (s < n_left) phi = -p.phi_mw - p.d_angle * (double)(n_left - 1 - s);
    else phi = p.phi_mw + p.d_angle * (double)(s - n_left);
    const double d = phi - (double)(k - h) * step;
    const double rn = sqrt(rr * rr + r * r - 2.0 * rr * r * cos(d));
    const double al = fmax(rr * cos(d) - r, 0.0) / rn;
    double sn, cs;
    sincos(2.0 * g.kw * rn, &sn, &cs);
    const double2 a = make_double2(al * cs, al * sn);
    if (s == s_cnt) B.a_m[k] = a;
    else B.a_s[(size_t)s * n_max + k] = a;
  }
  __syncthreads();
  // w_(0) = 1/sqrt(n), U'_(0) = |w_(0)^H a_m|
  const double w0 = 1.0 / sqrt((double)n);
  for (int k = threadIdx.x; k < n; k += kSasThreads) B.wi[k] = make_double2(w0, 0.0);
  double zr = 0.0, zi = 0.0;
  for (int k = threadIdx.x; k < n; k += kSasThreads) {
    zr += w0 * B.a_m[k].x;
    zi += w0 * B.a_m[k].y;
  }
  zr = block_sum(zr, red);
  zi = block_sum(zi, red);
  double u_i = sqrt(zr * zr + zi * zi);
  const double delta = delta_r[bin];
  const int nv = 3 * n + 4;
  const int ny = 2 * n + 4;
  const int m_deg = 2 * n + s_cnt + 7;
  const double se = sqrt(p.eta);
  const double umin = sqrt(p.u_min);
  double slack = 0.0;
  for (int it = 0; it < p.iters; ++it) {
    // linearisation at (w_i, U'_i): g = a_m (a_m^H w_i), c1 = |a_m^H w_i|^2 (eq. 33), alpha and
    // beta of eq. 34, c4 = 1 + ||w_i||^2 (eq. 35)
    double mr = 0.0, mi = 0.0, wn = 0.0;
    for (int k = threadIdx.x; k < n; k += kSasThreads) {
      const double2 pk = cmul_conj_a(B.a_m[k], B.wi[k]);
      mr += pk.x;
      mi += pk.y;
      wn += B.wi[k].x * B.wi[k].x + B.wi[k].y * B.wi[k].y;
    }
    mr = block_sum(mr, red);
    mi = block_sum(mi, red);
    wn = block_sum(wn, red);
    for (int k = threadIdx.x; k < n; k += kSasThreads) {
      const double2 a = B.a_m[k];
      B.g[k] = make_double2(a.x * mr - a.y * mi, a.x * mi + a.y * mr);
    }
    SubConst c;
    c.c1 = mr * mr + mi * mi;
    c.alpha = 2.0 * (se * delta - p.eta * u_i);
    c.beta = p.eta * u_i * u_i - delta * delta;
    c.c4 = 1.0 + wn;
    c.delta = delta;
    c.umin = umin;
    c.lam = p.lam_b;
    // strictly feasible start: w = w_i, t = |w_i| + 1, U' = U'_i (or U'_min + 1), slacks one
    // above the largest violation of what they relax
    for (int k = threadIdx.x; k < n; k += kSasThreads) {
      const double2 w = B.wi[k];
      B.x[k] = w.x;
      B.x[n + k] = w.y;
      B.x[2 * n + k] = sqrt(w.x * w.x + w.y * w.y) + 1.0;
    }
    __syncthreads();
    const double u0 = u_i > umin + 1e-3 ? u_i : umin + 1.0;
    side_products(B, B.x, n, n_max, s_cnt);
    double f2max = -INFINITY;
    for (int s = threadIdx.x; s < s_cnt; s += kSasThreads) {
      const double2 z = B.z[s];
      f2max = fmax(f2max, z.x * z.x + z.y * z.y + c.alpha * u0 + c.beta);
    }
    f2max = block_max(f2max, red);
    // at w = w_i: ||w||^2 - 1 = wn - 1, c4 - 2 Re(w_i^H w_i) = 1 - wn, Re(g^H w_i) = c1
    if (threadIdx.x == 0) {
      B.x[3 * n] = u0;
      B.x[3 * n + 1] = fmax(fmax(wn - 1.0, 1.0 - wn), 0.0) + 1.0;
      B.x[3 * n + 2] = fmax((u0 + delta) * (u0 + delta) - c.c1, 0.0) + 1.0;
      B.x[3 * n + 3] = fmax(f2max, 0.0) + 1.0;
    }
    __syncthreads();
    double tau = p.tau0;
    int newton = 0;
    while (true) {
      for (int step_i = 0; step_i < p.max_newton; ++step_i) {
        const double val = barrier_value(B, B.x, n, n_max, s_cnt, c, tau, red);
        assemble(B, B.x, n, n_max, s_cnt, c, tau, red, lds);
        if (!cholesky(B.H, ny, lds, red)) break;
        chol_solve(B.H, ny, B.rhs);
        // dx over [w, U', b's] and the eliminated t
        for (int i = threadIdx.x; i < nv; i += kSasThreads) {
          double d;
          if (i < 2 * n) {
            d = B.rhs[i];
          } else if (i < 3 * n) {
            const int k = i - 2 * n;
            const double wr = B.x[k], wim = B.x[n + k], t = B.x[2 * n + k];
            const double uu = t * t - (wr * wr + wim * wim);
            const double htt = -2.0 / uu + 4.0 * t * t / (uu * uu);
            const double hrt = -4.0 * wr * t / (uu * uu), hit = -4.0 * wim * t / (uu * uu);
            d = -(B.grad[2 * n + k] + hrt * B.rhs[k] + hit * B.rhs[n + k]) / htt;
          } else {
            d = B.rhs[2 * n + (i - 3 * n)];
          }
          B.dx[i] = d;
        }
        __syncthreads();
        double gd = 0.0;
        for (int i = threadIdx.x; i < nv; i += kSasThreads) gd += B.grad[i] * B.dx[i];
        gd = block_sum(gd, red);
        if (-gd / 2.0 <= p.newton_tol) break;
        double s = 1.0;
        bool moved = false;
        while (s >= p.ls_min) {
          for (int i = threadIdx.x; i < nv; i += kSasThreads) B.xt[i] = B.x[i] + s * B.dx[i];
          __syncthreads();
          const double vt = barrier_value(B, B.xt, n, n_max, s_cnt, c, tau, red);
          if (vt <= val + p.ls_alpha * s * gd) {
            moved = true;
            break;
          }
          s *= p.ls_beta;
        }
        if (!moved) break;
        for (int i = threadIdx.x; i < nv; i += kSasThreads) B.x[i] = B.xt[i];
        __syncthreads();
        ++newton;
      }
      if ((double)m_deg / tau < p.eps) break;
      tau *= p.mu;
    }
    // the sub-problem's solution becomes the next linearisation point
    double ww = 0.0, l1 = 0.0;
    for (int k = threadIdx.x; k < n; k += kSasThreads) {
      const double wr = B.x[k], wim = B.x[n + k];
      B.wi[k] = make_double2(wr, wim);
      l1 += sqrt(wr * wr + wim * wim);
    }
    l1 = block_sum(l1, red);
    (void)ww;
    u_i = B.x[3 * n];
    const double bb = B.x[3 * n + 1], bb1 = B.x[3 * n + 2], bb2 = B.x[3 * n + 3];
    slack = bb + bb1 + bb2;
    if (hist_bin && threadIdx.x == 0) {
      double* hrec = hist_bin + (size_t)it * 6;
      hrec[0] = l1 + p.lam_b * slack;
      hrec[1] = u_i;
      hrec[2] = bb;
      hrec[3] = bb1;
      hrec[4] = bb2;
      hrec[5] = (double)newton;
    }
    __syncthreads();
  }
  // thresholding (|w_k| < Th set to zero) and the nonzero taps first, in candidate order
  if (threadIdx.x == 0) {
    int q = 0;
    for (int k = 0; k < n && q < window; ++k) {
      const double2 w = B.wi[k];
      if (sqrt(w.x * w.x + w.y * w.y) >= p.th) {
        offsets[(size_t)bin * window + q] = k - h;
        weights[(size_t)bin * window + q] = make_float2((float)w.x, (float)w.y);
        ++q;
      }
    }
    count[bin] = q;
    for (int k = q; k < window; ++k) {
      offsets[(size_t)bin * window + k] = 0;
      weights[(size_t)bin * window + k] = make_float2(0.f, 0.f);
    }
  }
}

}  // namespace

SasSizes sas_sizes(const Geo& g, const SasDesignParams& p) {
  SasSizes z{};
  for (int bin = 0; bin < g.n_range; ++bin) {
    const double rr = g.r0 + bin * g.dr;
    int h = 0;
    while (h + 1 <= g.n / 2 && rr * std::cos((double)(h + 1) * kTwoPiD / (double)g.n) - g.radius > 0.0) ++h;
    if (!(rr - g.radius > 0.0)) continue;
    const int n = 2 * h + 1;
    const double d_min = (double)(-h) * kTwoPiD / (double)g.n, d_max = (double)h * kTwoPiD / (double)g.n;
    const int s = std::max((int)std::floor((-p.phi_mw - d_min) / p.d_angle) + 1, 0) +
                  std::max((int)std::floor((d_max - p.phi_mw) / p.d_angle) + 1, 0);
    z.n_max = std::max(z.n_max, n);
    z.s_max = std::max(z.s_max, s);
  }
  z.stride = bin_bytes(std::max(z.n_max, 1), std::max(z.s_max, 1));
  z.bytes = z.stride * (size_t)g.n_range;
  return z;
}

hipError_t launch_sas_design(const Geo& g, const SasDesignParams& p, const double* delta_r, const SasSizes& z,
                             void* ws, int32_t window, int32_t* offsets, float2* weights, int32_t* count,
                             double* hist, hipStream_t s) {
  sas_design_kernel<<<g.n_range, kSasThreads, 0, s>>>(g, p, delta_r, std::max(z.n_max, 1), std::max(z.s_max, 1),
                                                       z.stride, reinterpret_cast<char*>(ws), window, offsets, weights,
                                                       count, hist);
  return hipGetLastError();
}

}  // namespace rosar
