// Device helpers for the gfx950 kernels: complex sample loads by storage type, revolutions-
// based sine/cosine, launch-order remapping for the 8 XCDs of an MI355X.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rosar_internal.hpp"

namespace rosar {

constexpr int kWave = 64;
constexpr int kXcds = 8;

// ---------------------------------------------------------------- complex storage types
// DT: 0 = complex float32, 1 = complex half, 2 = complex bfloat16 (rosar_dtype values).
template <int DT> struct Elem;
template <> struct Elem<0> { using T = float2;   static constexpr int bytes = 8; };
template <> struct Elem<1> { using T = uint32_t; static constexpr int bytes = 4; };
template <> struct Elem<2> { using T = uint32_t; static constexpr int bytes = 4; };

__device__ __forceinline__ float2 unpack_f16x2(uint32_t v) {
  __half2 h = *reinterpret_cast<__half2*>(&v);
  return __half22float2(h);
}

__device__ __forceinline__ float2 unpack_bf16x2(uint32_t v) {
  return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
}

template <int DT>
__device__ __forceinline__ float2 load_c(const void* base, int64_t idx) {
  if constexpr (DT == 0) {
    return reinterpret_cast<const float2*>(base)[idx];
  } else if constexpr (DT == 1) {
    return unpack_f16x2(reinterpret_cast<const uint32_t*>(base)[idx]);
  } else {
    return unpack_bf16x2(reinterpret_cast<const uint32_t*>(base)[idx]);
  }
}

// Load through a byte offset from a base pointer (lets the compiler use an SGPR base with a
// VGPR offset when the base is wave-uniform).
template <int DT>
__device__ __forceinline__ float2 load_c_bytes(const char* base, uint32_t byte_off) {
  using T = typename Elem<DT>::T;
  T v = *reinterpret_cast<const T*>(base + byte_off);
  if constexpr (DT == 0) return v;
  else if constexpr (DT == 1) return unpack_f16x2(v);
  else return unpack_bf16x2(v);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int DT>
__device__ __forceinline__ void store_c(void* base, int64_t idx, float2 v) {
  if constexpr (DT == 0) {
    reinterpret_cast<float2*>(base)[idx] = v;
  } else if constexpr (DT == 1) {
    __half2 h = __floats2half2_rn(v.x, v.y);
    reinterpret_cast<__half2*>(base)[idx] = h;
  } else {
    uint32_t lo = f32_to_bf16_rne(v.x), hi = f32_to_bf16_rne(v.y);
    reinterpret_cast<uint32_t*>(base)[idx] = lo | (hi << 16);
  }
}

// Weight entry t of a sparse set as float2 (WDT 0 = C64, 1 = C16_F16).
template <int WDT>
__device__ __forceinline__ float2 load_w(const void* w, int64_t idx) {
  if constexpr (WDT == 0) return reinterpret_cast<const float2*>(w)[idx];
  else return unpack_f16x2(reinterpret_cast<const uint32_t*>(w)[idx]);
}

// ---------------------------------------------------------------- math
// sin / cos of 2*pi*x for |x| <= 0.5 revolutions (hardware transcendental units).
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }

// Fractional revolutions of a float64 phase counted in revolutions, in [-0.5, 0.5].
__device__ __forceinline__ float frac_rev(double q) { return (float)(q - rint(q)); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// acc += conj(w) * y
__device__ __forceinline__ void cmac_conj(float2& acc, float2 w, float2 y) {
  acc.x = fmaf(w.x, y.x, acc.x);
  acc.x = fmaf(w.y, y.y, acc.x);
  acc.y = fmaf(w.x, y.y, acc.y);
  acc.y = fmaf(-w.y, y.x, acc.y);
}

template <typename T>
__device__ __forceinline__ T readlane(T v, int lane) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32/64-bit only");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  }
}

__device__ __forceinline__ int wave_lane() { return __lane_id(); }

// Raw buffer resource over `bytes` bytes (gfx9 family word 3).  Loads address
// base + voffset + soffset; a load whose offset is not below `bytes` returns zero without a
// memory access (the descriptor's range check).
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

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).  Map
// the hardware block index to a logical one so that each XCD receives a contiguous range of
// logical blocks (neighbouring range rows share Y rows in that XCD's L2).
// ---------------------------------------------------------------- eq. 40 rounding ties
// NEAREST takes the bin floor(u + 1/2) of u = beta R (eq. 40, eq. 2).  The kernels evaluate u
// in a fast way whose error is bounded (float64 with fused operations, or a float64 nominal
// bin plus a float32 correction); where floor could then differ from the plain evaluation,
// i.e. within that bound of a rounding boundary, they recompute u the plain way below.

constexpr double kTwoPiD = 6.283185307179586476925286766559;

// cos x in float64 for |x| < 2^20 (angles of a rotation and their errors): Cody-Waite
// reduction by pi (a 33 + 33 + 53-bit split of pi, so q P1 and q P2 are exact for |q| < 2^20),
// cos x = (-1)^q cos r with |r| <= pi/2, and the Taylor series of cos r to the r^24 term
// (remainder below 4e-22).  About 1 ulp of absolute error; one polynomial, so few registers in
// the rarely taken branches that call it.
__device__ __forceinline__ double cos_reduced(double x) {
  constexpr double kInvPi = 0.31830988618379067154;
  constexpr double kP1 = 0x1.921fb54400000p+1;
  constexpr double kP2 = 0x1.0b4611a600000p-33;
  constexpr double kP3 = 0x1.3198a2e037073p-68;
  const double q = rint(x * kInvPi);
  const double r = ((x - q * kP1) - q * kP2) - q * kP3;
  const double z = r * r;
  double c = 1.0 / 620448401733239439360000.0;   // 1/24!
  c = c * z - 1.0 / 1124000727777607680000.0;    // 1/22!
  c = c * z + 1.0 / 2432902008176640000.0;       // 1/20!
  c = c * z - 1.0 / 6402373705728000.0;          // 1/18!
  c = c * z + 1.0 / 20922789888000.0;            // 1/16!
  c = c * z - 1.0 / 87178291200.0;               // 1/14!
  c = c * z + 1.0 / 479001600.0;                 // 1/12!
  c = c * z - 1.0 / 3628800.0;                   // 1/10!
  c = c * z + 1.0 / 40320.0;                     // 1/8!
  c = c * z - 1.0 / 720.0;                       // 1/6!
  c = c * z + 1.0 / 24.0;
  c = c * z - 0.5;
  c = c * z + 1.0;
  return ((int64_t)q & 1) ? -c : c;
}

// u + 1/2 of a point at range rr seen from a phase centre at angle d from it, with every
// operation rounded on its own in the order eq. 2 writes it:
// beta sqrt((rr rr + r r) - ((2 r) rr) cos d) + 1/2.
__device__ __attribute__((noinline)) double plain_bin_half(double rr, double radius, double d, double beta) {
#pragma clang fp contract(off)
  const double cd = cos_reduced(d);
  const double c1 = rr * rr + radius * radius;
  const double c2 = 2.0 * radius * rr;
  const double rn = sqrt(c1 - c2 * cd);
  return beta * rn + 0.5;
}

// True when floor(u) may differ from the plain evaluation's: u lies within `err` of an
// integer.
__device__ __forceinline__ bool near_bin_tie(double u, double err) {
  const double t = u - floor(u);
  return t < err || t > 1.0 - err;
}

// Bound on the error of a float64 bin evaluated with fused operations and a different but
// equivalent angle expression (a few ulps of u < 2^20): far below it.
constexpr double kBinErr64 = 0x1p-30;

// A float64 nominal bin split as floor(u) and its fraction in float32, so the per-pair work of
// the corrected paths (nominal bin plus a float32 correction) stays in float32.
struct SplitBin {
  int32_t i;
  float f;
};
__device__ __forceinline__ SplitBin split_bin(double u) {
  const double fl = floor(u);
  return SplitBin{(int32_t)fl, (float)(u - fl)};
}

// floor(i + f + corr) of a split nominal bin plus a float32 correction `corr` (in bins), and
// whether that sum lies near a rounding boundary: within the bound of its error, a few float32
// ulps relative to corr (hardware reciprocal square root and reciprocal) plus an absolute error
// below 2^-18 bins (the float32 geometry terms, sin and cos of the half angle error, and the
// float32 fraction).  The fraction of the sum comes out in *frac.
__device__ __forceinline__ int corr_bin(SplitBin nb, float corr, float* frac, bool* tie) {
  const float x = nb.f + corr;
  const float fl = floorf(x);
  const float fr = x - fl;
  const float err = 0x1p-18f + fabsf(corr) * 0x1p-12f;
  *frac = fr;
  *tie = fr < err || fr > 1.f - err;
  return nb.i + (int)fl;
}

__device__ __forceinline__ int xcd_logical_block(int b, int nblocks) {
  int per = nblocks / kXcds, rem = nblocks % kXcds;
  int xcd = b % kXcds, local = b / kXcds;
  int base = xcd * per + (xcd < rem ? xcd : rem);
  // XCD x receives per + (x < rem) blocks, so [base, base + count) tiles [0, nblocks)
  return base + local;
}

}  // namespace rosar
