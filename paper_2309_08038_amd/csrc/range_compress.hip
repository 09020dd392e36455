// Range compression (Sec. III-D, eq. 38): windowed L-point FFT of every pulse along fast
// time, keeping the band [l_lo, l_lo + l_count) and storing it range-bin major (pulses
// contiguous) so the azimuth filters read whole rows with coalesced loads.  The per-block work
// is fft::rc_block.
#include "fft_device.hpp"
#include "mixed_fft.hpp"

namespace rosar {
namespace {

// Consecutive pulse groups go to the same XCD so that the two halves of a 128-byte output line
// (two workgroups' 64-byte row segments) meet in one L2.
template <int L, int PPW, int NW, int DT>
__global__ __launch_bounds__(NW* kWave) void range_compress_kernel(RcArgs a) {
  __shared__ float2 lds[fft::rc_lds_elems(L, PPW, NW)];
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  fft::rc_block<L, PPW, DT, NW>(a, b * NW * PPW, lds);
}

// One pulse per wave keeps the LDS footprint per wave at one padded pulse row; eight waves per
// workgroup give 64-byte complex64 row segments in the transposed store.  Measured on gfx950
// against 1-2 pulses per wave and 4-16 waves for the 3600 x 512 and 7200 x 1024 workloads,
// this shape was the fastest or tied.
template <int L>
hipError_t launch_l(const RcArgs& a, hipStream_t s) {
  constexpr int NW = 8;
  dim3 grid((a.n + NW - 1) / NW);
  switch (a.dtype) {
    case ROSAR_C64: range_compress_kernel<L, 1, NW, 0><<<grid, NW * kWave, 0, s>>>(a); break;
    case ROSAR_C16_F16: range_compress_kernel<L, 1, NW, 1><<<grid, NW * kWave, 0, s>>>(a); break;
    default: range_compress_kernel<L, 1, NW, 2><<<grid, NW * kWave, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

// Other lengths L = 2^a 3^b 5^c (up to 8192): one pulse per workgroup, the windowed pulse
// zero-padded to L in LDS, the mixed-radix workgroup FFT, then the band rows of that pulse
// (one element per row: a functional path for lengths such as M = L = 225, not a tuned one).
template <int DT>
__global__ __launch_bounds__(mfft::kFftThreads) void range_compress_mixed_kernel(RcArgs a, FftFactors f) {
  extern __shared__ float2 buf[];   // [L] pulse, then the twiddle tables
  const int n = blockIdx.x;
  const int l = f.n;
  const int tid = threadIdx.x;
  mfft::Twiddles& tw = *reinterpret_cast<mfft::Twiddles*>(buf + l);
  mfft::make_twiddles(tw, l, tid);
  const float2* raw = a.raw + (int64_t)n * a.m;
  for (int i = tid; i < l; i += mfft::kFftThreads) {
    float2 x = make_float2(0.f, 0.f);
    if (i < a.m) {
      const float w = a.window ? a.window[i] : 1.f;
      x = raw[i];
      x.x *= w;
      x.y *= w;
    }
    buf[i] = x;
  }
  __syncthreads();
  mfft::block_fft<-1>(buf, f, tw, tid);
  for (int lr = tid; lr < a.l_count; lr += mfft::kFftThreads) {
    float2 v = buf[a.l_lo + lr];
    v.x *= a.scale;
    v.y *= a.scale;
    const int64_t row = (int64_t)lr * a.ld;
    store_c<DT>(a.out, row + n + a.halo, v);
    if (n < a.halo) store_c<DT>(a.out, row + n + a.halo + a.n, v);
    if (n >= a.n - a.halo) store_c<DT>(a.out, row + n + a.halo - a.n, v);
  }
}

hipError_t launch_mixed(const RcArgs& a, hipStream_t s) {
  FftFactors f{};
  if (!fft_factors(a.l, &f)) return hipErrorInvalidValue;
  const size_t lds = (size_t)a.l * sizeof(float2) + sizeof(mfft::Twiddles);
  switch (a.dtype) {
    case ROSAR_C64: range_compress_mixed_kernel<0><<<a.n, mfft::kFftThreads, lds, s>>>(a, f); break;
    case ROSAR_C16_F16: range_compress_mixed_kernel<1><<<a.n, mfft::kFftThreads, lds, s>>>(a, f); break;
    default: range_compress_mixed_kernel<2><<<a.n, mfft::kFftThreads, lds, s>>>(a, f); break;
  }
  return hipGetLastError();
}

}  // namespace

bool range_compress_length_supported(int32_t l) {
  if (l >= 64 && l <= 2048 && (l & (l - 1)) == 0) return true;
  FftFactors f{};
  return fft_factors(l, &f);
}

hipError_t launch_range_compress(const RcArgs& a, hipStream_t s) {
  switch (a.l) {
    case 64: return launch_l<64>(a, s);
    case 128: return launch_l<128>(a, s);
    case 256: return launch_l<256>(a, s);
    case 512: return launch_l<512>(a, s);
    case 1024: return launch_l<1024>(a, s);
    case 2048: return launch_l<2048>(a, s);
    default: return launch_mixed(a, s);
  }
}

}  // namespace rosar
