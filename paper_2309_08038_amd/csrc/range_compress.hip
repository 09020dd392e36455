// Range compression (Sec. III-D, eq. 38): windowed L-point FFT of every pulse along fast
// time, keeping the band [l_lo, l_lo + l_count) and storing it range-bin major (pulses
// contiguous) so the azimuth filters read whole rows with coalesced loads.  The per-block work
// is fft::rc_block.
#include "fft_device.hpp"

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

}  // namespace

hipError_t launch_range_compress(const RcArgs& a, hipStream_t s) {
  switch (a.l) {
    case 64: return launch_l<64>(a, s);
    case 128: return launch_l<128>(a, s);
    case 256: return launch_l<256>(a, s);
    case 512: return launch_l<512>(a, s);
    case 1024: return launch_l<1024>(a, s);
    case 2048: return launch_l<2048>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rosar
