// Range compression (Sec. III-D, eq. 38): windowed L-point FFT of every pulse along fast
// time, keeping the band [l_lo, l_lo + l_count) and storing it range-bin major (pulses
// contiguous) so the azimuth filters read whole rows with coalesced loads.  The per-block work
// is fft::rc_block.
#include "fft_device.hpp"

namespace rosar {
namespace {

using fft::kRcThreads;
using fft::kRcWaves;

template <int L, int PPW, int DT>
__global__ __launch_bounds__(kRcThreads) void range_compress_kernel(RcArgs a) {
  __shared__ float2 lds[fft::rc_lds_elems(L, PPW)];
  fft::rc_block<L, PPW, DT>(a, blockIdx.x * kRcWaves * PPW, lds);
}

template <int L>
hipError_t launch_l(const RcArgs& a, hipStream_t s) {
  constexpr int PPW = fft::kRcPulsesPerWave(L);
  constexpr int PW = kRcWaves * PPW;
  dim3 grid((a.n + PW - 1) / PW);
  switch (a.dtype) {
    case ROSAR_C64: range_compress_kernel<L, PPW, 0><<<grid, kRcThreads, 0, s>>>(a); break;
    case ROSAR_C16_F16: range_compress_kernel<L, PPW, 1><<<grid, kRcThreads, 0, s>>>(a); break;
    default: range_compress_kernel<L, PPW, 2><<<grid, kRcThreads, 0, s>>>(a); break;
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
