// Batched rotations: many independent rotations of uneven pulse, sample and range-row counts
// imaged by one range-compression launch per FFT length present and one persistent
// sparse-filter launch per occupancy class.
//
// The plan uploads one descriptor per rotation (derived float64 geometry, band, pointers,
// LDS layout) and the prefix sums of their tile counts.  A tile index is mapped to its rotation
// by binary search over the prefix sums and processed by the same block functions the
// single-rotation kernels use (fft::rc_block, sparse::lds_tile), so a batched image equals the
// image of the single-rotation call with the same launch shape, bit for bit.
//
// Range compression: the rotations are grouped by FFT length; each group is one launch with
// one workgroup per 8-pulse tile, the exact LDS of its length and XCD-aware tile order (the
// hardware dispatcher balanced these short tiles better than a work queue did).  Sparse filter:
// the rotations are grouped by the occupancy their LDS layout allows, and each group is a
// persistent launch sized for its widest window, whose workgroups take tile indices from the
// group's device counter.  The counters are reset by the plan's own kernel at the start of
// every run, so that the launches can be captured in a HIP graph and replayed.  Every
// workgroup leaves its loop once its counter passes the group's tile total.
#include <algorithm>
#include <functional>
#include <cstring>
#include <string>
#include <vector>

#include "fft_device.hpp"
#include "sparse_device.hpp"

namespace rosar {
namespace {

constexpr int kBatchP = 4;       // default sparse-filter shape of a batch: 4 pixels per lane,
constexpr int kBatchWaves = 8;   // 8 waves (2048-pixel tiles)
constexpr int kBatchRcWaves = 8; // range-compression workgroup: one pulse per wave, 8 waves
constexpr int kRcLengths = 6;    // FFT lengths 64 .. 2048
constexpr int kSfClasses = 8;    // sparse-filter launches: one per occupancy class

// Range compression of one rotation inside its FFT-length group.
struct BatchRc {
  RcArgs rc;
  int32_t tile0;             // first tile of this rotation within its group
  int32_t pad;
};

struct BatchRot {
  Geo g;                     // sparse filter geometry
  View y;
  const int32_t* offsets;
  const void* weights;
  float2* image;
  double cos_hw;              // cos of the half-window angle (bounds the staged rows of a range row)
  int32_t k, window;
  int32_t rows_cap, stride, dma, tiles_per_row;
  int32_t sf_tile0;          // first sparse-filter tile of this rotation
  int32_t pad;
};

// Index of the last entry whose first tile is <= t (entries sorted by first tile).
template <typename D>
__device__ __forceinline__ int find_entry(const D* d, int nd, int t, int32_t D::*tile0) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].*tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void batch_reset_kernel(int* counters, int n) {
  if ((int)threadIdx.x < n) counters[threadIdx.x] = 0;
}

template <int L>
__global__ __launch_bounds__(kBatchRcWaves* kWave) void batch_rc_kernel(const BatchRc* __restrict__ group,
                                                                         int nrot) {
  __shared__ float2 lds[fft::rc_lds_elems(L, 1, kBatchRcWaves)];
  const int t = xcd_logical_block(blockIdx.x, gridDim.x);
  const int i = find_entry(group, nrot, t, &BatchRc::tile0);
  fft::rc_block<L, 1, 0, kBatchRcWaves>(group[i].rc, (t - group[i].tile0) * kBatchRcWaves, lds);
}

template <int P, int NW>
__global__ __launch_bounds__(kWave* NW) void batch_sf_kernel(const BatchRot* __restrict__ rots, int nrot,
                                                              int total, int* counter) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_t;
  __shared__ int s_unstaged;
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_t;
    __syncthreads();
    if (t >= total) break;
    const int i = find_entry(rots, nrot, t, &BatchRot::sf_tile0);
    const BatchRot& R = rots[i];
    const int local = t - R.sf_tile0;
    const int row = local / R.tiles_per_row;
    sparse::lds_tile<ROSAR_C64, ROSAR_C64, ROSAR_NEAREST, P, NW>(
        R.g, R.y, R.k, R.window, row, local - row * R.tiles_per_row, R.rows_cap, R.cos_hw, R.stride, R.dma,
        R.offsets,
        R.weights, reinterpret_cast<const char*>(R.y.data), R.image, smem, s_unstaged);
    __syncthreads();  // the next tile reuses the LDS
  }
}

template <int P, int NW>
struct SfKernel {
  static const void* fn() { return reinterpret_cast<const void*>(&batch_sf_kernel<P, NW>); }
  static void launch(dim3 grid, size_t lds, hipStream_t s, const BatchRot* r, int n, int total, int* c) {
    batch_sf_kernel<P, NW><<<grid, kWave * NW, lds, s>>>(r, n, total, c);
  }
};

rosar_status bfail(rosar_status st, const std::string& m) { return set_error(st, m); }

}  // namespace
}  // namespace rosar

struct rosar_batch_plan {
  int n = 0;
  int device = -1;
  int ppl = rosar::kBatchP, waves = rosar::kBatchWaves;
  rosar::BatchRot* d_rots = nullptr;
  rosar::BatchRc* d_rc = nullptr;                 // grouped by FFT length
  int rc_first[rosar::kRcLengths] = {};           // first entry of each length's group in d_rc
  int rc_count[rosar::kRcLengths] = {};           // rotations in the group
  int rc_tiles[rosar::kRcLengths] = {};           // tiles (8-pulse groups) of the group
  int* d_counters = nullptr;                      // one work counter per sparse-filter class
  int rc_total = 0, sf_total = 0;
  int64_t pixels = 0;
  // sparse filter: rotations grouped by how many workgroups of their LDS layout fit on a CU;
  // class c is d_rots[sf_first[c], sf_first[c] + sf_count[c]), one persistent launch each
  int sf_classes = 0;
  int sf_first[rosar::kSfClasses] = {}, sf_count[rosar::kSfClasses] = {};
  int sf_tiles[rosar::kSfClasses] = {}, sf_grid[rosar::kSfClasses] = {};
  size_t sf_lds[rosar::kSfClasses] = {};
};

namespace rosar {

namespace {

// Groups the rotations by the occupancy their LDS layout allows (rotations with small windows
// should not run at the occupancy of the widest one), reorders hv class by class, numbers the
// tiles within each class and sizes each class's persistent grid.
template <int P, int NW>
rosar_status plan_shape(std::vector<BatchRot>& hv, const std::vector<size_t>& lds, rosar_batch_plan* pl, int cus) {
  const int n = (int)hv.size();
  std::vector<int> occ(n);
  for (int i = 0; i < n; ++i) {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, SfKernel<P, NW>::fn(), kWave * NW, lds[i]) != hipSuccess ||
        o < 1)
      return bfail(ROSAR_ERR_HIP, "occupancy query for the batched sparse-filter kernel failed");
    occ[i] = o;
  }
  std::vector<int> levels(occ.begin(), occ.end());
  std::sort(levels.begin(), levels.end(), std::greater<int>());
  levels.erase(std::unique(levels.begin(), levels.end()), levels.end());
  while ((int)levels.size() > kSfClasses) levels.pop_back();   // merge the lowest levels
  std::vector<BatchRot> sorted;
  sorted.reserve(n);
  pl->sf_classes = (int)levels.size();
  for (int c = 0; c < pl->sf_classes; ++c) {
    const bool last = c == pl->sf_classes - 1;
    pl->sf_first[c] = (int)sorted.size();
    int64_t tiles = 0;
    size_t bytes = 0;
    for (int i = 0; i < n; ++i) {
      if (!(occ[i] == levels[c] || (last && occ[i] < levels[c]))) continue;
      BatchRot R = hv[i];
      R.sf_tile0 = (int32_t)tiles;
      tiles += (int64_t)R.tiles_per_row * R.g.n_range;
      bytes = std::max(bytes, lds[i]);
      sorted.push_back(R);
    }
    pl->sf_count[c] = (int)sorted.size() - pl->sf_first[c];
    pl->sf_tiles[c] = (int)tiles;
    pl->sf_lds[c] = bytes;
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, SfKernel<P, NW>::fn(), kWave * NW, bytes) != hipSuccess ||
        o < 1)
      return bfail(ROSAR_ERR_HIP, "occupancy query for the batched sparse-filter kernel failed");
    pl->sf_grid[c] = (int)std::min<int64_t>((int64_t)cus * o, std::max<int64_t>(tiles, 1));
  }
  hv.swap(sorted);
  return ROSAR_OK;
}

template <int P, int NW>
void run_shape(rosar_batch_plan* pl, hipStream_t s) {
  for (int c = 0; c < pl->sf_classes; ++c)
    SfKernel<P, NW>::launch(dim3(pl->sf_grid[c]), pl->sf_lds[c], s, pl->d_rots + pl->sf_first[c], pl->sf_count[c],
                            pl->sf_tiles[c], pl->d_counters + c);
}

#define ROSAR_BATCH_SHAPES(X) X(1, 4) X(2, 4) X(4, 4) X(8, 4) X(2, 2) X(4, 2) X(8, 2) X(4, 8)

bool batch_shape_supported(int p, int nw) {
#define ROSAR_CHECK(P, NW) if (p == P && nw == NW) return true;
  ROSAR_BATCH_SHAPES(ROSAR_CHECK)
#undef ROSAR_CHECK
  return false;
}

}  // namespace
}  // namespace rosar

extern "C" {

rosar_status rosar_batch_plan_create(const rosar_rotation_desc* descs, int32_t n, const rosar_tile* tile,
                                     rosar_batch_plan** out) {
  using namespace rosar;
  clear_error();
  if (!out) return bfail(ROSAR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!descs || n < 1 || n > 65536) return bfail(ROSAR_ERR_INVALID_ARG, "need 1..65536 rotation descriptors");
  int p = kBatchP, nw = kBatchWaves;
  if (tile && (tile->pixels_per_lane || tile->waves)) {
    p = tile->pixels_per_lane ? tile->pixels_per_lane : p;
    nw = tile->waves ? tile->waves : nw;
  }
  if (!batch_shape_supported(p, nw))
    return bfail(ROSAR_ERR_UNSUPPORTED, "batch launch shape (" + std::to_string(p) + " pixels/lane, " +
                                            std::to_string(nw) + " waves) not supported");
  const int tpx = kWave * p * nw;
  std::vector<BatchRot> hv(n);
  std::vector<BatchRc> rc_by_len[kRcLengths];
  int64_t rc_tiles[kRcLengths] = {};
  int64_t sf_total = 0, pixels = 0;
  std::vector<size_t> sf_lds(n);
  for (int i = 0; i < n; ++i) {
    const rosar_rotation_desc& d = descs[i];
    const rosar_status st = validate_rotation(d, i);
    if (st != ROSAR_OK) return st;
    BatchRc C;
    std::memset(&C, 0, sizeof(C));
    C.rc.raw = reinterpret_cast<const float2*>(d.raw);
    C.rc.window = d.window;
    C.rc.out = d.y_t;
    C.rc.ld = d.ld;
    C.rc.n = d.geom.n_pulses;
    C.rc.m = d.geom.n_fast;
    C.rc.l = d.geom.n_fft;
    C.rc.l_lo = d.l_lo;
    C.rc.l_count = d.l_count;
    C.rc.halo = d.halo;
    C.rc.dtype = ROSAR_C64;
    C.rc.scale = 1.0f;
    int li = 0;
    while ((64 << li) < C.rc.l) ++li;   // n_fft is a power of two in [64, 2048]
    C.tile0 = (int32_t)rc_tiles[li];
    rc_tiles[li] += (C.rc.n + kBatchRcWaves - 1) / kBatchRcWaves;
    rc_by_len[li].push_back(C);

    BatchRot& R = hv[i];
    std::memset(&R, 0, sizeof(R));
    R.g = geo_of(&d.geom, &d.grid);
    R.y = View{d.y_t, d.ld, d.l_lo, d.l_count, d.halo, ROSAR_C64, 1.0f};
    R.offsets = d.set.offsets;
    R.weights = d.set.weights;
    R.image = reinterpret_cast<float2*>(d.image);
    R.k = d.set.k;
    R.window = d.set.window;
    // staged rows capped so that the window fits the LDS budget; capped taps go through the guard
    const sparse::LdsLayout L = sparse::lds_layout_capped(R.g, R.y, R.k, R.window, ROSAR_NEAREST, tpx);
    if (L.bytes > sparse::kLdsBudget)
      return bfail(ROSAR_ERR_UNSUPPORTED, "rotation " + std::to_string(i) + ": window does not fit in LDS");
    R.rows_cap = L.rows;
    R.cos_hw = L.cos_hw;
    R.stride = L.stride;
    R.dma = L.dma;
    R.tiles_per_row = (R.g.n + tpx - 1) / tpx;
    sf_total += (int64_t)R.tiles_per_row * R.g.n_range;
    pixels += (int64_t)R.g.n * R.g.n_range;
    sf_lds[i] = L.bytes;
  }
  int64_t rc_total = 0;
  for (int li = 0; li < kRcLengths; ++li) rc_total += rc_tiles[li];
  if (rc_total >= INT32_MAX / 2 || sf_total >= INT32_MAX / 2)
    return bfail(ROSAR_ERR_UNSUPPORTED, "too many tiles in one batch");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return bfail(ROSAR_ERR_HIP, "cannot query the current device");
  auto* pl = new (std::nothrow) rosar_batch_plan();
  if (!pl) return bfail(ROSAR_ERR_NO_MEMORY, "host allocation failed");
  pl->n = n;
  pl->device = dev;
  pl->ppl = p;
  pl->waves = nw;
  pl->rc_total = (int)rc_total;
  pl->sf_total = (int)sf_total;
  pl->pixels = pixels;
  std::vector<BatchRc> hrc;
  hrc.reserve(n);
  for (int li = 0; li < kRcLengths; ++li) {
    pl->rc_first[li] = (int)hrc.size();
    pl->rc_count[li] = (int)rc_by_len[li].size();
    pl->rc_tiles[li] = (int)rc_tiles[li];
    hrc.insert(hrc.end(), rc_by_len[li].begin(), rc_by_len[li].end());
  }
  auto fail = [pl](rosar_status st, const std::string& m) {
    (void)hipFree(pl->d_rots);
    (void)hipFree(pl->d_rc);
    (void)hipFree(pl->d_counters);
    delete pl;
    return bfail(st, m);
  };
  rosar_status st = ROSAR_ERR_UNSUPPORTED;
#define ROSAR_PLAN(P, NW) if (p == P && nw == NW) st = plan_shape<P, NW>(hv, sf_lds, pl, cus);
  ROSAR_BATCH_SHAPES(ROSAR_PLAN)
#undef ROSAR_PLAN
  if (st != ROSAR_OK) {
    delete pl;
    return st;
  }
  if (hipMalloc(&pl->d_rots, sizeof(BatchRot) * n) != hipSuccess ||
      hipMalloc(&pl->d_rc, sizeof(BatchRc) * n) != hipSuccess ||
      hipMalloc(&pl->d_counters, kSfClasses * sizeof(int)) != hipSuccess)
    return fail(ROSAR_ERR_NO_MEMORY, "device allocation of the batch descriptors failed");
  if (hipMemcpy(pl->d_rots, hv.data(), sizeof(BatchRot) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->d_rc, hrc.data(), sizeof(BatchRc) * n, hipMemcpyHostToDevice) != hipSuccess)
    return fail(ROSAR_ERR_HIP, "upload of the batch descriptors failed");
  *out = pl;
  return ROSAR_OK;
}

rosar_status rosar_batch_run(rosar_batch_plan* pl, rosar_stream stream) {
  using namespace rosar;
  clear_error();
  if (!pl) return bfail(ROSAR_ERR_INVALID_ARG, "plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device)
    return bfail(ROSAR_ERR_INVALID_ARG, "plan was created on another device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  batch_reset_kernel<<<1, 64, 0, s>>>(pl->d_counters, pl->sf_classes);
  for (int li = 0; li < kRcLengths; ++li) {
    if (!pl->rc_count[li]) continue;
    const BatchRc* g = pl->d_rc + pl->rc_first[li];
    const int nb = pl->rc_tiles[li], nr = pl->rc_count[li];
    switch (li) {
      case 0: batch_rc_kernel<64><<<nb, kBatchRcWaves * kWave, 0, s>>>(g, nr); break;
      case 1: batch_rc_kernel<128><<<nb, kBatchRcWaves * kWave, 0, s>>>(g, nr); break;
      case 2: batch_rc_kernel<256><<<nb, kBatchRcWaves * kWave, 0, s>>>(g, nr); break;
      case 3: batch_rc_kernel<512><<<nb, kBatchRcWaves * kWave, 0, s>>>(g, nr); break;
      case 4: batch_rc_kernel<1024><<<nb, kBatchRcWaves * kWave, 0, s>>>(g, nr); break;
      default: batch_rc_kernel<2048><<<nb, kBatchRcWaves * kWave, 0, s>>>(g, nr); break;
    }
  }
#define ROSAR_RUN(P, NW) if (pl->ppl == P && pl->waves == NW) run_shape<P, NW>(pl, s);
  ROSAR_BATCH_SHAPES(ROSAR_RUN)
#undef ROSAR_RUN
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(ROSAR_ERR_HIP, std::string("batch launch: ") + hipGetErrorString(e));
  return ROSAR_OK;
}

rosar_status rosar_batch_plan_info(const rosar_batch_plan* pl, int64_t* pixels, int64_t* rc_tiles,
                                   int64_t* sf_tiles) {
  using namespace rosar;
  clear_error();
  if (!pl) return bfail(ROSAR_ERR_INVALID_ARG, "plan is NULL");
  if (pixels) *pixels = pl->pixels;
  if (rc_tiles) *rc_tiles = pl->rc_total;
  if (sf_tiles) *sf_tiles = pl->sf_total;
  return ROSAR_OK;
}

rosar_status rosar_batch_autotune(const rosar_rotation_desc* descs, int32_t n, int32_t reps, rosar_tile* best,
                                  float* best_us, rosar_stream stream) {
  using namespace rosar;
  clear_error();
  if (!best || !best_us) return bfail(ROSAR_ERR_INVALID_ARG, "best / best_us is NULL");
  if (reps < 1 || reps > 1000) return bfail(ROSAR_ERR_INVALID_ARG, "reps must be in [1, 1000]");
  if (!descs || n < 1) return bfail(ROSAR_ERR_INVALID_ARG, "descs NULL or n < 1");
  // cache key: the shapes of every rotation (FNV-1a over their sizes, band layouts and sets)
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
  };
  for (int32_t i = 0; i < n; ++i) {
    const rosar_status vs = validate_rotation(descs[i], i);
    if (vs != ROSAR_OK) return vs;
    const rosar_rotation_desc& d = descs[i];
    const int64_t f[] = {d.geom.n_pulses, d.geom.n_fast, d.geom.n_fft, d.grid.n_range, d.grid.n_az, d.l_lo,
                         d.l_count, d.halo, d.ld, d.set.k, d.set.window, d.set.w_dtype};
    mix(f, sizeof(f));
    const double r[] = {d.geom.radius_m, d.grid.r0_m, d.grid.dr_m};
    mix(r, sizeof(r));
  }
  char kb[160];
  snprintf(kb, sizeof(kb), "%s|batch|n=%d|shapes=%016llx", tune_arch().c_str(), n, (unsigned long long)h);
  const std::string key = kb;
  if (tune_cache_get(key, best, best_us)) return ROSAR_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // it allocates, synchronises and times: refused on a capturing stream, which stays valid
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess)
    return bfail(ROSAR_ERR_HIP, "rosar_batch_autotune: cannot query the stream's capture status");
  if (cap != hipStreamCaptureStatusNone)
    return bfail(ROSAR_ERR_INVALID_ARG, "rosar_batch_autotune allocates and synchronises: it cannot run under "
                                        "stream capture");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return bfail(ROSAR_ERR_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(ROSAR_ERR_HIP, "hipEventCreate failed");
  }
  bool have = false;
  float best_t = 0.f;
  rosar_tile bt{};
  rosar_status st = ROSAR_OK;
  const int shapes[][2] = {{1, 4}, {2, 4}, {4, 4}, {8, 4}, {2, 2}, {4, 2}, {8, 2}, {4, 8}};
  for (const auto& sh : shapes) {
    rosar_tile t{1, sh[0], sh[1], 0};
    rosar_batch_plan* pl = nullptr;
    const rosar_status cs = rosar_batch_plan_create(descs, n, &t, &pl);
    if (cs == ROSAR_ERR_UNSUPPORTED) continue;  // this shape cannot hold some window
    if (cs != ROSAR_OK) {
      st = cs;
      break;
    }
    st = rosar_batch_run(pl, stream);  // warm-up
    hipError_t e = st == ROSAR_OK ? hipEventRecord(e0, s) : hipSuccess;
    for (int r = 0; st == ROSAR_OK && e == hipSuccess && r < reps; ++r) st = rosar_batch_run(pl, stream);
    if (st == ROSAR_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (st == ROSAR_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (st == ROSAR_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    rosar_batch_plan_destroy(pl);
    if (st != ROSAR_OK) break;
    if (e != hipSuccess) {
      st = bfail(ROSAR_ERR_HIP, std::string("batch autotune timing: ") + hipGetErrorString(e));
      break;
    }
    const float us = 1000.f * ms / (float)reps;
    if (!have || us < best_t) {
      have = true;
      best_t = us;
      bt = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ROSAR_OK) return st;
  if (!have) return bfail(ROSAR_ERR_UNSUPPORTED, "no batch launch shape holds these windows");
  *best = bt;
  *best_us = best_t;
  if (!tune_cache_put(key, bt, best_t)) return bfail(ROSAR_ERR_INVALID_ARG, "cannot write the autotune cache file");
  clear_error();
  return ROSAR_OK;
}

void rosar_batch_plan_destroy(rosar_batch_plan* pl) {
  if (!pl) return;
  (void)hipFree(pl->d_rots);
  (void)hipFree(pl->d_rc);
  (void)hipFree(pl->d_counters);
  delete pl;
}

}  // extern "C"
