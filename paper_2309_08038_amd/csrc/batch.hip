// Batched rotations: persistent range-compression and sparse-filter launches over many
// rotations of uneven size (placeholder until the persistent kernels land).
#include "rosar_device.hpp"

struct rosar_batch_plan {
  int32_t n;
};

extern "C" {

rosar_status rosar_batch_plan_create(const rosar_rotation_desc* descs, int32_t n, const rosar_tile* tile,
                                     rosar_batch_plan** out) {
  (void)descs;
  (void)n;
  (void)tile;
  if (out) *out = nullptr;
  return ROSAR_ERR_UNSUPPORTED;
}

rosar_status rosar_batch_run(rosar_batch_plan* plan, rosar_stream stream) {
  (void)plan;
  (void)stream;
  return ROSAR_ERR_UNSUPPORTED;
}

rosar_status rosar_batch_plan_info(const rosar_batch_plan* plan, int64_t* pixels, int64_t* rc_tiles,
                                   int64_t* sf_tiles) {
  (void)plan;
  (void)pixels;
  (void)rc_tiles;
  (void)sf_tiles;
  return ROSAR_ERR_UNSUPPORTED;
}

void rosar_batch_plan_destroy(rosar_batch_plan* plan) { delete plan; }

}  // extern "C"
