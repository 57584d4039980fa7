// Batched schedule: device-side view descriptors and the launchers of the
// persistent trace and reuse kernels that run many views in one launch each.
#pragma once
#include "ocr_common.hpp"

namespace ocr {

// One view as the batched kernels read it (device array, one per view).
struct BatchView {
    DeviceBVH bvh;
    GBufView g;
    OccView occ;
    LightF L;
    float R;            // AO radius (1 for shadows)
    float R2;
    uint32_t sd;        // folded seed
    uint32_t sample;
    int32_t mode;       // OCR_AO, OCR_SHADOW, kShadowSA or kDI (the last two trace shadow records)
    int32_t estimator;
    int32_t radius;     // window radius
    int32_t dark_guard; // already restricted to the biased estimator
    int32_t words;      // validation words per pixel
    int32_t r_tiles_x;  // reuse tiles (kWTX x kWTY) per row
    const uint32_t *bits;
    float *out;
    float scale;        // direct illumination: albedo * radiance / pi (1 otherwise)
};

// Work queues: counters [0, 8) for the trace ranges, [8, 16) for the reuse
// ranges, one 128-byte line each.  q_start[0..8] bounds the trace range of
// XCD x as [q_start[x], q_start[x+1]); q_start[9..17] the reuse ranges.
constexpr int kQueueStride = 32;
constexpr int kQueueWords = 16 * kQueueStride;

hipError_t launch_batch_reset(uint32_t *ctr, hipStream_t st);
hipError_t launch_batch_trace(const BatchView *views, const uint32_t *t_first, const uint32_t *t_tiles_x, int nviews,
                              const uint32_t *q_start, uint32_t *ctr, int tile_w, int tile_h, int packing, int grid,
                              hipStream_t st);
hipError_t launch_batch_reuse(const BatchView *views, const uint32_t *r_first, int nviews, const uint32_t *q_start,
                              uint32_t *ctr, size_t lds_bytes, int grid, hipStream_t st);
// Resident blocks per CU of the two kernels (occupancy query).  The reuse
// query also raises the kernel's dynamic-LDS limit to lds_bytes (call it
// before launching or capturing); it returns 0 if that fails.
int batch_trace_blocks_per_cu();
int batch_reuse_blocks_per_cu(size_t lds_bytes);
// Dynamic LDS the batched reuse kernel needs for a window view.
size_t batch_reuse_lds(int radius, int mode, bool unbiased, int words);

}  // namespace ocr
