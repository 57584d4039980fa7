// Host-side pieces shared by the C-ABI translation units (api.cpp, plan.cpp,
// server.cpp): the BVH handle's layout, argument checks and the thread-local
// error report.
#pragma once
#include <hip/hip_runtime.h>

#include "ocr_common.hpp"

struct ocr_bvh {
    ocr::DeviceBVH dev;
    void *mem = nullptr;  // one allocation: nodes then triangles
    int device = 0;
    ocr_bvh_info info{};
};

namespace ocr {

// Record `fmt` as this thread's last error and return `st`.
ocr_status fail(ocr_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ocr_status hip_fail(hipError_t e, const char *what);

ocr_status check_gbuf(const ocr_gbuffer *g);
ocr_status check_params(const ocr_reuse_params *p);
// Validate a rectangular light and derive the kernels' FP32 form.
ocr_status make_light(const ocr_rect_light *l, LightF &L);
// OCR_ERR_UNSUPPORTED for a light not sampled uniformly (entry points that
// take the uniform emitter density only); `who` names the caller.
ocr_status uniform_only(const ocr_rect_light *l, const char *who);
// Validate (mode, AO radius, light) as the batched plan, the server and the
// counted trace take them (uniform emitter density only); fills L (zero for AO).
ocr_status check_effect(int32_t mode, float ao_radius, const ocr_rect_light *light, LightF &L);

inline GBufView view(const ocr_gbuffer *g) { return GBufView{g->pos, g->nrm, g->prim, g->width, g->height}; }

// Several rectangular lights (lights.hpp): validated set, and the shadow
// launchers that take it (trace.hip, reuse.hip).
struct LightSetF;
ocr_status make_lights(const ocr_rect_light *lights, int32_t n, LightSetF &S);
hipError_t launch_trace_lights(const DeviceBVH &bvh, const GBufView &g, const LightSetF &L, uint32_t seed32,
                               uint32_t sample, const OccView &out, hipStream_t st);
hipError_t launch_validate_lights(const DeviceBVH &bvh, const GBufView &g, const OccView &occ, const LightSetF &L,
                                  const ocr_reuse_params &p, uint32_t *bits, uint64_t *stats, hipStream_t st);
hipError_t launch_reuse_lights(const GBufView &g, const OccView &occ, const LightSetF &L, const ocr_reuse_params &p,
                               const uint32_t *bits, float *out, hipStream_t st);

// One light sampled from the bilinear emitter density (lights.hpp): the
// launchers that take it (trace.hip, reuse.hip); its validation is the
// uniform light's (the support does not depend on the density).
struct LightBilinF;
hipError_t launch_trace_bilinear(const DeviceBVH &bvh, const GBufView &g, const LightBilinF &L, uint32_t seed32,
                                 uint32_t sample, const OccView &out, hipStream_t st);
hipError_t launch_samples_bilinear(const GBufView &g, const LightBilinF &L, uint32_t seed32, uint32_t sample,
                                   float *o, float *d, uint8_t *kind, hipStream_t st);
hipError_t launch_reuse_bilinear(const GBufView &g, const OccView &occ, int mode, const LightBilinF &L,
                                 const ocr_reuse_params &p, const uint32_t *bits, float *out, hipStream_t st,
                                 float scale);

// Scratch of the no-allocation entry point (scratch.hip): a static device
// array of kScratchBytes per device; scratch_address gives its address on
// the current device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxScratchDevices = 64;
hipError_t scratch_address(void **ptr);

// The simple reuse baselines (baselines.hip).
hipError_t launch_filter(const GBufView &g, const ocr_reuse_params &p, const float *in, float *out, hipStream_t st);
hipError_t launch_light_reuse(const DeviceBVH &bvh, const GBufView &g, const LightF &L, uint32_t seed32,
                              uint32_t sample, const ocr_reuse_params &p, float *out, hipStream_t st);

}  // namespace ocr
