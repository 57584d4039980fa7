// Per-pixel first-hit trace (step 1 of App. D / App. H), shared by the
// per-frame trace kernel and the batched schedule.
#pragma once
#include "lights.hpp"
#include "ocr_common.hpp"
#include "traverse.hpp"

namespace ocr {

__device__ inline void load3(const float *p, int64_t i, float v[3]) {
    v[0] = p[3 * i];
    v[1] = p[3 * i + 1];
    v[2] = p[3 * i + 2];
}

// Sample pixel (px, py), trace its ray and write its occluder record.
// `stack` is this lane's LDS stack, `stride` apart between entries.  With
// COUNT the walk's work is added to *ws.  LT: one light (LightF) or several
// (LightSetF, shadows).
template <int MODE, bool COUNT = false, class LT = LightF>
__device__ inline void trace_pixel(const DeviceBVH &bvh, const GBufView &g, float R, const LT &L, uint32_t sd,
                                   uint32_t sample, const OccView &out, int px, int py, uint32_t *stack,
                                   int stride, WalkStats *ws = nullptr) {
    int64_t i = (int64_t)py * g.w + px;
    uint32_t prim = g.prim[i];
    if (prim == OCR_HIT_MISS) {
        out.hit[i] = OCR_HIT_MISS;
        return;
    }
    float x[3], n[3], o[3], d[3];
    load3(g.pos, i, x);
    load3(g.nrm, i, n);
    offset_point(x, n, o);
    float tmax;
    if (MODE == OCR_AO) {
        ao_direction((uint32_t)px, (uint32_t)py, sample, sd, n, d);
        tmax = R;
    } else {
        float y[3];
        LightF Lc;  // the light the sample lies on
        pick_light((uint32_t)px, (uint32_t)py, sample, sd, L, o, y, Lc);
        d[0] = y[0] - o[0];
        d[1] = y[1] - o[1];
        d[2] = y[2] - o[2];
        if (!shadow_traced(n, o, d, Lc)) {
            out.hit[i] = OCR_HIT_SELF;
            return;
        }
        tmax = 1.0f;
    }
    TRay r;
    make_ray(o, d, prim, OCR_HIT_MISS, tmax, r);
    Hit h = traverse<false, MODE == OCR_AO, COUNT>(bvh, r, tmax, stack, stride, ws);
    out.hit[i] = h.tri;
    if (h.tri == OCR_HIT_MISS) return;
    float nz[3];
    oriented_normal(bvh, h.leaf_tri, d, nz);
    for (int c = 0; c < 3; ++c) {
        out.dz[3 * i + c] = h.t * d[c];
        out.nz[3 * i + c] = nz[c];
    }
}

}  // namespace ocr
