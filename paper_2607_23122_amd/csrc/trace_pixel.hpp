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
// Every lane of the wave calls it (`inside` false: the lane rides along).
// AO rays take per-lane walks from the wave's entry node (wave_entry_node);
// `stack` is this lane's LDS stack, `stride` apart between entries, and
// `wstack` the wave's stack of kStackTotal entries for the rays whose
// per-lane walk overflowed its stack (decided again by a wave-coherent walk:
// the same closest hit).  Shadow rays take one wave-coherent walk.  With
// COUNT every ray takes the per-lane walk from the root, whose work is added
// to *ws.  LT: one light (LightF) or several (LightSetF, shadows).
template <int MODE, bool COUNT = false, class LT = LightF>
__device__ inline void trace_pixel(const DeviceBVH &bvh, const GBufView &g, float R, const LT &L, uint32_t sd,
                                   uint32_t sample, const OccView &out, int px, int py, bool inside,
                                   uint32_t *stack, int stride, uint32_t *wstack, WalkStats *ws = nullptr) {
    const int64_t i = inside ? (int64_t)py * g.w + px : 0;
    const uint32_t prim = inside ? g.prim[i] : OCR_HIT_MISS;
    uint32_t code = OCR_HIT_MISS;  // background, or a shadow sample that is not traced
    float d[3] = {0.f, 0.f, 0.f};
    const float tmax = MODE == OCR_AO ? R : 1.0f;
    bool want = false;
    TRay r{};
    // the segment's box, for the AO walks' common entry node
    float slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (prim != OCR_HIT_MISS) {
        float x[3], n[3], o[3];
        load3(g.pos, i, x);
        load3(g.nrm, i, n);
        offset_point(x, n, o);
        if (MODE == OCR_AO) {
            ao_direction((uint32_t)px, (uint32_t)py, sample, sd, n, d);
            want = true;
        } else {
            float y[3];
            LightF Lc;  // the light the sample lies on
            pick_light((uint32_t)px, (uint32_t)py, sample, sd, L, o, y, Lc);
            d[0] = y[0] - o[0];
            d[1] = y[1] - o[1];
            d[2] = y[2] - o[2];
            want = shadow_traced(n, o, d, Lc);
            if (!want) code = OCR_HIT_SELF;
        }
        if (want) {
            make_ray(o, d, prim, OCR_HIT_MISS, tmax, r);
            for (int c = 0; c < 3; ++c) {
                const float e = __fmaf_rn(d[c], tmax, o[c]);
                slo[c] = fminf(o[c], e);
                shi[c] = fmaxf(o[c], e);
            }
        }
    }
    Hit h;
    h.t = tmax;
    h.tri = OCR_HIT_MISS;
    h.leaf_tri = 0;
    bool overflow = false;
    if (MODE != OCR_AO && !COUNT) {
        // shadow segments of a wave's 8x8 pixels head for the same light and
        // share most of their path: one wave-coherent walk (same closest hit)
        h = traverse_wave_closest<false>(bvh, r, tmax, want, wstack);
    } else {
        // AO segments are short: the wave's walks start below the levels where
        // their common box meets one child only
        const uint32_t entry = MODE == OCR_AO && !COUNT ? wave_entry_node(bvh, slo, shi) : 0u;
        if (want) h = traverse<false, MODE == OCR_AO, COUNT>(bvh, r, tmax, stack, stride, overflow, ws, entry);
    }
    if (wave_ballot(overflow) != 0ull) {
        const Hit hw = traverse_wave_closest<MODE == OCR_AO>(bvh, r, tmax, overflow, wstack);
        if (overflow) h = hw;
    }
    if (!inside) return;
    if (!want) {
        out.hit[i] = code;
        return;
    }
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
