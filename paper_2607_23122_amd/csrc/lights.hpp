// Shadows of several rectangular lights.  The paper shows a two-light result
// without a formulation; the target taken is the visible fraction of the total
// emitting area, sum_l (A_l / A_tot) Shadow_l.  A sample picks light l with
// probability A_l / A_tot, so that its point is uniform over the union of the
// lights; the induced density of an occluder is then the area-weighted sum of
// the per-light densities (as for one light, the factor 1 / A_tot common to
// all receivers is dropped) and F_i the area-weighted front fraction.
//
// The kernels take the light type as a template parameter: LightF (one
// light) or LightSetF (up to kMaxLights); the overloads below give both the
// same interface, and one light keeps its single-light code.
#pragma once

#include "density.hpp"
#include "ocr_common.hpp"

namespace ocr {

constexpr int kMaxLights = 4;

struct LightSetF {
    int n;  // 1..kMaxLights
    LightF l[kMaxLights];
};

// FP32 area |e_u x e_v| of a light, in the sample specification's operation order.
__device__ inline float light_area32(const LightF &L) {
#pragma clang fp contract(off)
    return sqrtf(__fmaf_rn(L.nlu[2], L.nlu[2], __fmaf_rn(L.nlu[1], L.nlu[1], L.nlu[0] * L.nlu[0])));
}

// The sample point of a pixel and the light it lies on.
__device__ inline void pick_light(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const LightF &L, float y[3],
                                  LightF &chosen) {
    light_point(px, py, s, sd, L, y);
    chosen = L;
}

// Several lights: with u2 = unit24(h[2]) of the sample's hash, the first l
// whose running FP32 sum A_0 + ... + A_l exceeds u2 * A_tot (the last light if
// rounding leaves none); the point on it uses h[0], h[1] as for one light.
__device__ inline void pick_light(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const LightSetF &S, float y[3],
                                  LightF &chosen) {
#pragma clang fp contract(off)
    uint32_t h0 = px, h1 = py, h2 = s, h3 = sd;
    pcg4d(h0, h1, h2, h3);
    float A[kMaxLights], tot = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxLights; ++k) {
        A[k] = k < S.n ? light_area32(S.l[k]) : 0.0f;
        tot = tot + A[k];
    }
    const float u = unit24(h2) * tot;
    float C = 0.0f;
    int l = S.n - 1;
    bool found = false;
#pragma unroll
    for (int k = 0; k < kMaxLights; ++k) {
        if (k < S.n) {
            C = C + A[k];
            if (!found && u < C) {
                l = k;
                found = true;
            }
        }
    }
    // (no runtime index into the set: the lanes select their light's fields)
    chosen = S.l[0];
#pragma unroll
    for (int k = 1; k < kMaxLights; ++k)
        if (k == l) chosen = S.l[k];
    const float a = unit24(h0) - 0.5f;
    const float b = unit24(h1) - 0.5f;
    for (int c = 0; c < 3; ++c) y[c] = __fmaf_rn(b, chosen.ev[c], __fmaf_rn(a, chosen.eu[c], chosen.c[c]));
}

// Per-receiver terms of the shadow density: for one light the light-frame
// terms of recv_shadow, for several the receiver point (the per-light terms
// are recomputed in the density).
struct RecvSet {
    float o[3];
};

__device__ inline RecvShadow recv_of(const float ok[3], const LightF &L) { return recv_shadow(ok, L); }
__device__ inline RecvSet recv_of(const float ok[3], const LightSetF &) { return RecvSet{{ok[0], ok[1], ok[2]}}; }

__device__ inline void recv_store(const RecvShadow &r, float v[3]) {
    v[0] = r.hk;
    v[1] = r.ak;
    v[2] = r.bk;
}
__device__ inline void recv_store(const RecvSet &r, float v[3]) {
    v[0] = r.o[0];
    v[1] = r.o[1];
    v[2] = r.o[2];
}
__device__ inline RecvShadow recv_load(const float v[3], const LightF &) { return RecvShadow{v[0], v[1], v[2]}; }
__device__ inline RecvSet recv_load(const float v[3], const LightSetF &) { return RecvSet{{v[0], v[1], v[2]}}; }

__device__ inline float dens_light(const float w[3], const float nk[3], const RecvShadow &rk, const float nz[3],
                                   const LightF &L) {
    return dens_shadow(w, nk, rk, nz, L);
}

// sum_l J_l chi_l: the union's density times A_tot
__device__ inline float dens_light(const float w[3], const float nk[3], const RecvSet &rk, const float nz[3],
                                   const LightSetF &S) {
    float p = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxLights; ++k)
        if (k < S.n) p += dens_shadow(w, nk, recv_shadow(rk.o, S.l[k]), nz, S.l[k]);
    return p;
}

__device__ inline float front_light(const float o[3], const float n[3], const LightF &L) {
    return front_fraction(o, n, L);
}

__device__ inline float front_light(const float o[3], const float n[3], const LightSetF &S) {
    float f = 0.0f, tot = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxLights; ++k) {
        if (k < S.n) {
            const float a = light_area32(S.l[k]);
            f += a * front_fraction(o, n, S.l[k]);
            tot += a;
        }
    }
    return f / tot;
}

}  // namespace ocr
