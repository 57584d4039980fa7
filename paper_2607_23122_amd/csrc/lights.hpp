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
//
// A light can also be sampled from a general emitter-area density p_A(y | x)
// (LightBilinF below); its samples, densities and estimator factors follow it.
#pragma once

#include <type_traits>

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

// The sample point of a pixel with receiver point o and the light it lies on.
__device__ inline void pick_light(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const LightF &L, const float *,
                                  float y[3], LightF &chosen) {
    light_point(px, py, s, sd, L, y);
    chosen = L;
}

// Several lights: with u2 = unit24(h[2]) of the sample's hash, the first l
// whose running FP32 sum A_0 + ... + A_l exceeds u2 * A_tot (the last light if
// rounding leaves none); the point on it uses h[0], h[1] as for one light.
__device__ inline void pick_light(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const LightSetF &S,
                                  const float *, float y[3], LightF &chosen) {
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

// One light sampled from the receiver-dependent bilinear density: over the
// light coordinates (a, b) it interpolates the corner weights 1 / |o - y_k|^3
// (the shape of the solid-angle density cos(theta_y) / |o - y|^2 at the
// corners: cos(theta_y) = h / |o - y| with one height h for the whole
// rectangle), normalised to unit mass.  Reuse evaluates it at every receiver
// of a candidate: the occluder density p_A(y' | x) J chi_A = q_x(y') (1 /
// Area) J chi_A with q_x = Area p_A, and every estimator factor divides by
// q_x(y') (the appendix's general area-domain sampling density).
struct LightBilinF : LightF {};

template <class LT>
constexpr bool kBilinear = std::is_same<LT, LightBilinF>::value;

// FP32 corner weights of receiver point o (sample specification): corners
// k = 0..3 at (a, b) = (-1/2,-1/2), (1/2,-1/2), (-1/2,1/2), (1/2,1/2);
// |o - y_k|^2 clamped below at 2^-40; divided by their maximum.  Division
// and sqrtf are correctly rounded.
__device__ inline void bilinear_weights(const float o[3], const LightF &L, float w[4]) {
#pragma clang fp contract(off)
    float m = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float ak = (k & 1) ? 0.5f : -0.5f, bk = (k & 2) ? 0.5f : -0.5f;
        float d[3];
        for (int c = 0; c < 3; ++c) d[c] = o[c] - __fmaf_rn(bk, L.ev[c], __fmaf_rn(ak, L.eu[c], L.c[c]));
        const float d2 = fmaxf(__fmaf_rn(d[2], d[2], __fmaf_rn(d[1], d[1], d[0] * d[0])), 0x1p-40f);
        w[k] = 1.0f / (d2 * sqrtf(d2));
        m = fmaxf(m, w[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = w[k] / m;
}

// Inverse CDF of the density proportional to (1 - t) e0 + t e1 on [0, 1]:
// the root of (e1 - e0) t^2 + 2 e0 t = xi (e0 + e1), in the form without
// cancellation, capped at 1.
__device__ inline float sample_linear(float xi, float e0, float e1) {
#pragma clang fp contract(off)
    const float r = sqrtf((1.0f - xi) * (e0 * e0) + xi * (e1 * e1));
    const float den = e0 + r;
    if (!(den > 0.0f)) return 0.0f;
    return fminf(xi * (e0 + e1) / den, 1.0f);
}

// v = b + 1/2 from its marginal (linear between the corner sums at v = 0 and
// v = 1) with h[1], then u = a + 1/2 from the conditional at v (linear between
// the edge weights interpolated at v) with h[0]; the point as for uniform
// sampling.
__device__ inline void pick_light(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const LightBilinF &L,
                                  const float o[3], float y[3], LightF &chosen) {
#pragma clang fp contract(off)
    uint32_t h0 = px, h1 = py, h2 = s, h3 = sd;
    pcg4d(h0, h1, h2, h3);
    float w[4];
    bilinear_weights(o, L, w);
    const float tv = sample_linear(unit24(h1), w[0] + w[1], w[2] + w[3]);
    const float f0 = (1.0f - tv) * w[0] + tv * w[2];
    const float f1 = (1.0f - tv) * w[1] + tv * w[3];
    const float tu = sample_linear(unit24(h0), f0, f1);
    const float a = tu - 0.5f, b = tv - 0.5f;
    for (int c = 0; c < 3; ++c) y[c] = __fmaf_rn(b, L.ev[c], __fmaf_rn(a, L.eu[c], L.c[c]));
    chosen = L;
}

// Receiver terms of the bilinear density: the light-frame terms of
// recv_shadow and q_x(a, b) = 1 + a qa + b qb + a b qab, the interpolation of
// the corner values 4 w_k / sum w (mean 1 over the rectangle).
struct RecvBilin {
    float hk, ak, bk, qa, qb, qab;
};

__device__ inline RecvBilin recv_of(const float ok[3], const LightBilinF &L) {
#pragma clang fp contract(off)
    const RecvShadow r = recv_shadow(ok, L);
    float w[4];
    bilinear_weights(ok, L, w);
    const float k = 4.0f / ((w[0] + w[1]) + (w[2] + w[3]));
    RecvBilin q;
    q.hk = r.hk;
    q.ak = r.ak;
    q.bk = r.bk;
    q.qa = 0.5f * k * ((w[1] + w[3]) - (w[0] + w[2]));
    q.qb = 0.5f * k * ((w[2] + w[3]) - (w[0] + w[1]));
    q.qab = k * ((w[3] - w[1]) - (w[2] - w[0]));
    return q;
}

__device__ inline float bilinear_q(const RecvBilin &r, float a, float b) {
    return __fmaf_rn(a, __fmaf_rn(b, r.qab, r.qa), __fmaf_rn(b, r.qb, 1.0f));
}

__device__ inline float dens_light(const float w[3], const float nk[3], const RecvBilin &rk, const float nz[3],
                                   const LightBilinF &L) {
    float ab[2];
    const float p = dens_shadow_t<true>(w, nk, RecvShadow{rk.hk, rk.ak, rk.bk}, nz, L, ab);
    return p > 0.0f ? p * bilinear_q(rk, ab[0], ab[1]) : 0.0f;
}

// 1 / q_x(y'(x, z)) for a target x whose density of z is positive: the
// factor that turns p_A J chi_A back into the target's (1 / Area) J chi_A.
__device__ inline float inv_bilinear_q(const float w[3], const RecvBilin &rk, const LightF &L) {
#pragma clang fp contract(off)
    const float s = rk.hk * __builtin_amdgcn_rcpf(dot3f(L.nl, w));
    const float a = __fmaf_rn(s, dot3f(L.uhat, w), rk.ak);
    const float b = __fmaf_rn(s, dot3f(L.vhat, w), rk.bk);
    return __builtin_amdgcn_rcpf(bilinear_q(rk, a, b));
}

// Floats of a receiver's light terms in LDS.
template <class LT>
constexpr int kRecvFloats = kBilinear<LT> ? 6 : 3;

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
__device__ inline void recv_store(const RecvBilin &r, float v[6]) {
    v[0] = r.hk;
    v[1] = r.ak;
    v[2] = r.bk;
    v[3] = r.qa;
    v[4] = r.qb;
    v[5] = r.qab;
}
__device__ inline RecvShadow recv_load(const float v[3], const LightF &) { return RecvShadow{v[0], v[1], v[2]}; }
__device__ inline RecvSet recv_load(const float v[3], const LightSetF &) { return RecvSet{{v[0], v[1], v[2]}}; }
__device__ inline RecvBilin recv_load(const float v[6], const LightBilinF &) {
    return RecvBilin{v[0], v[1], v[2], v[3], v[4], v[5]};
}

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
