// Shadows under the solid-angle definition and direct illumination in the
// occluder domain.
//
// Shadows under the solid-angle definition (the appendix deriving the
// occluder-domain form of Eq. reapp-shadow-definition-solid-angle): the
// target is the visible part of the solid angle Omega_A(x) that the light
// subtends, estimated (Eq. reapp-shadow-solid-angle-estimator) as
//   F_Omega(x_i) - (Area / Omega_A(x_i)) sum_j g_ij p_i(j) / P_i(j),
// with g_ij = <n_y', w_{y'->x_i}> / |x_i - y'|^2 at the light crossing y' of
// the ray from x_i through z_j (the factor C_Omega of Eq.
// reapp-shadow-solid-angle-mis-factor without its per-target part) and
// F_Omega = Omega_front / Omega_A, the part of the light's solid angle in
// front of the receiver's tangent plane.  Samples and densities are those of
// the area definition: the light is still sampled uniformly on its area.
#pragma once

#include "density.hpp"
#include "ocr_common.hpp"

namespace ocr {

// g for the pair vector w = z_j - o_i and the receiver term hk = n_L.(c - o_i)
// (negative on the emitting side); 0 where the ray does not run towards the
// light's plane.  y' = o_i + s w with s = hk / <n_L, w>, so
// |x_i - y'|^2 = s^2 |w|^2 and <n_y', w_{y'->x_i}> = -<n_L, w> / |w|.
__device__ inline float sa_pair_g(const float w[3], float hk, const LightF &L) {
    const float nlw = dot3f(L.nl, w);
    if (!(nlw < 0.0f)) return 0.0f;
    const float d2 = dot3f(w, w);
    const float s = hk * __builtin_amdgcn_rcpf(nlw);
    return -nlw * __builtin_amdgcn_rsqf(d2) * __builtin_amdgcn_rcpf(s * s * d2);
}

// Streaming fan of a convex polygon in the light's plane: vertices arrive
// in order as light coordinates (a, b) (y = c + a e_u + b e_v); each new
// vertex closes the triangle (first, previous, new), whose solid angle at o
// is added by the formula of Van Oosterom and Strackee (IEEE Trans. Biomed.
// Eng. BME-30, 1983):
//   tan(Omega / 2) = |a.(b x c)| / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|).
// For a triangle in the light's plane a.(b x c) = h * D, with
// h = (c - o).(e_u x e_v), the same for every triangle, and D twice its
// signed area in light coordinates, which avoids the cancellation of a
// triple product of three long, nearly parallel vectors.
struct SolidFan {
    float a0, b0, v0[3], l0;
    float ap, bp, vp[3], lp;
    float acc;
    int m;
};

__device__ inline void fan_init(SolidFan &f) {
    f.acc = 0.0f;
    f.m = 0;
}

__device__ inline void fan_add(SolidFan &f, float va, float vb, const float co[3], float h, const LightF &L) {
    float v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = __fmaf_rn(vb, L.ev[k], __fmaf_rn(va, L.eu[k], co[k]));
    const float lv = sqrtf(dot3f(v, v));
    if (f.m == 0) {
        f.a0 = va;
        f.b0 = vb;
#pragma unroll
        for (int k = 0; k < 3; ++k) f.v0[k] = v[k];
        f.l0 = lv;
    } else {
        if (f.m >= 2) {
            const float D = (f.ap - f.a0) * (vb - f.b0) - (f.bp - f.b0) * (va - f.a0);
            const float num = h * fabsf(D);
            const float den = f.l0 * f.lp * lv + dot3f(f.v0, f.vp) * lv + dot3f(f.v0, v) * f.lp + dot3f(f.vp, v) * f.l0;
            f.acc += 2.0f * atan2f(num, den);
        }
    }
    f.ap = va;
    f.bp = vb;
#pragma unroll
    for (int k = 0; k < 3; ++k) f.vp[k] = v[k];
    f.lp = lv;
    ++f.m;
}

// Omega_A (the whole one-sided light) and Omega_front (its part with
// <n, y - o> > 0) at o; both 0 when o is not on the emitting side.  With the
// whole light in front both sums take the same triangles: F_Omega = 1 exactly.
__device__ inline void emitter_solid_angles(const float o[3], const float n[3], const LightF &L, float &all,
                                            float &front) {
    all = 0.0f;
    front = 0.0f;
    const float co[3] = {L.c[0] - o[0], L.c[1] - o[1], L.c[2] - o[2]};
    if (!(dot3f(L.nl, co) < 0.0f)) return;
    const float h = fabsf(dot3f(L.nlu, co));
    const float ca[4] = {-0.5f, 0.5f, 0.5f, -0.5f};
    const float cb[4] = {-0.5f, -0.5f, 0.5f, 0.5f};
    const float f0 = dot3f(n, co), fu = dot3f(n, L.eu), fv = dot3f(n, L.ev);
    SolidFan fa, ff;
    fan_init(fa);
    fan_init(ff);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const float ga = f0 + ca[k] * fu + cb[k] * fv;
        const float gb = f0 + ca[k1] * fu + cb[k1] * fv;
        fan_add(fa, ca[k], cb[k], co, h, L);
        if (ga > 0.0f) fan_add(ff, ca[k], cb[k], co, h, L);
        if ((ga > 0.0f) != (gb > 0.0f)) {
            const float t = ga / (ga - gb);
            fan_add(ff, ca[k] + t * (ca[k1] - ca[k]), cb[k] + t * (cb[k1] - cb[k]), co, h, L);
        }
    }
    all = fa.acc;
    front = ff.acc;
}

// Estimate of one target from its accumulated sum_j g_ij p_i(j) / P_i(j).
__device__ inline float sa_estimate(const float o[3], const float n[3], const LightF &L, float Bg) {
    float all, front;
    emitter_solid_angles(o, n, L, all, front);
    if (!(all > 0.0f)) return 0.0f;
    const float area = sqrtf(dot3f(L.nlu, L.nlu));
    return front / all - (area / all) * Bg;
}

// ---------------------------------------------------------------------------
// Occluder-domain direct illumination (the appendix deriving Eq.
// reapp-di-occluder-domain-compact) for a Lambertian receiver of albedo rho
// under the one-sided emitter of radiance L_e:
//   L_DI(x_i) = (rho L_e / pi) (E(x_i) - Area sum_j gd_ij p_i(j) / P_i(j)),
// gd_ij = cos+_x <n_y', w_{y'->x_i}> / |x_i - y'|^2 (the factor C_DI of Eq.
// reapp-di-general-mis-factor for uniform light sampling, without its
// per-target part) and E the irradiance of the unit-radiance light's part in
// front of the tangent plane (the unshadowed term, Lambert's polygon formula).
// ---------------------------------------------------------------------------

// gd for the pair vector w = z_j - o_i, the receiver normal n and hk.
__device__ inline float di_pair_g(const float w[3], const float n[3], float hk, const LightF &L) {
    const float nw = dot3f(n, w);
    if (!(nw > 0.0f)) return 0.0f;
    return nw * __builtin_amdgcn_rsqf(dot3f(w, w)) * sa_pair_g(w, hk, L);
}

// Streaming Lambert polygon formula, E = 1/2 |sum_k theta_k <n, c_k / |c_k|>|,
// c_k = q_k x q_{k+1}, over vertices arriving in order as light coordinates.
// The cross product of the two long vertex vectors is taken as
// co x (short edge) + (a_k b_{k+1} - b_k a_{k+1}) (e_u x e_v), co = c - o,
// which avoids their cancellation.
struct LambertFan {
    float a0, b0, v0[3];
    float ap, bp, vp[3];
    float acc;
    int m;
};

__device__ inline void lambert_edge(float &acc, float a1, float b1, const float v1[3], float a2, float b2,
                                    const float v2[3], const float co[3], const float n[3], const LightF &L) {
    float e[3], c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = (a2 - a1) * L.eu[k] + (b2 - b1) * L.ev[k];
    const float t = a1 * b2 - b1 * a2;
    c[0] = __fmaf_rn(t, L.nlu[0], co[1] * e[2] - co[2] * e[1]);
    c[1] = __fmaf_rn(t, L.nlu[1], co[2] * e[0] - co[0] * e[2]);
    c[2] = __fmaf_rn(t, L.nlu[2], co[0] * e[1] - co[1] * e[0]);
    const float lc = sqrtf(dot3f(c, c));
    if (!(lc > 0.0f)) return;
    acc += atan2f(lc, dot3f(v1, v2)) * dot3f(n, c) / lc;
}

__device__ inline void lfan_add(LambertFan &f, float va, float vb, const float co[3], const float n[3],
                                const LightF &L) {
    float v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = __fmaf_rn(vb, L.ev[k], __fmaf_rn(va, L.eu[k], co[k]));
    if (f.m == 0) {
        f.a0 = va;
        f.b0 = vb;
#pragma unroll
        for (int k = 0; k < 3; ++k) f.v0[k] = v[k];
    } else {
        lambert_edge(f.acc, f.ap, f.bp, f.vp, va, vb, v, co, n, L);
    }
    f.ap = va;
    f.bp = vb;
#pragma unroll
    for (int k = 0; k < 3; ++k) f.vp[k] = v[k];
    ++f.m;
}

// E(o): the irradiance of the unit-radiance light's part with <n, y - o> > 0
// (0 when o is not on the emitting side).
__device__ inline float emitter_irradiance(const float o[3], const float n[3], const LightF &L) {
    const float co[3] = {L.c[0] - o[0], L.c[1] - o[1], L.c[2] - o[2]};
    if (!(dot3f(L.nl, co) < 0.0f)) return 0.0f;
    const float ca[4] = {-0.5f, 0.5f, 0.5f, -0.5f};
    const float cb[4] = {-0.5f, -0.5f, 0.5f, 0.5f};
    const float f0 = dot3f(n, co), fu = dot3f(n, L.eu), fv = dot3f(n, L.ev);
    LambertFan f;
    f.acc = 0.0f;
    f.m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const float ga = f0 + ca[k] * fu + cb[k] * fv;
        const float gb = f0 + ca[k1] * fu + cb[k1] * fv;
        if (ga > 0.0f) lfan_add(f, ca[k], cb[k], co, n, L);
        if ((ga > 0.0f) != (gb > 0.0f)) {
            const float t = ga / (ga - gb);
            lfan_add(f, ca[k] + t * (ca[k1] - ca[k]), cb[k] + t * (cb[k1] - cb[k]), co, n, L);
        }
    }
    if (f.m < 3) return 0.0f;
    lambert_edge(f.acc, f.ap, f.bp, f.vp, f.a0, f.b0, f.v0, co, n, L);  // closing edge
    return 0.5f * fabsf(f.acc);
}

// Estimate of one target from its accumulated sum_j gd_ij p_i(j) / P_i(j);
// scale = rho L_e / pi.
__device__ inline float di_estimate(const float o[3], const float n[3], const LightF &L, float Bg, float scale) {
    const float area = sqrtf(dot3f(L.nlu, L.nlu));
    return scale * (emitter_irradiance(o, n, L) - area * Bg);
}

}  // namespace ocr
