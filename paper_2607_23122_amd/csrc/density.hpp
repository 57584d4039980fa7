// FP32 pair densities shared by the validation and reuse kernels, so both
// take identical support decisions for every (receiver, candidate) pair.
//
// Only ratios of densities of the same candidate enter the estimator (the
// balance-heuristic weight of Eq. generic-mis-weight), so constant factors
// common to all receivers -- 1/pi for AO, 1/Area for the light -- are dropped.
//
// Geometry is relative: the vector from receiver k to candidate j is
// w = (o_j - o_k) + dz_j, where dz_j = z_j - o_j is stored by the trace.  Both
// terms are small and accurately rounded, which keeps w accurate to a few
// ulps of |w| even far from the world origin.
#pragma once

#include "ocr_common.hpp"

namespace ocr {

__device__ inline float dot3f(const float a[3], const float b[3]) {
#pragma clang fp contract(off)
    return __fmaf_rn(a[2], b[2], __fmaf_rn(a[1], b[1], a[0] * b[0]));
}

__device__ inline void rel_vec(const float oj[3], const float ok[3], const float dzj[3], float w[3]) {
#pragma clang fp contract(off)
    w[0] = (oj[0] - ok[0]) + dzj[0];
    w[1] = (oj[1] - ok[1]) + dzj[1];
    w[2] = (oj[2] - ok[2]) + dzj[2];
}

// p_AO (Eq. ao-pdf) without the first-hit factor, times pi:
//   <n_k, w> <n_z, -w> / |w|^4  with |w| <= R, both cosines positive.
__device__ inline float dens_ao(const float w[3], const float nk[3], const float nz[3], float R2) {
#pragma clang fp contract(off)
    float nw = dot3f(nk, w);
    float zw = dot3f(nz, w);
    float d2 = dot3f(w, w);
    bool ok = nw > 0.0f && zw < 0.0f && d2 <= R2;
    float p = (nw * -zw) * __builtin_amdgcn_rcpf(d2 * d2);
    return ok ? p : 0.0f;
}

// Per-receiver terms of the shadow density: hk = n_L.(c - o_k) (negative for
// a receiver on the emitting side), ak = (o_k - c).e_u/|e_u|^2,
// bk = (o_k - c).e_v/|e_v|^2.
struct RecvShadow {
    float hk, ak, bk;
};

__device__ inline RecvShadow recv_shadow(const float ok[3], const LightF &L) {
#pragma clang fp contract(off)
    float oc[3] = {ok[0] - L.c[0], ok[1] - L.c[1], ok[2] - L.c[2]};
    RecvShadow r;
    r.hk = -dot3f(L.nl, oc);
    r.ak = dot3f(L.uhat, oc);
    r.bk = dot3f(L.vhat, oc);
    return r;
}

// p_Sh (Eq. shadow-pdf) without the first-hit factor, times Area:
// J = <n_z, w_{z->x}> |x - y'|^2 / (<n_L, w_{y'->x}> |x - z|^2) = s^2 <n_z,-w> / <n_L,-w>
// where y' = o_k + s w is the ray's crossing of the light plane; support:
// z in front of the receiver's tangent plane, ray towards the emitting face,
// s > 1 (the light beyond z) and y' inside the rectangle.
// AB: also return the light coordinates (a, b) of y' in ab[0..1], for
// densities that vary over the light (without it the coordinates are only
// tested, and the tests may be skipped once one fails).
template <bool AB>
__device__ inline float dens_shadow_t(const float w[3], const float nk[3], const RecvShadow &rk, const float nz[3],
                                      const LightF &L, float *ab) {
#pragma clang fp contract(off)
    float front = dot3f(nk, w);
    float nlw = dot3f(L.nl, w);
    float zw = dot3f(nz, w);
    // one hardware reciprocal (1 ulp) for s and the ratio; thresholds on s
    // move by an ulp at most
    float inl = __builtin_amdgcn_rcpf(nlw);
    float s = rk.hk * inl;
    float a = __fmaf_rn(s, dot3f(L.uhat, w), rk.ak);
    float b = __fmaf_rn(s, dot3f(L.vhat, w), rk.bk);
    bool ok = front > 0.0f && nlw < 0.0f && zw < 0.0f && s > 1.0f && fabsf(a) <= 0.5f && fabsf(b) <= 0.5f;
    float p = (s * s) * (zw * inl);
    if constexpr (AB) {
        ab[0] = a;
        ab[1] = b;
    }
    return ok ? p : 0.0f;
}

__device__ inline float dens_shadow(const float w[3], const float nk[3], const RecvShadow &rk, const float nz[3],
                                    const LightF &L) {
    return dens_shadow_t<false>(w, nk, rk, nz, L, nullptr);
}

// Fraction of the light rectangle in front of the tangent plane of (o, n):
// the unit square (a, b) in [-1/2, 1/2]^2 clipped by the half-plane
// f0 + a fu + b fv > 0 with f0 = n.(c - o), fu = n.e_u, fv = n.e_v; zero when
// the receiver is not on the emitting side.
__device__ inline float front_fraction(const float o[3], const float n[3], const LightF &L) {
    float oc[3] = {o[0] - L.c[0], o[1] - L.c[1], o[2] - L.c[2]};
    if (!(dot3f(L.nl, oc) > 0.0f)) return 0.0f;
    float f0 = -dot3f(n, oc), fu = dot3f(n, L.eu), fv = dot3f(n, L.ev);
    const float ca[4] = {-0.5f, 0.5f, 0.5f, -0.5f};
    const float cb[4] = {-0.5f, -0.5f, 0.5f, 0.5f};
    // Walk the square's edges emitting the clipped polygon's vertices in
    // order and accumulate the shoelace sum on the fly (first and previous
    // vertex only: no arrays, so nothing goes to private memory).
    float area = 0.0f, a0 = 0.0f, b0 = 0.0f, ap = 0.0f, bp = 0.0f;
    int m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const float fa = f0 + ca[k] * fu + cb[k] * fv;
        const float fb = f0 + ca[k1] * fu + cb[k1] * fv;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            float va, vb;
            bool emit;
            if (e == 0) {
                emit = fa > 0.0f;
                va = ca[k];
                vb = cb[k];
            } else {
                emit = (fa > 0.0f) != (fb > 0.0f);
                const float t = emit ? fa / (fa - fb) : 0.0f;
                va = ca[k] + t * (ca[k1] - ca[k]);
                vb = cb[k] + t * (cb[k1] - cb[k]);
            }
            if (emit) {
                if (m == 0) {
                    a0 = va;
                    b0 = vb;
                } else {
                    area += ap * vb - va * bp;
                }
                ap = va;
                bp = vb;
                ++m;
            }
        }
    }
    if (m > 0) area += ap * b0 - a0 * bp;
    return 0.5f * fabsf(area);
}

}  // namespace ocr
