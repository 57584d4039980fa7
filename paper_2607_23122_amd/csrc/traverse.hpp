// Software ray traversal of the 4-wide BVH on gfx950 (no ray-tracing units).
//
// One lane per ray.  The traversal stack lives in LDS, one column per lane
// (entry k of lane t at [k * blockDim + t], so lanes at equal depth hit
// distinct banks), kStackLds entries deep and nothing in private memory: a
// walk that would push past it stops and reports the overflow, and the
// caller decides that ray with the wave-coherent walk below (its stack, one
// per wave, holds the 3 depth + 1 entries any walk of the tree can need).
// Child boxes are tested with a conservative slab test (one FMA per plane,
// offsets and far distances widened so no box that the ray touches is
// skipped; see TRay), and
// triangles with the watertight test of Woop, Benthin and Wald (JCGT 2013):
// the edge functions are 2x2 determinants of sheared vertex coordinates,
// evaluated without contraction and recomputed in FP64 when one is exactly
// zero, so rays through shared edges and vertices never slip between
// triangles.
#pragma once

#include "ocr_common.hpp"

namespace ocr {

// Slab test with one FMA per plane: the distance to the plane x_c = l is
// l * inv_c + off, with off = -o_c * inv_c moved by eps_c towards the ray for
// the near plane of the axis and away from it for the far plane (which plane
// is near follows the sign of inv_c).  Against the exact (l - o_c) / d_c the
// computed distance errs by at most about 2^-23 |o_c inv_c| (the rounded
// product and offset) plus 2^-22 of the distance itself (the rounded 1/d_c
// and FMA).  Only boxes entered before tmax can matter, so the relative part
// is at most 2^-22 tmax there, and eps_c = 2^-21 |o_c inv_c| + 2^-20 tmax
// covers both with margin.  So the test stays conservative: no box the ray
// enters is skipped, and hits do not depend on it.
struct TRay {
    float o[3];
    float inv[3];   // 1 / d with zero components replaced by +-1e-20
    float off_lo[3], off_hi[3];  // plane offsets for the box's low / high planes
    float m0[3], m1[3], m2[3];  // shear rows: x' = m0.(p-o), y' = m1.(p-o), z' = m2.(p-o)
    uint32_t ign0, ign1;
};

// tmax: the end of the ray's t range (sets the relative part of the slack).
__device__ inline void make_ray(const float o[3], const float d[3], uint32_t ign0, uint32_t ign1, float tmax,
                                TRay &r) {
    for (int c = 0; c < 3; ++c) {
        r.o[c] = o[c];
        float dc = fabsf(d[c]) < 1e-20f ? copysignf(1e-20f, d[c]) : d[c];
        r.inv[c] = 1.0f / dc;
        const float oi = o[c] * r.inv[c];
        const float eps = __fmaf_rn(0x1p-21f, fabsf(oi), 0x1p-20f * tmax);
        // inv > 0: the low plane is near (offset lowered), the high plane far (raised)
        const float s = r.inv[c] > 0.0f ? eps : -eps;
        r.off_lo[c] = -oi - s;
        r.off_hi[c] = -oi + s;
    }
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    if (d[kz] < 0.0f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    float dkz = d[kz];
    float Sx = d[kx] / dkz, Sy = d[ky] / dkz, Sz = 1.0f / dkz;
    for (int c = 0; c < 3; ++c) {
        r.m0[c] = (c == kx ? 1.0f : 0.0f) - (c == kz ? Sx : 0.0f);
        r.m1[c] = (c == ky ? 1.0f : 0.0f) - (c == kz ? Sy : 0.0f);
        r.m2[c] = c == kz ? Sz : 0.0f;
    }
    r.ign0 = ign0;
    r.ign1 = ign1;
}

// Watertight triangle test.  Returns the ray parameter t (> 0) or -1.
__device__ inline float tri_hit(const TRay &r, const float4 &v0, const float4 &v1, const float4 &v2) {
#pragma clang fp contract(off)
    float A[3] = {v0.x - r.o[0], v0.y - r.o[1], v0.z - r.o[2]};
    float B[3] = {v1.x - r.o[0], v1.y - r.o[1], v1.z - r.o[2]};
    float C[3] = {v2.x - r.o[0], v2.y - r.o[1], v2.z - r.o[2]};
    float Ax = __fmaf_rn(r.m0[2], A[2], __fmaf_rn(r.m0[1], A[1], r.m0[0] * A[0]));
    float Ay = __fmaf_rn(r.m1[2], A[2], __fmaf_rn(r.m1[1], A[1], r.m1[0] * A[0]));
    float Bx = __fmaf_rn(r.m0[2], B[2], __fmaf_rn(r.m0[1], B[1], r.m0[0] * B[0]));
    float By = __fmaf_rn(r.m1[2], B[2], __fmaf_rn(r.m1[1], B[1], r.m1[0] * B[0]));
    float Cx = __fmaf_rn(r.m0[2], C[2], __fmaf_rn(r.m0[1], C[1], r.m0[0] * C[0]));
    float Cy = __fmaf_rn(r.m1[2], C[2], __fmaf_rn(r.m1[1], C[1], r.m1[0] * C[0]));
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        double u = (double)Cx * (double)By - (double)Cy * (double)Bx;
        double v = (double)Ax * (double)Cy - (double)Ay * (double)Cx;
        double w = (double)Bx * (double)Ay - (double)By * (double)Ax;
        U = (float)u;
        V = (float)v;
        W = (float)w;
        if ((u < 0.0 || v < 0.0 || w < 0.0) && (u > 0.0 || v > 0.0 || w > 0.0)) return -1.0f;
    } else if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) {
        return -1.0f;
    }
    float det = U + V + W;
    if (det == 0.0f) return -1.0f;
    float Az = __fmaf_rn(r.m2[2], A[2], __fmaf_rn(r.m2[1], A[1], r.m2[0] * A[0]));
    float Bz = __fmaf_rn(r.m2[2], B[2], __fmaf_rn(r.m2[1], B[1], r.m2[0] * B[0]));
    float Cz = __fmaf_rn(r.m2[2], C[2], __fmaf_rn(r.m2[1], C[1], r.m2[0] * C[0]));
    float T = __fmaf_rn(W, Cz, __fmaf_rn(V, Bz, U * Az));
    float t = T / det;
    return t > 0.0f ? t : -1.0f;
}

// Work of BVH walks: walks, node visits, box tests and triangle tests (a
// test of one ray or segment counts once).
struct WalkStats {
    uint64_t walks = 0, nodes = 0, box_tests = 0, tri_tests = 0, segments = 0;
};

// Result of a closest-hit query: `tri` is the scene triangle index or
// OCR_HIT_MISS, `leaf_tri` its position in the leaf-ordered array.
struct Hit {
    float t;
    uint32_t tri;
    uint32_t leaf_tri;
};

// Closest hit over t in (0, tmax] (INCLUSIVE) or (0, tmax); with ANY, the
// first hit found over (0, tmax) ends the query.  Equal distances resolve
// to the smaller scene triangle index.  With COUNT the walk's work is added
// to *ws (a separate instantiation; the result is the same).  If a push would
// take the stack past kStackLds entries the walk stops, sets `overflow` and
// its result is not to be used.  The walk starts at `start` (the root, or a
// node below which every triangle the ray can meet lies: wave_entry_node).
template <bool ANY, bool INCLUSIVE, bool COUNT = false>
__device__ inline Hit traverse(const DeviceBVH &bvh, const TRay &r, float tmax, uint32_t *lds_stack, int stride,
                               bool &overflow, WalkStats *ws = nullptr, uint32_t start = 0) {
    if (COUNT) ws->walks += 1;
    Hit h;
    h.t = tmax;
    h.tri = OCR_HIT_MISS;
    h.leaf_tri = 0;
    int sp = 0;
    uint32_t node = start;
    const float grow = 1.0f + 0x1p-20f;
    for (;;) {
        if (!(node & kLeafBit)) {
            const float4 *np = reinterpret_cast<const float4 *>(bvh.nodes + node);
            float4 lx = np[0], hx = np[1], ly = np[2], hy = np[3], lz = np[4], hz = np[5];
            uint4 ch = reinterpret_cast<const uint4 *>(np)[6];
            if (COUNT) {
                // a useful box test per non-empty child
                ws->nodes += 1;
                ws->box_tests += (ch.x != kEmpty) + (ch.y != kEmpty) + (ch.z != kEmpty) + (ch.w != kEmpty);
            }
            float lxs[4] = {lx.x, lx.y, lx.z, lx.w}, hxs[4] = {hx.x, hx.y, hx.z, hx.w};
            float lys[4] = {ly.x, ly.y, ly.z, ly.w}, hys[4] = {hy.x, hy.y, hy.z, hy.w};
            float lzs[4] = {lz.x, lz.y, lz.z, lz.w}, hzs[4] = {hz.x, hz.y, hz.z, hz.w};
            uint32_t chs[4] = {ch.x, ch.y, ch.z, ch.w};
            float tn[4];
            uint32_t cand[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float t0x = __fmaf_rn(lxs[i], r.inv[0], r.off_lo[0]), t1x = __fmaf_rn(hxs[i], r.inv[0], r.off_hi[0]);
                float t0y = __fmaf_rn(lys[i], r.inv[1], r.off_lo[1]), t1y = __fmaf_rn(hys[i], r.inv[1], r.off_hi[1]);
                float t0z = __fmaf_rn(lzs[i], r.inv[2], r.off_lo[2]), t1z = __fmaf_rn(hzs[i], r.inv[2], r.off_hi[2]);
                float tnear = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
                float tfar = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
                tfar = fminf(tfar, h.t * grow);
                bool hit = tnear <= tfar && chs[i] != kEmpty;
                tn[i] = hit ? tnear : INFINITY;
                cand[i] = chs[i];
            }
            // sort the four (distance, child) pairs, nearest first (5 compare-exchanges)
#define OCR_CSWAP(a, b)                                      \
    if (tn[b] < tn[a]) {                                     \
        float tt = tn[a]; tn[a] = tn[b]; tn[b] = tt;         \
        uint32_t cc = cand[a]; cand[a] = cand[b]; cand[b] = cc; \
    }
            OCR_CSWAP(0, 1)
            OCR_CSWAP(2, 3)
            OCR_CSWAP(0, 2)
            OCR_CSWAP(1, 3)
            OCR_CSWAP(1, 2)
#undef OCR_CSWAP
            if (tn[0] < INFINITY) {
                // push the farther ones (farthest first), continue with the nearest
#pragma unroll
                for (int k = 3; k >= 1; --k) {
                    if (tn[k] < INFINITY) {
                        if (sp == kStackLds) {
                            overflow = true;
                            return h;
                        }
                        lds_stack[sp * stride] = cand[k];
                        ++sp;
                    }
                }
                node = cand[0];
                continue;
            }
        } else {
            uint32_t first = node & 0x07FFFFFFu;
            uint32_t count = ((node >> 27) & 0xFu) + 1u;
            for (uint32_t q = 0; q < count; ++q) {
                const float4 *tp = bvh.tris + 3 * (size_t)(first + q);
                float4 v0 = tp[0], v1 = tp[1], v2 = tp[2];
                uint32_t id = __float_as_uint(v0.w);
                if (id == r.ign0 || id == r.ign1) continue;
                if (COUNT) ws->tri_tests += 1;
                float t = tri_hit(r, v0, v1, v2);
                if (!(t > 0.0f)) continue;
                bool take;
                if (ANY) {
                    take = t < tmax;
                } else if (t < h.t) {
                    take = true;
                } else if (t == h.t) {
                    take = h.tri == OCR_HIT_MISS ? INCLUSIVE : id < h.tri;
                } else {
                    take = false;
                }
                if (take) {
                    h.t = t;
                    h.tri = id;
                    h.leaf_tri = first + q;
                    if (ANY) return h;
                }
            }
        }
        if (sp == 0) break;
        --sp;
        node = lds_stack[sp * stride];
    }
    return h;
}

// Unit geometric normal of a leaf-ordered triangle, facing against d.
__device__ inline void oriented_normal(const DeviceBVH &bvh, uint32_t leaf_tri, const float d[3], float n[3]) {
    const float4 *tp = bvh.tris + 3 * (size_t)leaf_tri;
    float4 a = tp[0], b = tp[1], c = tp[2];
    float e1[3] = {b.x - a.x, b.y - a.y, b.z - a.z};
    float e2[3] = {c.x - a.x, c.y - a.y, c.z - a.z};
    float x = e1[1] * e2[2] - e1[2] * e2[1];
    float y = e1[2] * e2[0] - e1[0] * e2[2];
    float z = e1[0] * e2[1] - e1[1] * e2[0];
    float inv = rsqrtf(x * x + y * y + z * z);
    float s = (x * d[0] + y * d[1] + z * d[2]) > 0.0f ? -inv : inv;
    n[0] = x * s;
    n[1] = y * s;
    n[2] = z * s;
}

}  // namespace ocr

namespace ocr {

// Read-only view of the BVH in the constant address space: with a
// wave-uniform index, node and triangle fetches become scalar loads.
typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const uint32_t cuint;

__device__ inline float wave_fmin(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fminf(v, __shfl_xor(v, d));
    return v;
}
__device__ inline float wave_fmax(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d));
    return v;
}

// A value the wave holds in every lane, as a scalar.
__device__ inline float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Where walks of segments inside the wave-uniform box [ulo, uhi] may start.
// The box, padded, is U; from the root the descent goes on while exactly one
// child box of the node overlaps U and that child is not a leaf.  A triangle
// that meets a segment holds a point of U, so each of its ancestors' boxes
// overlaps U: at every node of the descent the triangle's ancestor is the one
// overlapping child, and the triangle lies below the node returned.  The
// padding (1e-4 of the coordinates and of U's extent) is far above the
// rounding of the segment ends and of the triangle test's distance.
__device__ inline uint32_t entry_node(const DeviceBVH &bvh, const float ulo[3], const float uhi[3]) {
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float l = ulo[a], h = uhi[a];
        const float pad = 1e-4f * (fmaxf(fabsf(l), fabsf(h)) + (h - l)) + 1e-6f;
        lo[a] = uniform_f(l - pad);
        hi[a] = uniform_f(h + pad);
    }
    uint32_t node = 0;
    if (!(lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2])) return node;  // no segment
    for (int lev = 0; lev < kMaxDepth; ++lev) {
        const cfloat *f = (const cfloat *)(bvh.nodes + node);
        const cuint *c = (const cuint *)(bvh.nodes + node);
        int n = 0;
        uint32_t only = kEmpty;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool ov = c[24 + i] != kEmpty && f[i] <= hi[0] && f[4 + i] >= lo[0] && f[8 + i] <= hi[1] &&
                            f[12 + i] >= lo[1] && f[16 + i] <= hi[2] && f[20 + i] >= lo[2];
            n += ov ? 1 : 0;
            only = ov ? c[24 + i] : only;
        }
        if (n != 1 || (only & kLeafBit)) break;
        node = only;
    }
    return node;
}

// The same for the union of the lanes' segment boxes slo/shi (empty, +inf /
// -inf, for a lane without a segment); every lane calls it.
__device__ inline uint32_t wave_entry_node(const DeviceBVH &bvh, const float slo[3], const float shi[3]) {
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = uniform_f(wave_fmin(slo[a]));
        hi[a] = uniform_f(wave_fmax(shi[a]));
    }
    return entry_node(bvh, lo, hi);
}

// Wave-coherent any-hit traversal of up to NR segments per lane.  Every lane
// of the wave must call it (wave-uniform control flow); slots with
// want[q] == false only ride along.  The wave walks one node order -- the
// union of its active segments' paths -- from a wave-uniform stack in LDS
// (`wstack`, kStackTotal entries for this wave); node and triangle fetches
// use a wave-uniform index (scalar loads); each lane tests its own segments
// against the shared node's four boxes and the leaf's triangles and drops a
// segment as soon as it is blocked.  blocked[q] reports segment q (t in
// (0, tmax)).
// Work counters of a walk (wave-uniform): node visits, and box / triangle
// tests performed for active segments (lane-tests).
template <int NR>
__device__ inline void traverse_wave_any(const DeviceBVH &bvh, const TRay (&r)[NR], float tmax,
                                         const bool (&want)[NR], bool (&blocked)[NR], uint32_t *wstack,
                                         WalkStats &st, uint32_t start = 0) {
    bool active[NR];
    // the active lanes of each segment set as a wave-uniform mask, kept in
    // step with active[] (box-test ballots are masked with it)
    unsigned long long amask[NR];
    unsigned long long any = 0ull;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        active[q] = want[q];
        blocked[q] = false;
        amask[q] = wave_ballot(active[q]);
        any |= amask[q];
    }
    if (any == 0ull) return;
    st.walks += 1;
    const float grow = 1.0f + 0x1p-20f;
    int sp = 0;
    uint32_t node = start;  // the root, or a wave_entry_node of the segments
    for (;;) {
        if (!(node & kLeafBit)) {
            {
                uint32_t na = 0;
#pragma unroll
                for (int q = 0; q < NR; ++q) na += __popcll(__ballot(active[q]));
                st.nodes += 1;
                st.box_tests += 4u * na;
            }
            const cfloat *np = (const cfloat *)(bvh.nodes + node);
            const cuint *cp = (const cuint *)(bvh.nodes + node);
            float lxs[4], hxs[4], lys[4], hys[4], lzs[4], hzs[4];
            uint32_t chs[4], pads[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                lxs[i] = np[i];
                hxs[i] = np[4 + i];
                lys[i] = np[8 + i];
                hys[i] = np[12 + i];
                lzs[i] = np[16 + i];
                hzs[i] = np[20 + i];
                chs[i] = cp[24 + i];
                pads[i] = cp[28 + i];
            }
            // all of the node's scalar loads issue together, ahead of the
            // per-child branches (else each child waits for its own); the
            // whole 128-byte node, pad words included, is two 64-byte loads
#pragma unroll
            for (int i = 0; i < 4; ++i)
                asm volatile("" ::"s"(lxs[i]), "s"(hxs[i]), "s"(lys[i]), "s"(hys[i]), "s"(lzs[i]), "s"(hzs[i]),
                             "s"(chs[i]), "s"(pads[i]));
            uint32_t next = kEmpty;
#pragma unroll
            for (int i = 3; i >= 0; --i) {
                if (chs[i] == kEmpty) continue;  // wave-uniform: skip the slot's tests
                // every lane tests (no exec-mask branch); the active mask is
                // applied to the ballot
                unsigned long long hit = 0ull;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const TRay &rq = r[q];
                    float t0x = __fmaf_rn(lxs[i], rq.inv[0], rq.off_lo[0]);
                    float t1x = __fmaf_rn(hxs[i], rq.inv[0], rq.off_hi[0]);
                    float t0y = __fmaf_rn(lys[i], rq.inv[1], rq.off_lo[1]);
                    float t1y = __fmaf_rn(hys[i], rq.inv[1], rq.off_hi[1]);
                    float t0z = __fmaf_rn(lzs[i], rq.inv[2], rq.off_lo[2]);
                    float t1z = __fmaf_rn(hzs[i], rq.inv[2], rq.off_hi[2]);
                    float tnear = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
                    float tfar = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
                    tfar = fminf(tfar, tmax * grow);
                    hit |= wave_ballot(tnear <= tfar) & amask[q];
                }
                if (chs[i] != kEmpty && hit != 0ull) {
                    // children pushed in reverse so that child 0 is visited first
                    if (next != kEmpty) {
                        wstack[sp] = next;
                        ++sp;
                    }
                    next = chs[i];
                }
            }
            if (next != kEmpty) {
                node = __builtin_amdgcn_readfirstlane(next);
                continue;
            }
        } else {
            const uint32_t first = node & 0x07FFFFFFu;
            const uint32_t count = ((node >> 27) & 0xFu) + 1u;
            for (uint32_t t3 = 0; t3 < count; ++t3) {
                const cfloat *tp = (const cfloat *)(bvh.tris + 3 * (size_t)(first + t3));
                float4 v0, v1, v2;
                v0.x = tp[0]; v0.y = tp[1]; v0.z = tp[2]; v0.w = tp[3];
                v1.x = tp[4]; v1.y = tp[5]; v1.z = tp[6]; v1.w = tp[7];
                v2.x = tp[8]; v2.y = tp[9]; v2.z = tp[10]; v2.w = tp[11];
                // the triangle's 12 words as one batch of scalar loads
                asm volatile("" ::"s"(v0.x), "s"(v0.y), "s"(v0.z), "s"(v0.w), "s"(v1.x), "s"(v1.y), "s"(v1.z),
                             "s"(v1.w), "s"(v2.x), "s"(v2.y), "s"(v2.z), "s"(v2.w));
                const uint32_t id = __float_as_uint(v0.w);
#pragma unroll
                for (int q = 0; q < NR; ++q) st.tri_tests += __popcll(__ballot(active[q] && id != r[q].ign0 && id != r[q].ign1));
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    if (active[q] && id != r[q].ign0 && id != r[q].ign1) {
                        const float t = tri_hit(r[q], v0, v1, v2);
                        if (t > 0.0f && t < tmax) {
                            blocked[q] = true;
                            active[q] = false;
                        }
                    }
                }
            }
            unsigned long long still = 0ull;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                amask[q] = wave_ballot(active[q]);
                still |= amask[q];
            }
            if (still == 0ull) return;
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(wstack[sp]);
    }
}

// Wave-coherent closest-hit traversal for coherent rays (shadow segments of
// a pixel tile towards one light).  Every lane of the wave calls it with its
// own ray (want = false: the lane rides along).  The wave walks the union of
// its rays' paths from a wave-uniform stack in LDS (`wstack`, kStackTotal
// entries), node and triangle fetches by scalar loads; each lane keeps its
// own closest hit and tests boxes against it (the per-lane walk's culling),
// a child is taken when some active lane's ray meets its box, and children
// are visited nearest first for the first active lane.  The closest
// (t, triangle id) with traverse's tie-break does not depend on the order in
// which nodes are visited, so the result is traverse<false, INCLUSIVE>'s.
template <bool INCLUSIVE>
__device__ inline Hit traverse_wave_closest(const DeviceBVH &bvh, const TRay &r, float tmax, bool want,
                                            uint32_t *wstack) {
    Hit h;
    h.t = tmax;
    h.tri = OCR_HIT_MISS;
    h.leaf_tri = 0;
    const unsigned long long amask = wave_ballot(want);
    if (amask == 0ull) return h;
    const int leader = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(amask));
    const float grow = 1.0f + 0x1p-20f;
    int sp = 0;
    uint32_t node = 0;
    for (;;) {
        if (!(node & kLeafBit)) {
            const cfloat *np = (const cfloat *)(bvh.nodes + node);
            const cuint *cp = (const cuint *)(bvh.nodes + node);
            float lxs[4], hxs[4], lys[4], hys[4], lzs[4], hzs[4];
            uint32_t chs[4], pads[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                lxs[i] = np[i];
                hxs[i] = np[4 + i];
                lys[i] = np[8 + i];
                hys[i] = np[12 + i];
                lzs[i] = np[16 + i];
                hzs[i] = np[20 + i];
                chs[i] = cp[24 + i];
                pads[i] = cp[28 + i];
            }
            // all of the node's scalar loads issue together: the whole 128-byte
            // node, pad words included, as two 64-byte loads
#pragma unroll
            for (int i = 0; i < 4; ++i)
                asm volatile("" ::"s"(lxs[i]), "s"(hxs[i]), "s"(lys[i]), "s"(hys[i]), "s"(lzs[i]), "s"(hzs[i]),
                             "s"(chs[i]), "s"(pads[i]));
            // per child: taken by some lane, and its order key (the leader's
            // entry distance as bits -- entry distances are >= 0, so their bits
            // order as integers -- or after all of those if the leader misses it)
            uint32_t key[4], cand[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                key[i] = 0xFFFFFFFFu;
                cand[i] = kEmpty;
                if (chs[i] == kEmpty) continue;  // wave-uniform
                float t0x = __fmaf_rn(lxs[i], r.inv[0], r.off_lo[0]), t1x = __fmaf_rn(hxs[i], r.inv[0], r.off_hi[0]);
                float t0y = __fmaf_rn(lys[i], r.inv[1], r.off_lo[1]), t1y = __fmaf_rn(hys[i], r.inv[1], r.off_hi[1]);
                float t0z = __fmaf_rn(lzs[i], r.inv[2], r.off_lo[2]), t1z = __fmaf_rn(hzs[i], r.inv[2], r.off_hi[2]);
                float tnear = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
                float tfar = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
                tfar = fminf(tfar, h.t * grow);
                const bool in = want && tnear <= tfar;
                const unsigned long long m = wave_ballot(in);
                if (m != 0ull) {
                    cand[i] = chs[i];
                    const uint32_t lt = (uint32_t)__builtin_amdgcn_readlane(__float_as_int(in ? tnear : INFINITY),
                                                                            leader);
                    key[i] = (m >> leader) & 1ull ? lt : 0xFFFFFFFEu;
                }
            }
            // nearest first: sort the four (key, child) pairs (5 compare-exchanges)
#define OCR_KSWAP(a, b)                                          \
    if (key[b] < key[a]) {                                       \
        uint32_t tk = key[a]; key[a] = key[b]; key[b] = tk;      \
        uint32_t tc = cand[a]; cand[a] = cand[b]; cand[b] = tc;  \
    }
            OCR_KSWAP(0, 1)
            OCR_KSWAP(2, 3)
            OCR_KSWAP(0, 2)
            OCR_KSWAP(1, 3)
            OCR_KSWAP(1, 2)
#undef OCR_KSWAP
            if (cand[0] != kEmpty) {
#pragma unroll
                for (int k = 3; k >= 1; --k) {
                    if (cand[k] != kEmpty) {
                        wstack[sp] = cand[k];
                        ++sp;
                    }
                }
                node = __builtin_amdgcn_readfirstlane(cand[0]);
                continue;
            }
        } else {
            const uint32_t first = node & 0x07FFFFFFu;
            const uint32_t count = ((node >> 27) & 0xFu) + 1u;
            for (uint32_t q = 0; q < count; ++q) {
                const cfloat *tp = (const cfloat *)(bvh.tris + 3 * (size_t)(first + q));
                float4 v0, v1, v2;
                v0.x = tp[0]; v0.y = tp[1]; v0.z = tp[2]; v0.w = tp[3];
                v1.x = tp[4]; v1.y = tp[5]; v1.z = tp[6]; v1.w = tp[7];
                v2.x = tp[8]; v2.y = tp[9]; v2.z = tp[10]; v2.w = tp[11];
                // the triangle's 12 words as one batch of scalar loads
                asm volatile("" ::"s"(v0.x), "s"(v0.y), "s"(v0.z), "s"(v0.w), "s"(v1.x), "s"(v1.y), "s"(v1.z),
                             "s"(v1.w), "s"(v2.x), "s"(v2.y), "s"(v2.z), "s"(v2.w));
                const uint32_t id = __float_as_uint(v0.w);
                if (want && id != r.ign0 && id != r.ign1) {
                    const float t = tri_hit(r, v0, v1, v2);
                    if (t > 0.0f) {
                        bool take;
                        if (t < h.t) take = true;
                        else if (t == h.t) take = h.tri == OCR_HIT_MISS ? INCLUSIVE : id < h.tri;
                        else take = false;
                        if (take) {
                            h.t = t;
                            h.tri = id;
                            h.leaf_tri = first + q;
                        }
                    }
                }
            }
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(wstack[sp]);
    }
    return h;
}

// The same walk with lane masks, for work accounting: each stack entry
// carries the ballot mask of the lanes whose segment touches that child's
// box, and only those lanes (less any found blocked since) test the
// subtree, so the counts are the tests each segment needs on its own
// (useful work), not the tests every unblocked lane of the wave executes.
// Same results as traverse_wave_any.  On SIMD hardware the masks do not
// save time (the wave visits the same nodes), so frames use the plain walk.
// `wnode` / `wmask` are this wave's stack (kStackTotal entries each, LDS).
__device__ inline bool traverse_wave_any_masked(const DeviceBVH &bvh, const TRay &r, float tmax, bool want, uint32_t *wnode,
                                         unsigned long long *wmask, WalkStats &st) {
    unsigned long long mask = __ballot(want);
    if (mask == 0ull) return false;
    st.walks += 1;
    st.segments += (uint64_t)__popcll(mask);
    const unsigned long long me = 1ull << (threadIdx.x & 63);
    bool blocked = false;
    const float grow = 1.0f + 0x1p-20f;
    int sp = 0;
    uint32_t node = 0;
    for (;;) {
        const bool in = (mask & me) != 0ull && !blocked;
        const unsigned long long live = __ballot(in);
        if (live != 0ull) {
            if (!(node & kLeafBit)) {
                st.nodes += 1;
                // the whole node in one batch of scalar loads, before any test
                const cfloat *np = (const cfloat *)(bvh.nodes + node);
                const cuint *cp = (const cuint *)(bvh.nodes + node);
                float lxs[4], hxs[4], lys[4], hys[4], lzs[4], hzs[4];
                uint32_t chs[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    lxs[i] = np[i];
                    hxs[i] = np[4 + i];
                    lys[i] = np[8 + i];
                    hys[i] = np[12 + i];
                    lzs[i] = np[16 + i];
                    hzs[i] = np[20 + i];
                    chs[i] = cp[24 + i];
                }
                uint32_t next = kEmpty;
                unsigned long long next_mask = 0ull;
#pragma unroll
                for (int i = 3; i >= 0; --i) {
                    if (chs[i] == kEmpty) continue;  // wave-uniform: skip the slot's tests
                    st.box_tests += (uint32_t)__popcll(live);
                    const float t0x = __fmaf_rn(lxs[i], r.inv[0], r.off_lo[0]);
                    const float t1x = __fmaf_rn(hxs[i], r.inv[0], r.off_hi[0]);
                    const float t0y = __fmaf_rn(lys[i], r.inv[1], r.off_lo[1]);
                    const float t1y = __fmaf_rn(hys[i], r.inv[1], r.off_hi[1]);
                    const float t0z = __fmaf_rn(lzs[i], r.inv[2], r.off_lo[2]);
                    const float t1z = __fmaf_rn(hzs[i], r.inv[2], r.off_hi[2]);
                    const float tnear = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
                    float tfar = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
                    tfar = fminf(tfar, tmax * grow);
                    const unsigned long long m = __ballot(in && tnear <= tfar);
                    const uint32_t ch = chs[i];
                    if (ch != kEmpty && m != 0ull) {
                        // children pushed in reverse so that child 0 is visited first
                        if (next != kEmpty) {
                            wnode[sp] = next;
                            wmask[sp] = next_mask;
                            ++sp;
                        }
                        next = ch;
                        next_mask = m;
                    }
                }
                if (next != kEmpty) {
                    node = __builtin_amdgcn_readfirstlane(next);
                    mask = next_mask;
                    continue;
                }
            } else {
                const uint32_t first = node & 0x07FFFFFFu;
                const uint32_t count = ((node >> 27) & 0xFu) + 1u;
                bool test = in;
                for (uint32_t t3 = 0; t3 < count; ++t3) {
                    const cfloat *tp = (const cfloat *)(bvh.tris + 3 * (size_t)(first + t3));
                    float4 v0, v1, v2;
                    v0.x = tp[0]; v0.y = tp[1]; v0.z = tp[2]; v0.w = tp[3];
                    v1.x = tp[4]; v1.y = tp[5]; v1.z = tp[6]; v1.w = tp[7];
                    v2.x = tp[8]; v2.y = tp[9]; v2.z = tp[10]; v2.w = tp[11];
                    const uint32_t id = __float_as_uint(v0.w);
                    const bool mine = test && id != r.ign0 && id != r.ign1;
                    st.tri_tests += (uint32_t)__popcll(__ballot(mine));
                    if (mine) {
                        const float t = tri_hit(r, v0, v1, v2);
                        if (t > 0.0f && t < tmax) {
                            blocked = true;
                            test = false;
                        }
                    }
                }
                // every wanted segment decided: done
                if (__ballot(want && !blocked) == 0ull) return blocked;
            }
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(wnode[sp]);
        const unsigned long long mm = wmask[sp];
        // (readfirstlane returns int: widen through uint32_t, not by sign)
        mask = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(mm >> 32)) << 32) |
               (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)mm);
    }
    return blocked;
}

}  // namespace ocr
