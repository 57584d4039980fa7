// Internal layouts and device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ocr.h"

namespace ocr {

// ---------------------------------------------------------------------------
// Device layout of the acceleration structure.
//
// 4-wide nodes of exactly one 128-byte cache line: the child boxes in SoA
// order (so one node is eight dwordx4 loads) and four child links.
// Link encoding: bit 31 clear -> interior node index; bit 31 set -> leaf with
// (count-1) in bits 30..27 and the first triangle in bits 26..0; 0xFFFFFFFF ->
// empty slot (its box is empty so it is never entered).
// Triangles of a leaf are contiguous, 48 bytes each: three float4 vertices,
// the first vertex's w holding the scene triangle index.
// ---------------------------------------------------------------------------
struct alignas(128) Node4 {
    float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
    uint32_t child[4];
    uint32_t pad[4];
};
static_assert(sizeof(Node4) == 128, "node must be one cache line");

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kMaxLeaf = 8;
// Per-lane traversal stack: 16 entries in LDS per lane (16 KB per 256-lane
// block lets the register limit, not LDS, set the trace kernel's occupancy;
// measured 17% faster than 32 entries).  A walk that needs more stops and
// its ray is decided by a wave-coherent walk, whose stack of kStackTotal
// entries per wave the builder guarantees (3 * depth + 1 <= kStackTotal).
constexpr int kStackLds = 16;
constexpr int kStackTotal = 64;
constexpr int kMaxDepth = (kStackTotal - 1) / 3;

// Sliding-window reuse target tile: 16 x 16 pixels.  Candidates in the
// R-pixel halo are processed by every tile whose halo holds them (at R = 3,
// 1.89 candidate instances per pixel); a 32 x 16 tile (1.63) was measured
// 20-60% slower, its larger LDS footprint costing more resident blocks than
// the halo saves.
constexpr int kWTX = 16, kWTY = 16;

struct DeviceBVH {
    const Node4 *nodes;
    const float4 *tris;  // 3 per triangle
    int64_t nnodes;
    int64_t ntris;
    int32_t depth;
};

// Light in the form the kernels use (FP32).
// Internal modes of the reuse kernels, with the records, densities and
// validation of OCR_SHADOW: rectangular-light shadows under the solid-angle
// definition, and occluder-domain direct illumination.
constexpr int kShadowSA = 2;
constexpr int kDI = 3;

struct LightF {
    float c[3], eu[3], ev[3];
    float nl[3];       // unit normal of the emitting side
    float nlu[3];      // e_u x e_v unnormalised (the sampler's sidedness test)
    float uhat[3];     // e_u / |e_u|^2
    float vhat[3];     // e_v / |e_v|^2
};

// ---------------------------------------------------------------------------
// Sample specification (FP32, rounding exactly as written; contraction off).
// ---------------------------------------------------------------------------
__host__ __device__ inline void pcg4d(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d) {
    a = a * 1664525u + 1013904223u;
    b = b * 1664525u + 1013904223u;
    c = c * 1664525u + 1013904223u;
    d = d * 1664525u + 1013904223u;
    a += b * d;
    b += c * a;
    c += a * b;
    d += b * c;
    a ^= a >> 16;
    b ^= b >> 16;
    c ^= c >> 16;
    d ^= d >> 16;
    a += b * d;
    b += c * a;
    c += a * b;
    d += b * c;
}

__host__ __device__ inline uint32_t fold_seed(uint64_t s) { return (uint32_t)s ^ (uint32_t)(s >> 32); }

__device__ inline float unit24(uint32_t h) { return (float)(h >> 8) * 0x1p-24f; }

// o = x + eps n, eps = 2^-16 (1 + max_c |x_c|)
__device__ inline void offset_point(const float x[3], const float n[3], float o[3]) {
#pragma clang fp contract(off)
    float m = fmaxf(fabsf(x[0]), fmaxf(fabsf(x[1]), fabsf(x[2])));
    float eps = (1.0f + m) * 0x1p-16f;
    o[0] = __fmaf_rn(eps, n[0], x[0]);
    o[1] = __fmaf_rn(eps, n[1], x[1]);
    o[2] = __fmaf_rn(eps, n[2], x[2]);
}

// Cosine-weighted direction by Malley's method: a uniform point of the unit
// disc (rejection, at most 16 draws, then the disc centre) lifted along n,
// in the branchless orthonormal basis of Duff et al.
__device__ inline void ao_direction(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const float n[3],
                                    float w[3]) {
#pragma clang fp contract(off)
    float al = 0.0f, be = 0.0f, q = 0.0f;
    for (uint32_t a = 0; a < 16u; ++a) {
        uint32_t h0 = px, h1 = py, h2 = s, h3 = sd + a * 0x9E3779B9u;
        pcg4d(h0, h1, h2, h3);
        float ta = 2.0f * unit24(h0) - 1.0f;
        float tb = 2.0f * unit24(h1) - 1.0f;
        float tq = __fmaf_rn(tb, tb, ta * ta);
        if (tq < 1.0f) {
            al = ta;
            be = tb;
            q = tq;
            break;
        }
    }
    float g = sqrtf(1.0f - q);  // correctly rounded (HIP default)
    float sign = copysignf(1.0f, n[2]);
    float a = -1.0f / (sign + n[2]);  // correctly rounded (HIP default)
    float b = n[0] * n[1] * a;
    float t0 = 1.0f + sign * n[0] * n[0] * a, t1 = sign * b, t2 = -sign * n[0];
    float b0 = b, b1 = sign + n[1] * n[1] * a, b2 = -n[1];
    w[0] = (al * t0 + be * b0) + g * n[0];
    w[1] = (al * t1 + be * b1) + g * n[1];
    w[2] = (al * t2 + be * b2) + g * n[2];
}

// Uniform light point y = c + (u0 - 1/2) e_u + (u1 - 1/2) e_v.
__device__ inline void light_point(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const LightF &L,
                                   float y[3]) {
#pragma clang fp contract(off)
    uint32_t h0 = px, h1 = py, h2 = s, h3 = sd;
    pcg4d(h0, h1, h2, h3);
    float a = unit24(h0) - 0.5f;
    float b = unit24(h1) - 0.5f;
    for (int c = 0; c < 3; ++c) y[c] = __fmaf_rn(b, L.ev[c], __fmaf_rn(a, L.eu[c], L.c[c]));
}

// Shadow sample sidedness: traced iff y is in front of the tangent plane and
// the receiver is on the emitting side of the light.
__device__ inline bool shadow_traced(const float n[3], const float o[3], const float dir[3], const LightF &L) {
#pragma clang fp contract(off)
    float front = __fmaf_rn(n[2], dir[2], __fmaf_rn(n[1], dir[1], n[0] * dir[0]));
    float lit = __fmaf_rn(L.nlu[2], o[2] - L.c[2], __fmaf_rn(L.nlu[1], o[1] - L.c[1], L.nlu[0] * (o[0] - L.c[0])));
    return front > 0.0f && lit > 0.0f;
}

// q / d for 0 <= q < 2^21 and d >= 1 with one FP32 multiply by inv_d, an
// approximation of 1/d within one ulp (correctly rounded, or the hardware
// reciprocal): (q + 1/2) / d lies at least 1/(2d) from an integer and the
// FP32 product is within (q + 1/2) 3 2^-24 / d of it, so the truncation is
// the exact quotient (checked exhaustively on the host for q < 2^16,
// d <= 1024 with both neighbours of 1/d).  Integer division by a runtime
// value is a long instruction sequence on this hardware.
__device__ inline int small_div(int q, float inv_d) { return (int)(((float)q + 0.5f) * inv_d); }

// Lane mask of the wave's lanes (active ones) where p holds; the compiler
// builtin takes the compare's own mask, where __ballot materialises the bool
// in a vector register and compares it again.
__device__ inline unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Inclusive prefix sum over the wave's 64 lanes.
__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---------------------------------------------------------------------------
// Launch-side helpers
// ---------------------------------------------------------------------------
struct GBufView {
    const float *pos;
    const float *nrm;
    const uint32_t *prim;
    int32_t w, h;
};

struct OccView {
    float *dz;
    float *nz;
    uint32_t *hit;
};

// Host-side launchers (defined in the .hip files).
hipError_t launch_trace(const DeviceBVH &bvh, const GBufView &g, int mode, float R, const LightF &L, uint32_t seed32,
                        uint32_t sample, const OccView &out, hipStream_t st);
hipError_t launch_trace_count(const DeviceBVH &bvh, const GBufView &g, int mode, float R, const LightF &L,
                              uint32_t seed32, uint32_t sample, const OccView &out, uint64_t *stats, hipStream_t st);
hipError_t launch_validate(const DeviceBVH &bvh, const GBufView &g, const OccView &occ, int mode, float R,
                           const LightF &L, const ocr_reuse_params &p, uint32_t *bits, uint64_t *stats,
                           hipStream_t st);
// scale: rho L_e / pi for direct illumination (kDI), unused otherwise
hipError_t launch_reuse(const GBufView &g, const OccView &occ, int mode, float R, const LightF &L,
                        const ocr_reuse_params &p, const uint32_t *bits, float *out, hipStream_t st,
                        float scale = 1.0f);
hipError_t launch_scale(float *out, int64_t n, float s, hipStream_t st);
hipError_t launch_samples(const GBufView &g, int mode, const LightF &L, uint32_t seed32, uint32_t sample, float *o,
                          float *d, uint8_t *kind, hipStream_t st);

// Validation bit layout: per receiver pixel k, `words` uint32 holding one
// bit per offset (j - k) in [-D, D]^2, row-major, with D = 2r (window) or the
// group's extent (group).
inline int pair_extent(const ocr_reuse_params &p) {
    if (p.pattern == OCR_WINDOW) return 2 * p.radius;
    return p.group_n == 8 ? 3 : (p.group_n >= 2 ? 1 : 0);
}
inline int pair_words(const ocr_reuse_params &p) {
    int side = 2 * pair_extent(p) + 1;
    return (side * side + 31) / 32;
}
inline void group_dims(int n, int &gw, int &gh) {
    gw = n == 8 ? 4 : (n >= 2 ? 2 : 1);
    gh = n >= 4 ? 2 : 1;
}

}  // namespace ocr
