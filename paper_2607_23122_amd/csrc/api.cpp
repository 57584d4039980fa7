// C-ABI entry points: argument validation, error reporting, the BVH handle,
// and dispatch to the kernel launchers.  Per-frame entry points only enqueue
// work on the caller's stream; they allocate nothing and never synchronise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "api_internal.hpp"
#include "bvh_build.hpp"
#include "lights.hpp"

using namespace ocr;

namespace {
thread_local std::string g_err;
bool finite3(const float *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }
}  // namespace

namespace ocr {

ocr_status fail(ocr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

ocr_status hip_fail(hipError_t e, const char *what) {
    return fail(OCR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

ocr_status check_gbuf(const ocr_gbuffer *g) {
    if (!g) return fail(OCR_ERR_INVALID_ARG, "gbuffer is NULL");
    if (!g->pos || !g->nrm || !g->prim) return fail(OCR_ERR_INVALID_ARG, "gbuffer has a NULL array");
    if (g->width < 1 || g->height < 1) return fail(OCR_ERR_INVALID_ARG, "gbuffer size %dx%d", g->width, g->height);
    if ((int64_t)g->width * g->height >= (int64_t)1 << 31)
        return fail(OCR_ERR_INVALID_ARG, "gbuffer too large (%dx%d)", g->width, g->height);
    return OCR_OK;
}

ocr_status make_light(const ocr_rect_light *l, LightF &L) {
    // e_u x e_v below in FP32 exactly as the sampler specifies it: no contraction
#pragma clang fp contract(off)
    std::memset(&L, 0, sizeof L);
    if (!l) return fail(OCR_ERR_INVALID_ARG, "light is NULL");
    if (!finite3(l->center) || !finite3(l->edge_u) || !finite3(l->edge_v))
        return fail(OCR_ERR_INVALID_ARG, "light has non-finite values");
    if (l->pdf != OCR_LIGHT_UNIFORM && l->pdf != OCR_LIGHT_BILINEAR)
        return fail(OCR_ERR_INVALID_ARG, "light pdf %d out of range", l->pdf);
    const float *u = l->edge_u, *v = l->edge_v;
    double uu = (double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2];
    double vv = (double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2];
    double uv = (double)u[0] * v[0] + (double)u[1] * v[1] + (double)u[2] * v[2];
    if (!(uu > 0.0) || !(vv > 0.0)) return fail(OCR_ERR_INVALID_ARG, "light edge has zero length");
    if (std::fabs(uv) > 1e-6 * std::sqrt(uu * vv)) return fail(OCR_ERR_INVALID_ARG, "light edges not orthogonal");
    for (int c = 0; c < 3; ++c) {
        L.c[c] = l->center[c];
        L.eu[c] = u[c];
        L.ev[c] = v[c];
        L.uhat[c] = (float)(u[c] / uu);
        L.vhat[c] = (float)(v[c] / vv);
    }
    // e_u x e_v in FP32 as the sampler specifies (products rounded, then the difference)
    L.nlu[0] = u[1] * v[2] - u[2] * v[1];
    L.nlu[1] = u[2] * v[0] - u[0] * v[2];
    L.nlu[2] = u[0] * v[1] - u[1] * v[0];
    double nx = (double)u[1] * v[2] - (double)u[2] * v[1];
    double ny = (double)u[2] * v[0] - (double)u[0] * v[2];
    double nz = (double)u[0] * v[1] - (double)u[1] * v[0];
    double nl = std::sqrt(nx * nx + ny * ny + nz * nz);
    L.nl[0] = (float)(nx / nl);
    L.nl[1] = (float)(ny / nl);
    L.nl[2] = (float)(nz / nl);
    return OCR_OK;
}

ocr_status check_params(const ocr_reuse_params *p) {
    if (!p) return fail(OCR_ERR_INVALID_ARG, "params is NULL");
    if (p->estimator < OCR_NOREUSE || p->estimator > OCR_UNBIASED)
        return fail(OCR_ERR_INVALID_ARG, "estimator %d out of range", p->estimator);
    if (p->pattern == OCR_WINDOW) {
        if (p->radius < 0 || p->radius > 8) return fail(OCR_ERR_INVALID_ARG, "window radius %d not in [0,8]", p->radius);
    } else if (p->pattern == OCR_GROUP) {
        if (p->group_n != 1 && p->group_n != 2 && p->group_n != 4 && p->group_n != 8)
            return fail(OCR_ERR_INVALID_ARG, "group size %d not in {1,2,4,8}", p->group_n);
    } else {
        return fail(OCR_ERR_INVALID_ARG, "pattern %d out of range", p->pattern);
    }
    return OCR_OK;
}

ocr_status uniform_only(const ocr_rect_light *l, const char *who) {
    if (l && l->pdf != OCR_LIGHT_UNIFORM)
        return fail(OCR_ERR_UNSUPPORTED, "%s samples lights uniformly only (pdf %d)", who, l->pdf);
    return OCR_OK;
}

ocr_status make_lights(const ocr_rect_light *lights, int32_t n, LightSetF &S) {
    std::memset(&S, 0, sizeof S);
    if (!lights) return fail(OCR_ERR_INVALID_ARG, "lights is NULL");
    if (n < 1 || n > kMaxLights) return fail(OCR_ERR_INVALID_ARG, "%d lights not in [1,%d]", n, kMaxLights);
    S.n = n;
    for (int k = 0; k < n; ++k) {
        ocr_status st = make_light(&lights[k], S.l[k]);
        if (st) return st;
        if ((st = uniform_only(&lights[k], "several lights"))) return st;
    }
    return OCR_OK;
}

ocr_status check_effect(int32_t mode, float ao_radius, const ocr_rect_light *light, LightF &L) {
    std::memset(&L, 0, sizeof L);
    if (mode == OCR_AO) {
        if (!(std::isfinite(ao_radius) && ao_radius > 0.0f))
            return fail(OCR_ERR_INVALID_ARG, "AO radius %g must be finite and > 0", (double)ao_radius);
        return OCR_OK;
    }
    if (mode == OCR_SHADOW) {
        ocr_status st = make_light(light, L);
        return st ? st : uniform_only(light, "this entry point");
    }
    return fail(OCR_ERR_INVALID_ARG, "mode %d out of range", mode);
}

}  // namespace ocr

namespace {

// pdf: the light's emitter density (OCR_LIGHT_UNIFORM for AO).
ocr_status reuse_common(const ocr_bvh *bvh, const ocr_gbuffer *g, const ocr_occluders *occ, int mode, float R,
                        const LightF &L, const ocr_reuse_params *p, void *ws, size_t ws_bytes, float *out,
                        void *stream, float scale = 1.0f, int pdf = OCR_LIGHT_UNIFORM) {
    ocr_status st = check_gbuf(g);
    if (st) return st;
    if ((st = check_params(p))) return st;
    if (!occ || !occ->dz || !occ->nz || !occ->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    if (!out) return fail(OCR_ERR_INVALID_ARG, "out is NULL");
    size_t need = ocr_workspace_bytes(g->width, g->height, p);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(OCR_ERR_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (p->estimator == OCR_UNBIASED && !p->validated && !bvh)
        return fail(OCR_ERR_INVALID_ARG, "unbiased reuse needs the BVH");
    hipStream_t s = (hipStream_t)stream;
    OccView ov{occ->dz, occ->nz, occ->hit};
    GBufView gv = view(g);
    hipError_t e;
    if (p->estimator == OCR_UNBIASED && !p->validated) {
        // the light modes validate the same pairs (same densities)
        e = launch_validate(bvh->dev, gv, ov, mode == OCR_AO ? OCR_AO : OCR_SHADOW, R, L, *p, (uint32_t *)ws,
                            nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "validation launch");
    }
    if (pdf == OCR_LIGHT_BILINEAR)
        e = launch_reuse_bilinear(gv, ov, mode, LightBilinF{L}, *p, (const uint32_t *)ws, out, s, scale);
    else
        e = launch_reuse(gv, ov, mode, R, L, *p, (const uint32_t *)ws, out, s, scale);
    if (e != hipSuccess) return hip_fail(e, "reuse launch");
    return OCR_OK;
}

}  // namespace

extern "C" {

const char *ocr_last_error(void) { return g_err.c_str(); }

const char *ocr_version(void) { return "ocr-mi355x 0.1 (gfx950)"; }

}  // extern "C"

namespace {

// Argument checks and the host build shared by ocr_build_bvh and
// ocr_build_bvh_host.
ocr_status host_build(const float *verts, int64_t nverts, const uint32_t *tris, int64_t ntris, HostBVH &hb) {
    if (!verts || !tris) return fail(OCR_ERR_INVALID_ARG, "NULL vertex or triangle array");
    if (nverts < 1 || ntris < 1) return fail(OCR_ERR_INVALID_ARG, "empty scene (%lld verts, %lld tris)",
                                             (long long)nverts, (long long)ntris);
    if (ntris >= ((int64_t)1 << 27)) return fail(OCR_ERR_INVALID_ARG, "too many triangles (%lld)", (long long)ntris);
    for (int64_t i = 0; i < 3 * ntris; ++i)
        if ((int64_t)tris[i] >= nverts)
            return fail(OCR_ERR_INVALID_ARG, "triangle %lld references vertex %u >= %lld", (long long)(i / 3),
                        tris[i], (long long)nverts);
    for (int64_t i = 0; i < 3 * nverts; ++i)
        if (!std::isfinite(verts[i])) return fail(OCR_ERR_INVALID_ARG, "vertex %lld is not finite", (long long)(i / 3));
    try {
        if (build_bvh_host(verts, nverts, tris, ntris, hb) != 0)
            return fail(OCR_ERR_UNSUPPORTED, "BVH depth %d exceeds the traversal stack", hb.depth);
    } catch (const std::bad_alloc &) {
        return fail(OCR_ERR_OOM, "host allocation failed while building the BVH");
    }
    return OCR_OK;
}

}  // namespace

extern "C" {

ocr_status ocr_build_bvh_host(const float *verts, int64_t nverts, const uint32_t *tris, int64_t ntris, void *nodes,
                              int64_t node_capacity, float *tri_data, int64_t *out_nnodes, int32_t *out_depth) {
    if (!out_nnodes || !out_depth) return fail(OCR_ERR_INVALID_ARG, "NULL count output");
    HostBVH hb;
    ocr_status st = host_build(verts, nverts, tris, ntris, hb);
    if (st) return st;
    *out_nnodes = (int64_t)hb.nodes.size();
    *out_depth = hb.depth;
    if (nodes) {
        if (node_capacity < (int64_t)hb.nodes.size())
            return fail(OCR_ERR_INVALID_ARG, "node buffer holds %lld nodes, %lld needed", (long long)node_capacity,
                        (long long)hb.nodes.size());
        std::memcpy(nodes, hb.nodes.data(), hb.nodes.size() * sizeof(Node4));
    }
    if (tri_data) std::memcpy(tri_data, hb.tris.data(), hb.tris.size() * sizeof(float4));
    return OCR_OK;
}

ocr_status ocr_build_bvh(const float *verts, int64_t nverts, const uint32_t *tris, int64_t ntris, void *stream,
                         ocr_bvh **out) {
    if (!out) return fail(OCR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    HostBVH hb;
    ocr_status st = host_build(verts, nverts, tris, ntris, hb);
    if (st) return st;
    ocr_bvh *b = new (std::nothrow) ocr_bvh;
    if (!b) return fail(OCR_ERR_OOM, "handle allocation failed");
    size_t nbytes = hb.nodes.size() * sizeof(Node4), tbytes = hb.tris.size() * sizeof(float4);
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc(&b->mem, nbytes + tbytes);
    if (e != hipSuccess) {
        delete b;
        return e == hipErrorOutOfMemory ? fail(OCR_ERR_OOM, "device allocation of %zu bytes", nbytes + tbytes)
                                        : hip_fail(e, "device allocation");
    }
    hipStream_t s = (hipStream_t)stream;
    e = hipMemcpyAsync(b->mem, hb.nodes.data(), nbytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char *)b->mem + nbytes, hb.tris.data(), tbytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(b->mem);
        delete b;
        return hip_fail(e, "BVH upload");
    }
    b->dev.nodes = (const Node4 *)b->mem;
    b->dev.tris = (const float4 *)((char *)b->mem + nbytes);
    b->dev.nnodes = (int64_t)hb.nodes.size();
    b->dev.ntris = ntris;
    b->dev.depth = hb.depth;
    b->info.ntris = ntris;
    b->info.nnodes = (int64_t)hb.nodes.size();
    b->info.depth = hb.depth;
    b->info.max_leaf = hb.max_leaf;
    b->info.device_bytes = (int64_t)(nbytes + tbytes);
    b->info.build_ms = hb.build_ms;
    *out = b;
    return OCR_OK;
}

ocr_status ocr_bvh_free(ocr_bvh *bvh) {
    if (!bvh) return OCR_OK;
    hipError_t e = hipFree(bvh->mem);
    delete bvh;
    return e == hipSuccess ? OCR_OK : hip_fail(e, "BVH free");
}

ocr_status ocr_bvh_get_info(const ocr_bvh *bvh, ocr_bvh_info *info) {
    if (!bvh || !info) return fail(OCR_ERR_INVALID_ARG, "NULL argument");
    *info = bvh->info;
    return OCR_OK;
}

ocr_status ocr_trace_occluders(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, int32_t mode, float ao_radius,
                               const ocr_rect_light *light, uint64_t seed, uint32_t sample, ocr_occluders *out,
                               void *stream) {
    if (!bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if (!out || !out->dz || !out->nz || !out->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    LightF L;
    std::memset(&L, 0, sizeof L);
    if (mode == OCR_AO) {
        if (!(std::isfinite(ao_radius) && ao_radius > 0.0f))
            return fail(OCR_ERR_INVALID_ARG, "AO radius %g must be finite and > 0", (double)ao_radius);
    } else if (mode == OCR_SHADOW) {
        if ((st = make_light(light, L))) return st;
    } else {
        return fail(OCR_ERR_INVALID_ARG, "mode %d out of range", mode);
    }
    const OccView ov{out->dz, out->nz, out->hit};
    hipError_t e = mode == OCR_SHADOW && light->pdf == OCR_LIGHT_BILINEAR
                       ? launch_trace_bilinear(bvh->dev, view(gbuf), LightBilinF{L}, fold_seed(seed), sample, ov,
                                               (hipStream_t)stream)
                       : launch_trace(bvh->dev, view(gbuf), mode, ao_radius, L, fold_seed(seed), sample, ov,
                                      (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "trace launch");
}

ocr_status ocr_trace_occluders_counted(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, int32_t mode, float ao_radius,
                                       const ocr_rect_light *light, uint64_t seed, uint32_t sample,
                                       ocr_occluders *out, uint64_t *stats, void *stream) {
    if (!bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    if (!stats) return fail(OCR_ERR_INVALID_ARG, "stats is NULL");
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if (!out || !out->dz || !out->nz || !out->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    LightF L;
    if ((st = check_effect(mode, ao_radius, light, L))) return st;
    hipError_t e = launch_trace_count(bvh->dev, view(gbuf), mode, ao_radius, L, fold_seed(seed), sample,
                                      OccView{out->dz, out->nz, out->hit}, stats, (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "counted trace launch");
}

ocr_status ocr_sample_rays(const ocr_gbuffer *gbuf, int32_t mode, const ocr_rect_light *light, uint64_t seed,
                           uint32_t sample, float *origin, float *dir, uint8_t *kind, void *stream) {
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if (!origin || !dir || !kind) return fail(OCR_ERR_INVALID_ARG, "NULL output array");
    LightF L;
    std::memset(&L, 0, sizeof L);
    if (mode == OCR_SHADOW) {
        if ((st = make_light(light, L))) return st;
    } else if (mode != OCR_AO) {
        return fail(OCR_ERR_INVALID_ARG, "mode %d out of range", mode);
    }
    hipError_t e = mode == OCR_SHADOW && light->pdf == OCR_LIGHT_BILINEAR
                       ? launch_samples_bilinear(view(gbuf), LightBilinF{L}, fold_seed(seed), sample, origin, dir,
                                                 kind, (hipStream_t)stream)
                       : launch_samples(view(gbuf), mode, L, fold_seed(seed), sample, origin, dir, kind,
                                        (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "sample launch");
}

size_t ocr_workspace_bytes(int32_t width, int32_t height, const ocr_reuse_params *params) {
    if (!params || width < 1 || height < 1) return 0;
    if (params->estimator != OCR_UNBIASED) return 0;
    if (params->pattern == OCR_WINDOW && (params->radius < 0 || params->radius > 8)) return 0;
    if (params->pattern == OCR_GROUP && params->group_n != 1 && params->group_n != 2 && params->group_n != 4 &&
        params->group_n != 8)
        return 0;
    if (params->pattern != OCR_WINDOW && params->pattern != OCR_GROUP) return 0;
    size_t bytes = (size_t)width * (size_t)height * (size_t)pair_words(*params) * sizeof(uint32_t);
    // the validation also keeps per-XCD candidate lists: 8 counters of one
    // 128-byte line each, then room for every pixel of every 16x16 tile
    size_t tiles = (size_t)((width + 15) / 16) * (size_t)((height + 15) / 16);
    bytes += (8 * 32 + ((tiles + 7) / 8) * 8 * 256) * sizeof(uint32_t);
    return bytes;
}

ocr_status ocr_validate_pairs(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ, int32_t mode,
                              float ao_radius, const ocr_rect_light *light, const ocr_reuse_params *params,
                              void *workspace, size_t workspace_bytes, uint64_t *stats, void *stream) {
    if (!bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (params->estimator != OCR_UNBIASED) return fail(OCR_ERR_INVALID_ARG, "validation is for OCR_UNBIASED");
    if (!occ || !occ->dz || !occ->nz || !occ->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    LightF L;
    std::memset(&L, 0, sizeof L);
    if (mode == OCR_AO) {
        if (!(std::isfinite(ao_radius) && ao_radius > 0.0f))
            return fail(OCR_ERR_INVALID_ARG, "AO radius %g must be finite and > 0", (double)ao_radius);
    } else if (mode == OCR_SHADOW) {
        if ((st = make_light(light, L))) return st;
        ao_radius = 1.0f;
    } else {
        return fail(OCR_ERR_INVALID_ARG, "mode %d out of range", mode);
    }
    size_t need = ocr_workspace_bytes(gbuf->width, gbuf->height, params);
    if (!workspace || workspace_bytes < need)
        return fail(OCR_ERR_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    hipError_t e = launch_validate(bvh->dev, view(gbuf), OccView{occ->dz, occ->nz, occ->hit}, mode, ao_radius, L,
                                   *params, (uint32_t *)workspace, stats, (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "validation launch");
}

ocr_status ocr_reuse_ao(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ, float ao_radius,
                        const ocr_reuse_params *params, void *workspace, size_t workspace_bytes, float *out,
                        void *stream) {
    if (!(std::isfinite(ao_radius) && ao_radius > 0.0f))
        return fail(OCR_ERR_INVALID_ARG, "AO radius %g must be finite and > 0", (double)ao_radius);
    LightF L;
    std::memset(&L, 0, sizeof L);
    return reuse_common(bvh, gbuf, occ, OCR_AO, ao_radius, L, params, workspace, workspace_bytes, out, stream);
}

ocr_status ocr_reuse_ao_noalloc(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                float ao_radius, const ocr_reuse_params *params, float *out, void *stream) {
    if (!(std::isfinite(ao_radius) && ao_radius > 0.0f))
        return fail(OCR_ERR_INVALID_ARG, "AO radius %g must be finite and > 0", (double)ao_radius);
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (params->estimator == OCR_UNBIASED && params->validated)
        return fail(OCR_ERR_INVALID_ARG, "the no-allocation entry point validates within the call (validated = 0)");
    const size_t need = ocr_workspace_bytes(gbuf->width, gbuf->height, params);
    if (need > kScratchBytes)
        return fail(OCR_ERR_INVALID_ARG, "a %dx%d frame needs %zu bytes of scratch; this entry point holds %zu",
                    gbuf->width, gbuf->height, need, kScratchBytes);
    void *ws = nullptr;
    if (need > 0) {
        hipError_t e = scratch_address(&ws);
        if (e != hipSuccess) return hip_fail(e, "scratch address");
    }
    LightF L;
    std::memset(&L, 0, sizeof L);
    return reuse_common(bvh, gbuf, occ, OCR_AO, ao_radius, L, params, ws, need > 0 ? kScratchBytes : 0, out,
                        stream);
}

ocr_status ocr_reuse_shadow(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                            const ocr_rect_light *light, const ocr_reuse_params *params, void *workspace,
                            size_t workspace_bytes, float *out, void *stream) {
    LightF L;
    ocr_status st = make_light(light, L);
    if (st) return st;
    return reuse_common(bvh, gbuf, occ, OCR_SHADOW, 1.0f, L, params, workspace, workspace_bytes, out, stream, 1.0f,
                        light->pdf);
}

ocr_status ocr_reuse_shadow_solid_angle(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                        const ocr_rect_light *light, const ocr_reuse_params *params,
                                        void *workspace, size_t workspace_bytes, float *out, void *stream) {
    LightF L;
    ocr_status st = make_light(light, L);
    if (st) return st;
    return reuse_common(bvh, gbuf, occ, kShadowSA, 1.0f, L, params, workspace, workspace_bytes, out, stream, 1.0f,
                        light->pdf);
}

ocr_status ocr_trace_occluders_lights(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_rect_light *lights,
                                      int32_t nlights, uint64_t seed, uint32_t sample, ocr_occluders *out,
                                      void *stream) {
    if (!bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if (!out || !out->dz || !out->nz || !out->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    LightSetF S;
    if ((st = make_lights(lights, nlights, S))) return st;
    hipError_t e = launch_trace_lights(bvh->dev, view(gbuf), S, fold_seed(seed), sample,
                                       OccView{out->dz, out->nz, out->hit}, (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "trace launch");
}

ocr_status ocr_reuse_shadow_lights(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                   const ocr_rect_light *lights, int32_t nlights, const ocr_reuse_params *params,
                                   void *workspace, size_t workspace_bytes, float *out, void *stream) {
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (!occ || !occ->dz || !occ->nz || !occ->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    if (!out) return fail(OCR_ERR_INVALID_ARG, "out is NULL");
    LightSetF S;
    if ((st = make_lights(lights, nlights, S))) return st;
    size_t need = ocr_workspace_bytes(gbuf->width, gbuf->height, params);
    if (need > 0 && (!workspace || workspace_bytes < need))
        return fail(OCR_ERR_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if (params->estimator == OCR_UNBIASED && !params->validated && !bvh)
        return fail(OCR_ERR_INVALID_ARG, "unbiased reuse needs the BVH");
    hipStream_t s = (hipStream_t)stream;
    OccView ov{occ->dz, occ->nz, occ->hit};
    GBufView gv = view(gbuf);
    hipError_t e;
    if (params->estimator == OCR_UNBIASED && !params->validated) {
        e = launch_validate_lights(bvh->dev, gv, ov, S, *params, (uint32_t *)workspace, nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "validation launch");
    }
    e = launch_reuse_lights(gv, ov, S, *params, (const uint32_t *)workspace, out, s);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "reuse launch");
}

ocr_status ocr_validate_pairs_lights(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                     const ocr_rect_light *lights, int32_t nlights, const ocr_reuse_params *params,
                                     void *workspace, size_t workspace_bytes, uint64_t *stats, void *stream) {
    if (!bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (params->estimator != OCR_UNBIASED) return fail(OCR_ERR_INVALID_ARG, "validation is for OCR_UNBIASED");
    if (!occ || !occ->dz || !occ->nz || !occ->hit) return fail(OCR_ERR_INVALID_ARG, "occluder records incomplete");
    LightSetF S;
    if ((st = make_lights(lights, nlights, S))) return st;
    size_t need = ocr_workspace_bytes(gbuf->width, gbuf->height, params);
    if (!workspace || workspace_bytes < need)
        return fail(OCR_ERR_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    hipError_t e = launch_validate_lights(bvh->dev, view(gbuf), OccView{occ->dz, occ->nz, occ->hit}, S, *params,
                                          (uint32_t *)workspace, stats, (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "validation launch");
}

ocr_status ocr_reuse_direct_illumination(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                         const ocr_rect_light *light, float radiance, float albedo,
                                         const ocr_reuse_params *params, void *workspace, size_t workspace_bytes,
                                         float *out, void *stream) {
    if (!(std::isfinite(radiance) && radiance >= 0.0f) || !(std::isfinite(albedo) && albedo >= 0.0f))
        return fail(OCR_ERR_INVALID_ARG, "radiance %g and albedo %g must be finite and >= 0", (double)radiance,
                    (double)albedo);
    LightF L;
    ocr_status st = make_light(light, L);
    if (st) return st;
    const float scale = (float)((double)albedo * (double)radiance / 3.14159265358979323846);
    return reuse_common(bvh, gbuf, occ, kDI, 1.0f, L, params, workspace, workspace_bytes, out, stream, scale,
                        light->pdf);
}

ocr_status ocr_filter_values(const ocr_gbuffer *gbuf, const ocr_reuse_params *params, const float *in, float *out,
                             void *stream) {
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (!in || !out) return fail(OCR_ERR_INVALID_ARG, "in or out is NULL");
    if (in == out) return fail(OCR_ERR_INVALID_ARG, "out must not alias in");
    hipError_t e = launch_filter(view(gbuf), *params, in, out, (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "filter launch");
}

ocr_status ocr_light_reuse_shadow(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_rect_light *light,
                                  uint64_t seed, uint32_t sample, const ocr_reuse_params *params, float *out,
                                  void *stream) {
    ocr_status st = check_gbuf(gbuf);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (!bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    if (!out) return fail(OCR_ERR_INVALID_ARG, "out is NULL");
    LightF L;
    if ((st = make_light(light, L))) return st;
    if ((st = uniform_only(light, "light-sample reuse"))) return st;
    hipError_t e = launch_light_reuse(bvh->dev, view(gbuf), L, fold_seed(seed), sample, *params, out,
                                      (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "light-sample reuse launch");
}

ocr_status ocr_scale(float *out, int64_t n, float s, void *stream) {
    if (!out || n < 0) return fail(OCR_ERR_INVALID_ARG, "bad scale arguments");
    if (n == 0) return OCR_OK;
    hipError_t e = launch_scale(out, n, s, (hipStream_t)stream);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "scale launch");
}

}  // extern "C"
