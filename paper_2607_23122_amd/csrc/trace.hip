// First-hit occluder tracing (step 1 of App. D / App. H) and the first-hit
// validation rays of the unbiased estimators (Eq. occ-first-hit).
#include "density.hpp"
#include "ocr_common.hpp"
#include "traverse.hpp"

namespace ocr {

constexpr int kBlock = 256;
constexpr int kTile = 16;  // 16 x 16 pixels per block, one 8 x 8 sub-tile per wave

// Blocks are dealt to the 8 XCDs round-robin; remap so that each XCD walks a
// contiguous band of tiles, keeping the BVH paths a band touches in that
// XCD's L2.
__device__ inline void tile_of_block(int tiles_x, int ntiles, int &tx, int &ty) {
    int b = blockIdx.x;
    int per = (ntiles + 7) / 8;
    int xcd = b & 7, local = b >> 3;
    int t = xcd * per + local;
    if (t >= ntiles) t = ntiles;  // out of range -> caller exits
    tx = t % tiles_x;
    ty = t / tiles_x;
}

__device__ inline void pixel_of_thread(int tx, int ty, int &px, int &py) {
    int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    px = tx * kTile + (wv & 1) * 8 + (ln & 7);
    py = ty * kTile + (wv >> 1) * 8 + (ln >> 3);
}

__device__ inline void load3(const float *p, int64_t i, float v[3]) {
    v[0] = p[3 * i];
    v[1] = p[3 * i + 1];
    v[2] = p[3 * i + 2];
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void trace_kernel(DeviceBVH bvh, GBufView g, float R, LightF L, uint32_t sd,
                                                       uint32_t sample, OccView out, int tiles_x, int ntiles) {
    __shared__ uint32_t stack[kStackLds * kBlock];
    int tx, ty;
    tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;
    int px, py;
    pixel_of_thread(tx, ty, px, py);
    if (px >= g.w || py >= g.h) return;
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
        light_point((uint32_t)px, (uint32_t)py, sample, sd, L, y);
        d[0] = y[0] - o[0];
        d[1] = y[1] - o[1];
        d[2] = y[2] - o[2];
        if (!shadow_traced(n, o, d, L)) {
            out.hit[i] = OCR_HIT_SELF;
            return;
        }
        tmax = 1.0f;
    }
    TRay r;
    make_ray(o, d, prim, OCR_HIT_MISS, r);
    Hit h = traverse<false, MODE == OCR_AO>(bvh, r, tmax, stack + threadIdx.x, kBlock);
    out.hit[i] = h.tri;
    if (h.tri == OCR_HIT_MISS) return;
    float nz[3];
    oriented_normal(bvh, h.leaf_tri, d, nz);
    for (int c = 0; c < 3; ++c) {
        out.dz[3 * i + c] = h.t * d[c];
        out.nz[3 * i + c] = nz[c];
    }
}

// Receiver-centric first-hit validation.  Lane = receiver k; for every
// candidate j of the pair neighbourhood (offsets j - k in [-D, D]^2, same
// group for the group pattern) whose density at k is positive, an any-hit
// segment o_k -> z_j over t in (0, 1 - 1e-4), ignoring z_j's triangle and
// k's own, decides Occ(x_k, z_j).  Bit (dy+D)(2D+1) + (dx+D) of k's words
// is set when z_j is the first hit from o_k.
template <int MODE>
__global__ __launch_bounds__(kBlock) void validate_kernel(DeviceBVH bvh, GBufView g, OccView occ, float R2,
                                                          LightF L, int D, int pattern, int gw, int gh, int words,
                                                          uint32_t *bits, int tiles_x, int ntiles) {
    __shared__ uint32_t stack[kStackLds * kBlock];
    int tx, ty;
    tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;
    int px, py;
    pixel_of_thread(tx, ty, px, py);
    if (px >= g.w || py >= g.h) return;
    int64_t k = (int64_t)py * g.w + px;
    uint32_t *mine = bits + k * words;
    uint32_t primk = g.prim[k];
    if (primk == OCR_HIT_MISS) {
        for (int q = 0; q < words; ++q) mine[q] = 0u;
        return;
    }
    float xk[3], nk[3], ok[3];
    load3(g.pos, k, xk);
    load3(g.nrm, k, nk);
    offset_point(xk, nk, ok);
    RecvShadow rk = {0.f, 0.f, 0.f};
    if (MODE == OCR_SHADOW) rk = recv_shadow(ok, L);
    int side = 2 * D + 1;
    uint32_t word = 0u;
    int widx = 0;
    for (int idx = 0; idx < side * side; ++idx) {
        int dy = idx / side - D, dx = idx % side - D;
        int jx = px + dx, jy = py + dy;
        bool bit = false;
        bool inside = jx >= 0 && jx < g.w && jy >= 0 && jy < g.h;
        if (inside && pattern == OCR_GROUP) inside = (jx / gw == px / gw) && (jy / gh == py / gh);
        if (inside) {
            int64_t j = (int64_t)jy * g.w + jx;
            uint32_t hj = occ.hit[j];
            if (j == k) {
                bit = true;
            } else if (hj < OCR_HIT_SELF) {
                float xj[3], nj[3], oj[3], dzj[3], nzj[3], w[3];
                load3(g.pos, j, xj);
                load3(g.nrm, j, nj);
                offset_point(xj, nj, oj);
                load3(occ.dz, j, dzj);
                load3(occ.nz, j, nzj);
                rel_vec(oj, ok, dzj, w);
                float p = MODE == OCR_AO ? dens_ao(w, nk, nzj, R2) : dens_shadow(w, nk, rk, nzj, L);
                if (p > 0.0f) {
                    TRay r;
                    make_ray(ok, w, hj, primk, r);
                    Hit h = traverse<true, false>(bvh, r, 1.0f - 1e-4f, stack + threadIdx.x, kBlock);
                    bit = h.tri == OCR_HIT_MISS;
                }
            }
        }
        if (bit) word |= 1u << (idx & 31);
        if ((idx & 31) == 31 || idx == side * side - 1) {
            mine[widx++] = word;
            word = 0u;
        }
    }
    for (; widx < words; ++widx) mine[widx] = 0u;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void sample_kernel(GBufView g, LightF L, uint32_t sd, uint32_t sample, float *o_out,
                                                        float *d_out, uint8_t *kind) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)g.w * g.h) return;
    const int px = (int)(i % g.w), py = (int)(i / g.w);
    float x[3] = {0.f, 0.f, 0.f}, n[3] = {0.f, 0.f, 0.f}, o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 0.f};
    uint8_t k = 2;
    if (g.prim[i] != OCR_HIT_MISS) {
        load3(g.pos, i, x);
        load3(g.nrm, i, n);
        offset_point(x, n, o);
        if (MODE == OCR_AO) {
            ao_direction((uint32_t)px, (uint32_t)py, sample, sd, n, d);
            k = 0;
        } else {
            float y[3];
            light_point((uint32_t)px, (uint32_t)py, sample, sd, L, y);
            d[0] = y[0] - o[0];
            d[1] = y[1] - o[1];
            d[2] = y[2] - o[2];
            k = shadow_traced(n, o, d, L) ? 0 : 1;
        }
    }
    for (int c = 0; c < 3; ++c) {
        o_out[3 * i + c] = o[c];
        d_out[3 * i + c] = d[c];
    }
    kind[i] = k;
}

hipError_t launch_samples(const GBufView &g, int mode, const LightF &L, uint32_t seed32, uint32_t sample, float *o,
                          float *d, uint8_t *kind, hipStream_t st) {
    int64_t n = (int64_t)g.w * g.h;
    dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    if (mode == OCR_AO)
        hipLaunchKernelGGL(sample_kernel<OCR_AO>, grid, block, 0, st, g, L, seed32, sample, o, d, kind);
    else
        hipLaunchKernelGGL(sample_kernel<OCR_SHADOW>, grid, block, 0, st, g, L, seed32, sample, o, d, kind);
    return hipGetLastError();
}

static inline int ntiles_for(const GBufView &g, int &tiles_x) {
    tiles_x = (g.w + kTile - 1) / kTile;
    int tiles_y = (g.h + kTile - 1) / kTile;
    return tiles_x * tiles_y;
}

static inline int grid_for(int ntiles) { return ((ntiles + 7) / 8) * 8; }

hipError_t launch_trace(const DeviceBVH &bvh, const GBufView &g, int mode, float R, const LightF &L, uint32_t seed32,
                        uint32_t sample, const OccView &out, hipStream_t st) {
    int tiles_x;
    int nt = ntiles_for(g, tiles_x);
    dim3 grid(grid_for(nt)), block(kBlock);
    if (mode == OCR_AO)
        hipLaunchKernelGGL(trace_kernel<OCR_AO>, grid, block, 0, st, bvh, g, R, L, seed32, sample, out, tiles_x, nt);
    else
        hipLaunchKernelGGL(trace_kernel<OCR_SHADOW>, grid, block, 0, st, bvh, g, R, L, seed32, sample, out, tiles_x,
                           nt);
    return hipGetLastError();
}

hipError_t launch_validate(const DeviceBVH &bvh, const GBufView &g, const OccView &occ, int mode, float R,
                           const LightF &L, const ocr_reuse_params &p, uint32_t *bits, hipStream_t st) {
    int tiles_x;
    int nt = ntiles_for(g, tiles_x);
    dim3 grid(grid_for(nt)), block(kBlock);
    int D = pair_extent(p), words = pair_words(p), gw = 1, gh = 1;
    if (p.pattern == OCR_GROUP) group_dims(p.group_n, gw, gh);
    if (mode == OCR_AO)
        hipLaunchKernelGGL(validate_kernel<OCR_AO>, grid, block, 0, st, bvh, g, occ, R * R, L, D, p.pattern, gw, gh,
                           words, bits, tiles_x, nt);
    else
        hipLaunchKernelGGL(validate_kernel<OCR_SHADOW>, grid, block, 0, st, bvh, g, occ, R * R, L, D, p.pattern, gw,
                           gh, words, bits, tiles_x, nt);
    return hipGetLastError();
}

}  // namespace ocr
