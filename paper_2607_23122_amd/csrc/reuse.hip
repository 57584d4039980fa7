// Occluder-domain MIS reuse kernels (Sec. 4.2-4.4; steps 2-3 of App. D /
// App. H): the sliding window (one 16x16 target tile per block; the tile
// body is shared with the batched schedule), fixed groups, no reuse, and the
// sample-mean scale; each for AO, area-definition shadows, shadows under the
// solid-angle definition (kShadowSA) and direct illumination (kDI), with the
// light types of lights.hpp.
//
// Fixed groups (N = 1, 2, 4, 8): one lane per pixel; each receiver lane
// evaluates its densities for the N candidates of its group into LDS and each
// target lane sums its group's columns in a fixed order.
#include <atomic>

#include "density.hpp"
#include "lights.hpp"
#include "ocr_common.hpp"
#include "reuse_tile.hpp"
#include "solid_angle.hpp"

namespace ocr {

// Blocks are dealt to the 8 XCDs round-robin; XCD x takes runs x, x + 8, ...
// of kRTileRun consecutive tiles (row-major), so that every XCD samples the
// whole frame and they finish together.  (One contiguous band of tiles per
// XCD left XCDs idle at the end: 1080p window-3 reuse AO 0.143 -> 0.133 ms,
// shadows 0.334 -> 0.281 ms, GROUP 8 AO 24.5 -> 22.4 us with runs of 8, of
// 8-64 tiles and the plain block order; identical bits.)
constexpr int kRTileRun = 8;

__device__ inline void r_tile_of_block(int tiles_x, int ntiles, int &tx, int &ty) {
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    int t = (local / kRTileRun) * (8 * kRTileRun) + xcd * kRTileRun + local % kRTileRun;
    if (t >= ntiles) t = ntiles;  // out of range -> the block exits
    tx = t % tiles_x;
    ty = t / tiles_x;
}

// Blocks for r_tile_of_block: every tile has one.
static inline int r_grid_for(int ntiles) {
    const int per = (ntiles + 7) / 8;
    return 8 * ((per + kRTileRun - 1) / kRTileRun) * kRTileRun;
}

template <int MODE, bool UNB, class LT = LightF>
__global__ __launch_bounds__(kRBlock) void reuse_window_kernel(GBufView g, OccView occ, float R2, LT L,
                                                               const uint32_t *__restrict__ bits, int words, int R,
                                                               int dark_guard, int accumulate, float *out,
                                                               int tiles_x, int ntiles, float scale) {
    extern __shared__ __align__(16) unsigned char smem[];
    int tx, ty;
    r_tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;
    reuse_window_tile<MODE, UNB, LT>(smem, g, occ, R2, L, bits, words, R, dark_guard, accumulate, out, tx, ty, scale);
}

// Fixed groups.  Block = 32 x 8 pixels; the group shapes (1x1, 2x1, 2x2,
// 4x2) tile it exactly.  One lane per pixel, in three roles: as receiver k it
// evaluates the densities p_k(j) of its group's candidates; as candidate j it
// sums its denominator P(j) over the group's receivers once (every target of
// a group shares it); as target i it adds p_i(j) / P(j) over the candidates.
// The pixel's G-buffer entry, hit id and validation words are read in one
// round of loads, the hit's record in a second.  The group shape GW x GH is
// a template parameter: the member loops unroll and their indices are
// constants.
template <int MODE, bool UNB, class LT, int GW, int GH>
__global__ __launch_bounds__(kRBlock) void reuse_group_kernel(GBufView g, OccView occ, float R2, LT L,
                                                              const uint32_t *__restrict__ bits, int words, int D,
                                                              int dark_guard, int accumulate, float *out,
                                                              int tiles_x, int ntiles, float scale) {
    constexpr int N = GW * GH, gw = GW, gh = GH;
    __shared__ float s_o[3][kRBlock], s_dz[3][kRBlock], s_nz[3][kRBlock];
    __shared__ uint32_t s_hit[kRBlock];
    __shared__ uint8_t s_val[kRBlock];
    __shared__ uint32_t s_bits[2][UNB ? kRBlock : 1];
    __shared__ float s_p[N][kRBlock];  // s_p[m][k]: density of the group's candidate m at receiver k
    __shared__ float s_P[kRBlock];     // s_P[j]: denominator of candidate j

    int tx, ty;
    r_tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;
    const int tid = threadIdx.x;
    const int lx = tid & 31, ly = tid >> 5;
    const int px = tx * 32 + lx, py = ty * 8 + ly;
    const bool inside = px < g.w && py < g.h;
    const int64_t gi = inside ? (int64_t)py * g.w + px : 0;
    // first round: every load of the pixel issued together
    const uint32_t prim = inside ? g.prim[gi] : OCR_HIT_MISS;
    const uint32_t hit0 = inside ? occ.hit[gi] : OCR_HIT_MISS;
    float x[3] = {0.f, 0.f, 0.f}, n[3] = {0.f, 0.f, 0.f};
    uint32_t b0 = 0u, b1 = 0u;
    if (inside) {
        ld3(g.pos, gi, x);
        ld3(g.nrm, gi, n);
        if (UNB) {
            b0 = bits[gi * words];
            b1 = words > 1 ? bits[gi * words + 1] : 0u;
        }
    }
    const bool valid = prim != OCR_HIT_MISS;
    const uint32_t hit = valid ? hit0 : OCR_HIT_MISS;
    float o[3] = {0.f, 0.f, 0.f};
    if (valid) offset_point(x, n, o);
    else n[0] = n[1] = n[2] = 0.0f;
    for (int a = 0; a < 3; ++a) {
        s_o[a][tid] = o[a];
    }
    if (hit < OCR_HIT_SELF) {
        float dz[3], nz[3];
        ld3(occ.dz, gi, dz);
        ld3(occ.nz, gi, nz);
        for (int a = 0; a < 3; ++a) {
            s_dz[a][tid] = dz[a];
            s_nz[a][tid] = nz[a];
        }
    }
    // this lane's light terms as a receiver (its point, for several lights)
    const auto rk = recv_of(o, L);
    s_hit[tid] = hit;
    s_val[tid] = valid;
    if (UNB) {
        s_bits[0][tid] = valid ? b0 : 0u;
        s_bits[1][tid] = valid ? b1 : 0u;
    }
    __syncthreads();

    // this lane as receiver k: densities of the group's candidates
    const int gx0 = (lx / gw) * gw, gy0 = (ly / gh) * gh;
    const int SIDE = 2 * D + 1;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int mx = gx0 + m % gw, my = gy0 + m / gw;
        const int jt = my * 32 + mx;
        float p = 0.0f;
        if (valid && s_hit[jt] < OCR_HIT_SELF) {
            float oj[3] = {s_o[0][jt], s_o[1][jt], s_o[2][jt]};
            float dzj[3] = {s_dz[0][jt], s_dz[1][jt], s_dz[2][jt]};
            float nzj[3] = {s_nz[0][jt], s_nz[1][jt], s_nz[2][jt]};
            float w[3];
            rel_vec(oj, o, dzj, w);
            p = MODE == OCR_AO ? dens_ao(w, n, nzj, R2) : dens_light(w, n, rk, nzj, L);
            if (UNB && p > 0.0f) {
                const int bidx = (ly - my + D) * SIDE + (lx - mx + D);
                if (!((s_bits[bidx >> 5][jt] >> (bidx & 31)) & 1u)) p = 0.0f;
            }
        }
        s_p[m][tid] = p;
    }
    __syncthreads();

    // this lane as candidate j: P(j) over the group's receivers, in receiver order
    if (hit < OCR_HIT_SELF) {
        const int mj = (ly - gy0) * gw + (lx - gx0);
        float P = 0.0f;
#pragma unroll
        for (int k = 0; k < N; ++k) P += s_p[mj][(gy0 + k / gw) * 32 + gx0 + k % gw];
        s_P[tid] = P;
    }
    __syncthreads();

    // this lane as target i
    if (!inside) return;
    float B = 0.0f;
    int misses = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int mx = gx0 + m % gw, my = gy0 + m / gw;
        const int jt = my * 32 + mx;
        const uint32_t hj = s_hit[jt];
        if (s_val[jt] && hj == OCR_HIT_MISS) ++misses;
        if (hj >= OCR_HIT_SELF) continue;
        const float P = s_P[jt];
        const float pij = s_p[m][tid];
        if (pij > 0.0f && P > 0.0f) {
            float term = pij * __builtin_amdgcn_rcpf(P);
            if constexpr (MODE >= kShadowSA || kBilinear<LT>) {
                // times g_ij (solid angle) or gd_ij (direct illumination) of
                // this target and candidate m, over q_i(y'_ij) for the
                // bilinear emitter density
                const float oj[3] = {s_o[0][jt], s_o[1][jt], s_o[2][jt]};
                const float dzj[3] = {s_dz[0][jt], s_dz[1][jt], s_dz[2][jt]};
                float w[3];
                rel_vec(oj, o, dzj, w);
                if constexpr (MODE == kDI) term *= di_pair_g(w, n, rk.hk, L);
                else if constexpr (MODE == kShadowSA) term *= sa_pair_g(w, rk.hk, L);
                if constexpr (kBilinear<LT>) term *= inv_bilinear_q(w, rk, L);
            }
            B += term;
        }
    }
    float F = 1.0f;
    bool dark = false;
    if (MODE != OCR_AO && valid) {
        if constexpr (MODE == kShadowSA) {
            F = sa_estimate(o, n, L, B);
            B = 0.0f;
        } else if constexpr (MODE == kDI) {
            F = di_estimate(o, n, L, B, scale);
            B = 0.0f;
        } else {
            F = front_light(o, n, L);
        }
        dark = dark_guard && misses == 0;
    }
    out[gi] = finish(MODE, valid, B, F, dark, accumulate ? out[gi] : 0.0f, accumulate);
}

template <int MODE, class LT = LightF>
__global__ __launch_bounds__(kRBlock) void noreuse_kernel(GBufView g, OccView occ, LT L, int accumulate,
                                                          float *out, float scale) {
    const int64_t gi = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
    if (gi >= (int64_t)g.w * g.h) return;
    const float v = noreuse_value<MODE>(g, occ, L, gi, scale);
    out[gi] = accumulate ? out[gi] + v : v;
}

__global__ void scale_kernel(float *out, int64_t n, float s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] *= s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int MODE, bool UNB, class LT>
static hipError_t launch_win(const GBufView &g, const OccView &occ, float R2, const LT &L, const uint32_t *bits,
                             int words, const ocr_reuse_params &p, float *out, float scale, hipStream_t st) {
    int tiles_x = (g.w + kWTX - 1) / kWTX, tiles_y = (g.h + kWTY - 1) / kWTY;
    int nt = tiles_x * tiles_y;
    WinLayout lay = win_layout(p.radius, MODE, UNB, words, kRecvFloats<LT>);
    // dynamic-LDS limit raised so far (64 KB by default); several host
    // threads may launch at once
    static std::atomic<size_t> attr_bytes{64 * 1024};
    if (lay.total > attr_bytes.load()) {
        hipError_t e = hipFuncSetAttribute((const void *)reuse_window_kernel<MODE, UNB, LT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.total);
        if (e != hipSuccess) return e;
        size_t cur = attr_bytes.load();
        while (cur < lay.total && !attr_bytes.compare_exchange_weak(cur, lay.total)) {
        }
    }
    dim3 grid(r_grid_for(nt)), block(kRBlock);
    hipLaunchKernelGGL((reuse_window_kernel<MODE, UNB, LT>), grid, block, lay.total, st, g, occ, R2, L, bits, words,
                       p.radius, p.dark_guard, p.accumulate, out, tiles_x, nt, scale);
    return hipSuccess;
}

template <int MODE, bool UNB, class LT>
static void launch_grp(const GBufView &g, const OccView &occ, float R2, const LT &L, const uint32_t *bits,
                       int words, const ocr_reuse_params &p, float *out, float scale, hipStream_t st) {
    int tiles_x = (g.w + 31) / 32, tiles_y = (g.h + 7) / 8;
    int nt = tiles_x * tiles_y;
    dim3 grid(r_grid_for(nt)), block(kRBlock);
#define OCR_GRP(GW, GH)                                                                                        \
    hipLaunchKernelGGL((reuse_group_kernel<MODE, UNB, LT, GW, GH>), grid, block, 0, st, g, occ, R2, L, bits, words, \
                       pair_extent(p), p.dark_guard, p.accumulate, out, tiles_x, nt, scale)
    switch (p.group_n) {
        case 8: OCR_GRP(4, 2); break;
        case 4: OCR_GRP(2, 2); break;
        case 2: OCR_GRP(2, 1); break;
        default: OCR_GRP(1, 1); break;
    }
#undef OCR_GRP
}

template <int MODE, class LT = LightF>
static hipError_t launch_mode(const GBufView &g, const OccView &occ, float R2, const LT &L, const uint32_t *bits,
                              int words, const ocr_reuse_params &q, bool unb, float *out, float scale,
                              hipStream_t st) {
    if (q.estimator == OCR_NOREUSE) {
        int64_t n = (int64_t)g.w * g.h;
        dim3 grid((unsigned)((n + kRBlock - 1) / kRBlock)), block(kRBlock);
        hipLaunchKernelGGL((noreuse_kernel<MODE, LT>), grid, block, 0, st, g, occ, L, q.accumulate, out, scale);
        return hipSuccess;
    }
    if (q.pattern == OCR_WINDOW)
        return unb ? launch_win<MODE, true, LT>(g, occ, R2, L, bits, words, q, out, scale, st)
                   : launch_win<MODE, false, LT>(g, occ, R2, L, bits, words, q, out, scale, st);
    if (unb) launch_grp<MODE, true, LT>(g, occ, R2, L, bits, words, q, out, scale, st);
    else launch_grp<MODE, false, LT>(g, occ, R2, L, bits, words, q, out, scale, st);
    return hipSuccess;
}

hipError_t launch_reuse(const GBufView &g, const OccView &occ, int mode, float R, const LightF &L,
                        const ocr_reuse_params &p, const uint32_t *bits, float *out, hipStream_t st, float scale) {
    const float R2 = R * R;
    const int words = pair_words(p);
    const bool unb = p.estimator == OCR_UNBIASED;
    // the dark-region guard belongs to the biased estimators of the light modes only
    ocr_reuse_params q = p;
    q.dark_guard = (p.estimator == OCR_BIASED && p.dark_guard) ? 1 : 0;
    hipError_t e;
    switch (mode) {
        case OCR_AO: e = launch_mode<OCR_AO>(g, occ, R2, L, bits, words, q, unb, out, scale, st); break;
        case OCR_SHADOW: e = launch_mode<OCR_SHADOW>(g, occ, R2, L, bits, words, q, unb, out, scale, st); break;
        case kShadowSA: e = launch_mode<kShadowSA>(g, occ, R2, L, bits, words, q, unb, out, scale, st); break;
        default: e = launch_mode<kDI>(g, occ, R2, L, bits, words, q, unb, out, scale, st); break;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// several lights (shadows only)
hipError_t launch_reuse_lights(const GBufView &g, const OccView &occ, const LightSetF &L, const ocr_reuse_params &p,
                               const uint32_t *bits, float *out, hipStream_t st) {
    ocr_reuse_params q = p;
    q.dark_guard = (p.estimator == OCR_BIASED && p.dark_guard) ? 1 : 0;
    hipError_t e = launch_mode<OCR_SHADOW, LightSetF>(g, occ, 1.0f, L, bits, pair_words(p), q,
                                                      p.estimator == OCR_UNBIASED, out, 1.0f, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// one light sampled from the bilinear emitter density (shadows, solid-angle
// shadows, direct illumination)
hipError_t launch_reuse_bilinear(const GBufView &g, const OccView &occ, int mode, const LightBilinF &L,
                                 const ocr_reuse_params &p, const uint32_t *bits, float *out, hipStream_t st,
                                 float scale) {
    const int words = pair_words(p);
    const bool unb = p.estimator == OCR_UNBIASED;
    ocr_reuse_params q = p;
    q.dark_guard = (p.estimator == OCR_BIASED && p.dark_guard) ? 1 : 0;
    hipError_t e;
    switch (mode) {
        case OCR_SHADOW:
            e = launch_mode<OCR_SHADOW, LightBilinF>(g, occ, 1.0f, L, bits, words, q, unb, out, scale, st);
            break;
        case kShadowSA:
            e = launch_mode<kShadowSA, LightBilinF>(g, occ, 1.0f, L, bits, words, q, unb, out, scale, st);
            break;
        default: e = launch_mode<kDI, LightBilinF>(g, occ, 1.0f, L, bits, words, q, unb, out, scale, st); break;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_scale(float *out, int64_t n, float s, hipStream_t st) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(scale_kernel, grid, block, 0, st, out, n, s);
    return hipGetLastError();
}

}  // namespace ocr
