// The paper's simple reuse baselines (Sec. 6), kept for quality comparisons
// with occlusion-point reuse:
//   * final-value filtering, the paper's Filter (N) for AO and, for shadows,
//     Light (N) (light-sample reuse without visibility validation, which under
//     this formulation reduces to the same average): the mean of one-sample
//     estimates over the target's set;
//   * light-sample reuse with visibility re-evaluation, Light (NU): the target
//     re-traces the light sample of every pixel of its set.
#include "ocr_common.hpp"
#include "trace_pixel.hpp"
#include "traverse.hpp"

namespace ocr {

constexpr int kBBlock2 = 256;

// Reuse set of pixel (px, py) clipped to the image: the window of radius r
// (gw == 0) or the image-aligned gw x gh group (gw, gh powers of two).
__device__ inline void set_bounds(int px, int py, int r, int gw, int gh, int w, int h, int &x0, int &x1, int &y0,
                                  int &y1) {
    if (gw == 0) {
        x0 = px - r;
        x1 = px + r;
        y0 = py - r;
        y1 = py + r;
    } else {
        x0 = px & -gw;
        x1 = x0 + gw - 1;
        y0 = py & -gh;
        y1 = y0 + gh - 1;
    }
    x0 = max(x0, 0);
    y0 = max(y0, 0);
    x1 = min(x1, w - 1);
    y1 = min(y1, h - 1);
}

// 16 x 16 pixels per block, one 8 x 8 sub-tile per wavefront.
__device__ inline bool pixel_of(const GBufView &g, int &px, int &py) {
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    px = blockIdx.x * 16 + (wv & 1) * 8 + (ln & 7);
    py = blockIdx.y * 16 + (wv >> 1) * 8 + (ln >> 3);
    return px < g.w && py < g.h;
}

// out[i] = mean over the valid pixels of S(i) of in[j]; background keeps in[i].
__global__ __launch_bounds__(kBBlock2) void filter_kernel(GBufView g, const float *__restrict__ in, float *out,
                                                          int r, int gw, int gh, int accumulate) {
    int px, py;
    if (!pixel_of(g, px, py)) return;
    const int64_t i = (int64_t)py * g.w + px;
    float v = in[i];
    if (g.prim[i] != OCR_HIT_MISS) {
        int x0, x1, y0, y1;
        set_bounds(px, py, r, gw, gh, g.w, g.h, x0, x1, y0, y1);
        float acc = 0.0f;
        int m = 0;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const int64_t j = (int64_t)y * g.w + x;
                if (g.prim[j] == OCR_HIT_MISS) continue;
                acc += in[j];
                ++m;
            }
        v = acc / (float)m;
    }
    out[i] = accumulate ? out[i] + v : v;
}

// out[i] = (1/|S(i)|) sum_j V(x_i, y_j), y_j the light sample of pixel j.
// Every lane of a wave runs the same loop over the set's extent (lanes whose
// set is smaller, or that are outside the image, ride along), so that the
// segments whose per-lane walk overflowed its stack are decided together by
// a wave-coherent walk.
__global__ __launch_bounds__(kBBlock2) void light_reuse_kernel(DeviceBVH bvh, GBufView g, LightF L, uint32_t sd,
                                                               uint32_t sample, float *out, int r, int gw, int gh,
                                                               int accumulate) {
    __shared__ uint32_t stack[kStackLds * kBBlock2];
    __shared__ uint32_t wstack[kBBlock2 / 64][kStackTotal];
    int px, py;
    const bool inside = pixel_of(g, px, py);
    const int64_t i = inside ? (int64_t)py * g.w + px : 0;
    const uint32_t prim = inside ? g.prim[i] : OCR_HIT_MISS;
    float x[3] = {0.f, 0.f, 0.f}, n[3] = {0.f, 0.f, 0.f}, o[3] = {0.f, 0.f, 0.f};
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    if (prim != OCR_HIT_MISS) {
        load3(g.pos, i, x);
        load3(g.nrm, i, n);
        offset_point(x, n, o);
        set_bounds(px, py, r, gw, gh, g.w, g.h, x0, x1, y0, y1);
    }
    const int ex = gw == 0 ? 2 * r + 1 : gw, ey = gw == 0 ? 2 * r + 1 : gh;
    int vis = 0, m = 0;
    for (int dy = 0; dy < ey; ++dy)
        for (int dx = 0; dx < ex; ++dx) {
            const int y = y0 + dy, xx = x0 + dx;
            const bool in = y <= y1 && xx <= x1 && g.prim[(int64_t)y * g.w + xx] != OCR_HIT_MISS;
            bool want = false, overflow = false, blocked = false;
            TRay ray{};
            if (in) {
                ++m;
                float yl[3], d[3];
                light_point((uint32_t)xx, (uint32_t)y, sample, sd, L, yl);
                d[0] = yl[0] - o[0];
                d[1] = yl[1] - o[1];
                d[2] = yl[2] - o[2];
                if (shadow_traced(n, o, d, L)) {
                    want = true;
                    make_ray(o, d, prim, OCR_HIT_MISS, 1.0f, ray);
                    const Hit h = traverse<true, false>(bvh, ray, 1.0f, stack + threadIdx.x, kBBlock2, overflow);
                    blocked = h.tri != OCR_HIT_MISS;
                }
            }
            if (wave_ballot(overflow) != 0ull) {
                const TRay rr[1] = {ray};
                const bool wr[1] = {overflow};
                bool br[1];
                WalkStats st;
                traverse_wave_any<1>(bvh, rr, 1.0f, wr, br, wstack[threadIdx.x >> 6], st);
                if (overflow) blocked = br[0];
            }
            if (want && !blocked) ++vis;
        }
    if (!inside) return;
    const float v = prim != OCR_HIT_MISS ? (float)vis / (float)m : 0.0f;
    out[i] = accumulate ? out[i] + v : v;
}

static void set_shape(const ocr_reuse_params &p, int &r, int &gw, int &gh) {
    if (p.pattern == OCR_WINDOW) {
        r = p.radius;
        gw = gh = 0;
    } else {
        r = 0;
        group_dims(p.group_n, gw, gh);
    }
}

hipError_t launch_filter(const GBufView &g, const ocr_reuse_params &p, const float *in, float *out, hipStream_t st) {
    int r, gw, gh;
    set_shape(p, r, gw, gh);
    dim3 grid((g.w + 15) / 16, (g.h + 15) / 16), block(kBBlock2);
    hipLaunchKernelGGL(filter_kernel, grid, block, 0, st, g, in, out, r, gw, gh, p.accumulate);
    return hipGetLastError();
}

hipError_t launch_light_reuse(const DeviceBVH &bvh, const GBufView &g, const LightF &L, uint32_t seed32,
                              uint32_t sample, const ocr_reuse_params &p, float *out, hipStream_t st) {
    int r, gw, gh;
    set_shape(p, r, gw, gh);
    dim3 grid((g.w + 15) / 16, (g.h + 15) / 16), block(kBBlock2);
    hipLaunchKernelGGL(light_reuse_kernel, grid, block, 0, st, bvh, g, L, seed32, sample, out, r, gw, gh,
                       p.accumulate);
    return hipGetLastError();
}

}  // namespace ocr
