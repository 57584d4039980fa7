// Batched schedule kernels: many views of uneven size, over several scenes
// and mixed effects, in one persistent trace launch and one persistent reuse
// launch over a (view, tile) work list.  (The paper runs one view per pass.)
//
// The work items are split into 8 contiguous ranges, one per XCD (blocks are
// dealt to the XCDs round-robin, so block b starts on range b mod 8), which
// keeps the BVH nodes and G-buffer rows a range touches in that XCD's L2.
// Items are taken from a range with an atomic counter; a wave (trace) or
// block (reuse) whose range is exhausted moves on to the next range, so the
// ranges balance at the end whatever the per-item cost.  Every counter is
// incremented at most (its range size + the number of takers) times, and each
// taker leaves after seeing all 8 ranges exhausted, so the grid drains.
//
// A pixel's arithmetic is exactly the per-view kernels' (trace_pixel and
// reuse_window_tile are shared), so results are bitwise identical.
#include "batch.hpp"
#include "density.hpp"
#include "ocr_common.hpp"
#include "reuse_tile.hpp"
#include "trace_pixel.hpp"

namespace ocr {

constexpr int kBBlock = 256;

__global__ __launch_bounds__(64) void batch_reset_kernel(uint32_t *ctr) {
    if (threadIdx.x < 16) ctr[threadIdx.x * kQueueStride] = 0u;
}

// Index of the view whose item range [first[v], first[v+1]) holds `item`
// (binary search; views with empty ranges are skipped naturally).
__device__ inline int find_view(const uint32_t *__restrict__ first, int nviews, uint32_t item) {
    int lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline uint32_t compact_bits(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

// Pixel (lx, ly) of a tile_w x tile_h tile (powers of two, >= 8) that lane
// `lane` takes in pass `it`.
__device__ inline void tile_pixel(int packing, int tw, int th, int it, int lane, int &lx, int &ly) {
    if (packing == OCR_PACK_ROW) {
        const int i = it * 64 + lane;
        lx = i % tw;
        ly = i / tw;
    } else if (packing == OCR_PACK_BLOCK8) {
        const int bw = tw >> 3;
        lx = (it % bw) * 8 + (lane & 7);
        ly = (it / bw) * 8 + (lane >> 3);
    } else {
        // Morton order over the largest square of the tile, squares side by side
        const uint32_t i = (uint32_t)(it * 64 + lane);
        const int m = 31 - __clz(tw < th ? tw : th);  // log2 of the square side
        const uint32_t low = i & ((1u << (2 * m)) - 1u), high = i >> (2 * m);
        lx = (int)compact_bits(low);
        ly = (int)compact_bits(low >> 1);
        if (tw >= th) lx += (int)(high << m);
        else ly += (int)(high << m);
    }
}

// One wave per trace item: the wave traces the item's tile_w x tile_h pixels
// in (tile_w * tile_h / 64) passes of one ray per lane.  Bounded to 7 waves
// per SIMD: with both effects' walks inlined it takes 82 registers (5 waves)
// otherwise, measured 4% slower.
__global__ __launch_bounds__(kBBlock, 7) void batch_trace_kernel(const BatchView *__restrict__ views,
                                                              const uint32_t *__restrict__ t_first,
                                                              const uint32_t *__restrict__ t_tiles_x, int nviews,
                                                              const uint32_t *__restrict__ q_start, uint32_t *ctr,
                                                              int tw, int th, int packing) {
    __shared__ uint32_t stack[kStackLds * kBBlock];
    __shared__ uint32_t wstack[kBBlock / 64][kStackTotal];
    const int lane = threadIdx.x & 63;
    const int home = blockIdx.x & 7;
    const int passes = (tw * th) >> 6;
    int k = 0;
    while (k < 8) {
        const int x = (home + k) & 7;
        uint32_t idx = 0;
        if (lane == 0) idx = atomicAdd(&ctr[x * kQueueStride], 1u);
        idx = __builtin_amdgcn_readfirstlane(idx);
        const uint32_t end = q_start[x + 1];
        if (idx >= end - q_start[x]) {
            ++k;
            continue;
        }
        const uint32_t item = q_start[x] + idx;
        const int v = find_view(t_first, nviews, item);
        const BatchView &V = views[v];
        const uint32_t t = item - t_first[v], tx_n = t_tiles_x[v];
        const int tx = (int)(t % tx_n), ty = (int)(t / tx_n);
        const int w = V.g.w, h = V.g.h;
        for (int it = 0; it < passes; ++it) {
            int lx, ly;
            tile_pixel(packing, tw, th, it, lane, lx, ly);
            const int px = tx * tw + lx, py = ty * th + ly;
            // every lane calls (the view's mode is the wave's)
            if (V.mode == OCR_AO)
                trace_pixel<OCR_AO>(V.bvh, V.g, V.R, V.L, V.sd, V.sample, V.occ, px, py, px < w && py < h,
                                    stack + threadIdx.x, kBBlock, wstack[threadIdx.x >> 6]);
            else
                trace_pixel<OCR_SHADOW>(V.bvh, V.g, V.R, V.L, V.sd, V.sample, V.occ, px, py, px < w && py < h,
                                        stack + threadIdx.x, kBBlock, wstack[threadIdx.x >> 6]);
        }
    }
}

// One block per reuse item (a window target tile of a window or no-reuse view).
// Bounded to 7 waves per SIMD: every mode's body is inlined, and the
// heaviest (light effects) spill a few words at 72 registers, but the
// sixteen-view plan measured 3% faster than at 6 waves (4.33 against 4.46 ms,
// identical outputs; 8 waves 4.40 ms).
__global__ __launch_bounds__(kRBlock, 7) void batch_reuse_kernel(const BatchView *__restrict__ views,
                                                              const uint32_t *__restrict__ r_first, int nviews,
                                                              const uint32_t *__restrict__ q_start, uint32_t *ctr) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_item;
    const int home = blockIdx.x & 7;
    int k = 0;  // thread 0's position in the range sequence
    while (true) {
        __syncthreads();  // the previous item's LDS reads are done
        if (threadIdx.x == 0) {
            uint32_t item = 0xFFFFFFFFu;
            while (k < 8) {
                const int x = (home + k) & 7;
                const uint32_t idx = atomicAdd(&ctr[(8 + x) * kQueueStride], 1u);
                if (idx < q_start[9 + x + 1] - q_start[9 + x]) {
                    item = q_start[9 + x] + idx;
                    break;
                }
                ++k;
            }
            s_item = item;
        }
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item == 0xFFFFFFFFu) return;
        const int v = find_view(r_first, nviews, item);
        const BatchView &V = views[v];
        const uint32_t t = item - r_first[v];
        const int tx = (int)(t % (uint32_t)V.r_tiles_x), ty = (int)(t / (uint32_t)V.r_tiles_x);
        if (V.estimator == OCR_NOREUSE) {
            for (int t = threadIdx.x; t < kWTX * kWTY; t += kRBlock) {
                const int px = tx * kWTX + t % kWTX, py = ty * kWTY + t / kWTX;
                if (px < V.g.w && py < V.g.h) {
                    const int64_t gi = (int64_t)py * V.g.w + px;
                    float v;
                    switch (V.mode) {
                        case OCR_AO: v = noreuse_value<OCR_AO>(V.g, V.occ, V.L, gi, 1.0f); break;
                        case OCR_SHADOW: v = noreuse_value<OCR_SHADOW>(V.g, V.occ, V.L, gi, 1.0f); break;
                        case kShadowSA: v = noreuse_value<kShadowSA>(V.g, V.occ, V.L, gi, 1.0f); break;
                        default: v = noreuse_value<kDI>(V.g, V.occ, V.L, gi, V.scale); break;
                    }
                    V.out[gi] = v;
                }
            }
            continue;
        }
        const bool unb = V.estimator == OCR_UNBIASED;
        switch (V.mode) {
            case OCR_AO:
                if (unb)
                    reuse_window_tile<OCR_AO, true>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius, 0, 0,
                                                    V.out, tx, ty);
                else
                    reuse_window_tile<OCR_AO, false>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius, 0, 0,
                                                     V.out, tx, ty);
                break;
            case OCR_SHADOW:
                if (unb)
                    reuse_window_tile<OCR_SHADOW, true>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius,
                                                        V.dark_guard, 0, V.out, tx, ty);
                else
                    reuse_window_tile<OCR_SHADOW, false>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius,
                                                         V.dark_guard, 0, V.out, tx, ty);
                break;
            case kShadowSA:
                if (unb)
                    reuse_window_tile<kShadowSA, true>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius,
                                                       V.dark_guard, 0, V.out, tx, ty);
                else
                    reuse_window_tile<kShadowSA, false>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius,
                                                        V.dark_guard, 0, V.out, tx, ty);
                break;
            default:
                if (unb)
                    reuse_window_tile<kDI, true>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius,
                                                 V.dark_guard, 0, V.out, tx, ty, V.scale);
                else
                    reuse_window_tile<kDI, false>(smem, V.g, V.occ, V.R2, V.L, V.bits, V.words, V.radius,
                                                  V.dark_guard, 0, V.out, tx, ty, V.scale);
                break;
        }
    }
}

size_t batch_reuse_lds(int radius, int mode, bool unbiased, int words) {
    return win_layout(radius, mode, unbiased, words).total;
}

hipError_t launch_batch_reset(uint32_t *ctr, hipStream_t st) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, ctr);
    return hipGetLastError();
}

hipError_t launch_batch_trace(const BatchView *views, const uint32_t *t_first, const uint32_t *t_tiles_x, int nviews,
                              const uint32_t *q_start, uint32_t *ctr, int tile_w, int tile_h, int packing, int grid,
                              hipStream_t st) {
    hipLaunchKernelGGL(batch_trace_kernel, dim3(grid), dim3(kBBlock), 0, st, views, t_first, t_tiles_x, nviews,
                       q_start, ctr, tile_w, tile_h, packing);
    return hipGetLastError();
}

hipError_t launch_batch_reuse(const BatchView *views, const uint32_t *r_first, int nviews, const uint32_t *q_start,
                              uint32_t *ctr, size_t lds_bytes, int grid, hipStream_t st) {
    // (the dynamic-LDS limit was raised by batch_reuse_blocks_per_cu, outside any capture)
    hipLaunchKernelGGL(batch_reuse_kernel, dim3(grid), dim3(kRBlock), lds_bytes, st, views, r_first, nviews,
                       q_start, ctr);
    return hipGetLastError();
}

int batch_trace_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_trace_kernel, kBBlock, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

int batch_reuse_blocks_per_cu(size_t lds_bytes) {
    int n = 0;
    if (lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute((const void *)batch_reuse_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_reuse_kernel, kRBlock, lds_bytes) != hipSuccess ||
        n < 1)
        n = 1;
    return n;
}

}  // namespace ocr
