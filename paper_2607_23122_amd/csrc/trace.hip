// First-hit occluder tracing (step 1 of App. D / App. H) and the first-hit
// validation rays of the unbiased estimators (Eq. occ-first-hit).
#include "density.hpp"
#include "ocr_common.hpp"
#include "trace_pixel.hpp"
#include "traverse.hpp"

namespace ocr {

constexpr int kBlock = 256;
constexpr int kTile = 16;  // 16 x 16 pixels per block, one 8 x 8 sub-tile per wave

// Blocks are dealt to the 8 XCDs round-robin; remap so that each XCD takes
// runs of kTileRun consecutive tiles (row-major) in turn: XCD x gets tile
// runs x, x + 8, ...  A run's rays share much of their BVH paths in that
// XCD's L2, and every XCD samples the whole frame, so the XCDs finish
// together.  (One contiguous band of tiles per XCD left XCDs idle at the end:
// 1080p trace AO 0.385 -> 0.344 ms and shadows 0.43 -> 0.32 ms with runs of 16,
// the fastest of 8-64 tiles and of the plain block order; identical records.)
constexpr int kTileRun = 16;

__device__ inline void tile_of_block(int tiles_x, int ntiles, int &tx, int &ty) {
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    int t = (local / kTileRun) * (8 * kTileRun) + xcd * kTileRun + local % kTileRun;
    if (t >= ntiles) t = ntiles;  // out of range -> caller exits
    tx = t % tiles_x;
    ty = t / tiles_x;
}

__device__ inline void pixel_of_thread(int tx, int ty, int &px, int &py) {
    int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    px = tx * kTile + (wv & 1) * 8 + (ln & 7);
    py = ty * kTile + (wv >> 1) * 8 + (ln >> 3);
}

template <int MODE, class LT = LightF>
__global__ __launch_bounds__(kBlock) void trace_kernel(DeviceBVH bvh, GBufView g, float R, LT L, uint32_t sd,
                                                       uint32_t sample, OccView out, int tiles_x, int ntiles) {
    __shared__ uint32_t stack[kStackLds * kBlock];
    __shared__ uint32_t wstack[kBlock / 64][kStackTotal];
    int tx, ty;
    tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;  // the whole block
    int px, py;
    pixel_of_thread(tx, ty, px, py);
    trace_pixel<MODE, false, LT>(bvh, g, R, L, sd, sample, out, px, py, px < g.w && py < g.h, stack + threadIdx.x,
                                 kBlock, wstack[threadIdx.x >> 6]);
}

// Shadow records of several lights with wave-coherent walks: the wave walks
// the BVH once for the segments of its 8x8 pixels (traverse_wave_closest)
// instead of 64 per-lane walks, which diverge when neighbouring pixels'
// samples lie on different lights (measured 9% faster for two lights at
// 1080p; for one light the per-lane walks are as coherent and 3% faster).
// The same samples and records as trace_kernel (the closest hit does not
// depend on the walk's order); every lane reaches the walk.
template <class LT>
__global__ __launch_bounds__(kBlock) void trace_shadow_wave_kernel(DeviceBVH bvh, GBufView g, LT L, uint32_t sd,
                                                                   uint32_t sample, OccView out, int tiles_x,
                                                                   int ntiles) {
    __shared__ uint32_t wstack[kBlock / 64][kStackTotal];
    int tx, ty;
    tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;  // the whole block
    int px, py;
    pixel_of_thread(tx, ty, px, py);
    const int wave = threadIdx.x >> 6;
    const bool inside = px < g.w && py < g.h;
    const int64_t i = inside ? (int64_t)py * g.w + px : 0;
    const uint32_t prim = inside ? g.prim[i] : OCR_HIT_MISS;
    TRay r{};
    float d[3] = {0.f, 0.f, 0.f};
    bool want = false;
    if (prim != OCR_HIT_MISS) {
        float x[3], n[3], o[3], y[3];
        load3(g.pos, i, x);
        load3(g.nrm, i, n);
        offset_point(x, n, o);
        LightF Lc;  // the light the sample lies on
        pick_light((uint32_t)px, (uint32_t)py, sample, sd, L, o, y, Lc);
        d[0] = y[0] - o[0];
        d[1] = y[1] - o[1];
        d[2] = y[2] - o[2];
        want = shadow_traced(n, o, d, Lc);
        if (want) make_ray(o, d, prim, OCR_HIT_MISS, 1.0f, r);
    }
    const Hit h = traverse_wave_closest<false>(bvh, r, 1.0f, want, wstack[wave]);
    if (!inside) return;
    if (!want) {
        out.hit[i] = prim == OCR_HIT_MISS ? OCR_HIT_MISS : OCR_HIT_SELF;
        return;
    }
    out.hit[i] = h.tri;
    if (h.tri == OCR_HIT_MISS) return;
    float nz[3];
    oriented_normal(bvh, h.leaf_tri, d, nz);
    for (int c = 0; c < 3; ++c) {
        out.dz[3 * i + c] = h.t * d[c];
        out.nz[3 * i + c] = nz[c];
    }
}

// The trace with its walk work counted (walks, node visits, box and
// triangle tests, rays), summed over the wave and added to stats[0..4].  Same
// records as trace_kernel; used for work accounting, not timed.
template <int MODE>
__global__ __launch_bounds__(kBlock) void trace_count_kernel(DeviceBVH bvh, GBufView g, float R, LightF L,
                                                             uint32_t sd, uint32_t sample, OccView out, int tiles_x,
                                                             int ntiles, uint64_t *stats) {
    __shared__ uint32_t stack[kStackLds * kBlock];
    __shared__ uint32_t wstack[kBlock / 64][kStackTotal];
    int tx, ty;
    tile_of_block(tiles_x, ntiles, tx, ty);
    if (ty * tiles_x + tx >= ntiles) return;  // the whole block
    int px, py;
    pixel_of_thread(tx, ty, px, py);
    WalkStats ws;
    trace_pixel<MODE, true>(bvh, g, R, L, sd, sample, out, px, py, px < g.w && py < g.h, stack + threadIdx.x, kBlock,
                            wstack[threadIdx.x >> 6], &ws);
    uint64_t v[5] = {ws.walks, ws.nodes, ws.box_tests, ws.tri_tests, ws.walks};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) atomicAdd((unsigned long long *)&stats[k], (unsigned long long)v[k]);
    }
}

// Candidate lists for the window validation: every pixel whose ray found an
// occluder.  One list per XCD (blocks are dealt to the XCDs round-robin):
// XCD x compacts a contiguous band of ceil(ntiles / 8) tiles, a block
// kCompactTiles consecutive tiles of the band, appending their
// candidates (tile by tile, in pixel order within a wave) to list x with a
// single atomic, and the validation blocks of XCD x consume list x, so each
// XCD's L2 sees one contiguous set of tiles.  (The appends to one counter
// are serialised at the cache: with one tile per block, the 1080p
// compaction took ~16 us for ~1000 appends per counter.)  Layout: counts[8]
// (padded to a cache line each), then list x at offset x * per_xcd.  Only
// candidates' validation words are ever read, so other pixels' words are
// left as they are.
constexpr int kCountStride = 32;  // uint32 per counter: one 128-byte line
constexpr int kCompactTiles = 4;  // tiles per compaction block

__global__ __launch_bounds__(kBlock) void clear_count_kernel(uint32_t *lists) {
    if (threadIdx.x < 8) lists[threadIdx.x * kCountStride] = 0u;
}

// Blocks: 8 * ceil(ceil(ntiles / 8) / kCompactTiles).
__global__ __launch_bounds__(kBlock) void compact_kernel(GBufView g, OccView occ, uint32_t *lists, uint32_t per_xcd,
                                                         int tiles_x, int ntiles) {
    __shared__ uint32_t s_wave[kCompactTiles][kBlock / 64];
    __shared__ uint32_t s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t xcd = blockIdx.x & 7;
    const int per = (ntiles + 7) / 8;
    const int band_end = min((int)(xcd + 1) * per, ntiles);
    int64_t jj[kCompactTiles];
    unsigned long long m[kCompactTiles];
#pragma unroll
    for (int i = 0; i < kCompactTiles; ++i) {
        // this block's i-th tile of XCD xcd's band
        const int t = (int)xcd * per + (int)(blockIdx.x >> 3) * kCompactTiles + i;
        bool cand = false;
        jj[i] = 0;
        if (t < band_end) {
            int px, py;
            pixel_of_thread(t % tiles_x, t / tiles_x, px, py);
            if (px < g.w && py < g.h) {
                jj[i] = (int64_t)py * g.w + px;
                cand = occ.hit[jj[i]] < OCR_HIT_SELF;
            }
        }
        m[i] = __ballot(cand);
        if (lane == 0) s_wave[i][wave] = (uint32_t)__popcll(m[i]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0;
        for (int i = 0; i < kCompactTiles; ++i)
            for (int w2 = 0; w2 < kBlock / 64; ++w2) total += s_wave[i][w2];
        s_base = total ? atomicAdd(&lists[xcd * kCountStride], total) : 0u;
    }
    __syncthreads();
    uint32_t off = s_base;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < kCompactTiles; ++i) {
        uint32_t o = off;
        for (int w2 = 0; w2 < wave; ++w2) o += s_wave[i][w2];
        if ((m[i] >> lane) & 1ull)
            lists[8 * kCountStride + xcd * per_xcd + o + __popcll(m[i] & below)] = (uint32_t)jj[i];
        for (int w2 = 0; w2 < kBlock / 64; ++w2) off += s_wave[i][w2];
    }
}

constexpr int kMaxPairs = 33 * 33;             // (4r+1)^2 at r = 8
constexpr int kMaxWords = (kMaxPairs + 31) / 32;

// receiver k of candidate j at pair index q, its offset point and the segment
// vector w = z_j - o_k; false if k is outside the image or background
__device__ inline bool pair_receiver(const GBufView &g, int jx, int jy, int side, float inv_side, int D, int q,
                                     int64_t &k, uint32_t &primk, float ok[3], float nk[3]) {
    const int qy = small_div(q, inv_side);
    const int kx = jx + (q - qy * side) - D, ky = jy + qy - D;
    if (kx < 0 || kx >= g.w || ky < 0 || ky >= g.h) return false;
    k = (int64_t)ky * g.w + kx;
    // the three loads issue together; background is decided afterwards
    float xk[3];
    primk = g.prim[k];
    load3(g.pos, k, xk);
    load3(g.nrm, k, nk);
    if (primk == OCR_HIT_MISS) return false;
    offset_point(xk, nk, ok);
    return true;
}

// First-hit validation (Eq. occ-first-hit) for the sliding window.  The
// receivers k = j + (q % side - D, q / side - D), side = 2D + 1, D = 2r, of a
// candidate j whose density of z_j is positive are gathered (lane q of each
// 64-wide round) into a list in LDS, and the wave walks the BVH once per 64
// listed pairs: an any-hit segment o_k -> z_j over t in (0, 1 - 1e-4),
// ignoring z_j's triangle and k's own, decides Occ(x_k, z_j)
// (traverse_wave_any; each lane its own segment).  Bit q of j's words is set
// when z_j is the first hit from o_k (k == j: always).  A wave takes a run of
// consecutive candidates and lists the pairs of all of them, tagged with the
// candidate's place in the run, before walking: a shadow candidate has a few
// pairs (the light subtends a narrow cone), so a walk per candidate would
// leave most lanes idle, while neighbouring candidates' segments head for the
// same light from nearby points and share most of their path through the
// BVH; an AO candidate has dozens, and short runs only fill its last, partly
// empty walk.  The list is walked early when the next candidate might not
// fit.  An oversubscribed grid (12288 blocks) strides through the concatenated
// candidate lists (tile order) in blocks of kRunBlock runs dealt to the XCDs
// in turn: an XCD works on a few small parts of the frame at a time, so its
// L2 holds the part of the hierarchy their segments meet (1080p AO: 0.55 GB
// fetched per launch instead of 1.5 GB), while every XCD still samples the
// whole frame and the dispatcher balances the uneven per-run work at block
// granularity.  (Measured faster than one contiguous eighth of the runs per
// XCD, which fetched 0.25 GB but left XCDs idle at the end, than a
// resident-sized grid, and than taking runs from atomic counters; blocks of
// 256 runs were the fastest of 16-1024; run lengths 6 for the light effects
// and 4 for AO were the fastest measured, and for fixed groups 16 and 8 of
// the tried 6-24.)
constexpr int kLightRun = 6;                   // candidates per run, light effects
constexpr int kAoRun = 4;                      // candidates per run, AO
constexpr int kGroupAoRun = 8;                 // candidates per run, fixed groups, AO
constexpr int kGroupLightRun = 16;             // candidates per run, fixed groups, light effects
constexpr int kRunWords = 128;                 // validation words of a run in LDS
constexpr uint32_t kRunBlock = 256;            // consecutive runs an XCD takes at a time
static_assert(kRunWords >= kMaxWords, "a run holds at least one candidate's words");

// A candidate of the current run, as its walks need it.
struct RunCand {
    float oj[3], dzj[3];
    int32_t jx, jy;
    uint32_t hj;
    int32_t pad;
};

// COUNT: the work-accounting instantiation (lane-masked walk, same bits),
// which adds the segments' useful work to stats[0..4].  Bounded to 7 waves
// per SIMD (72 registers; a few words spill in the counting forms): at
// its natural register count (5 waves) the walk ran 12% slower.
//
// GROUP: the fixed groups of N pixels (2^lgw x 2^lgh, aligned to the image
// origin; D = the group extent).  The receivers of j are the other members of
// its group, so an offset q is listed only when it stays in j's group; the
// bit of pair (j, k) is the same offset bit.  A group candidate has at most
// N - 1 segments, so runs are longer.
template <int MODE, bool COUNT, class LT = LightF, bool GROUP = false>
__global__ __launch_bounds__(kBlock, 7) void validate_window_kernel(DeviceBVH bvh, GBufView g, OccView occ, float R2,
                                                                 LT L, int D, int words, uint32_t *bits,
                                                                 const uint32_t *lists, uint32_t per_xcd,
                                                                 uint64_t *stats, int lgw, int lgh) {
    constexpr int kRun = GROUP ? (MODE == OCR_AO ? kGroupAoRun : kGroupLightRun) : (MODE == OCR_AO ? kAoRun : kLightRun);
    // AO window runs (about 120 segments per candidate) start their walks at
    // the run's entry node; shadow candidates have a segment or two, and
    // groups at most N - 1, too few to pay for the per-candidate reductions
    constexpr bool kEntry = MODE == OCR_AO && !GROUP && !COUNT;
    __shared__ uint32_t wnode[kBlock / 64][kStackTotal];
    __shared__ unsigned long long wmask[kBlock / 64][COUNT ? kStackTotal : 1];
    // listed pairs: (place in the run << 11) | q
    __shared__ uint16_t wq[kBlock / 64][kMaxPairs];
    __shared__ uint32_t wbits[kBlock / 64][kRunWords];
    __shared__ RunCand wcand[kBlock / 64][kRun];
    WalkStats ws;
    // wave-uniform by construction; readfirstlane lets the compiler keep the
    // candidate bookkeeping derived from it in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int side = 2 * D + 1, npairs = side * side;
    const float inv_side = 1.0f / (float)side;
    const int qself = D * side + D;
    // candidates per run: bounded by the run's words in LDS
    const int run = min(kRun, kRunWords / words);
    // the 8 lists concatenated (roughly tile order); consecutive runs go to
    // the waves of one block, which then share the CU's caches
    uint32_t total = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) total += lists[x * kCountStride];
    // runs in blocks of kRunBlock; XCD x (blocks x, x + 8, ...) takes run blocks x,
    // x + 8, ...
    const uint32_t nruns = (total + (uint32_t)run - 1) / (uint32_t)run;
    const uint32_t xcd = blockIdx.x & 7;
    const uint32_t stride = (gridDim.x / 8) * (kBlock / 64);
    for (uint32_t u = (blockIdx.x >> 3) * (kBlock / 64) + wave;; u += stride) {
        const uint32_t ri = (u / kRunBlock) * (8u * kRunBlock) + xcd * kRunBlock + (u % kRunBlock);
        if (ri >= nruns) {
            if ((u / kRunBlock) * (8u * kRunBlock) >= nruns) break;
            continue;
        }
        const uint32_t c0 = ri * (uint32_t)run;
        const int nrun = (int)min((uint32_t)run, total - c0);
        for (int w = lane; w < nrun * words; w += 64) wbits[wave][w] = 0u;
        wave_sync();
        int count = 0, done = 0;  // listed pairs; candidates whose words are written
        // the box of the listed segments (wave-uniform), for the walks'
        // common entry node
        float slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
        // Walk the listed pairs (each lane its own segment), then write the
        // words of the candidates gathered so far.
        auto flush = [&](int upto) {
            wave_sync();
            // the listed segments of a run lie close together: their walks
            // start below the levels where their box meets one child only
            const uint32_t entry = kEntry ? entry_node(bvh, slo, shi) : 0u;
            for (int a = 0; a < 3; ++a) {
                slo[a] = INFINITY;
                shi[a] = -INFINITY;
            }
            for (int e0 = 0; e0 < count; e0 += 64) {
                TRay r;
                r.ign0 = r.ign1 = OCR_HIT_MISS;
                const int idx = e0 + lane;
                const bool want = idx < count;
                int q = 0, b = 0;
                if (want) {
                    const uint32_t e = wq[wave][idx];
                    b = (int)(e >> 11);
                    q = (int)(e & 2047u);
                    const RunCand &c = wcand[wave][b];
                    int64_t k;
                    uint32_t primk;
                    float ok[3], nk[3], w[3];
                    pair_receiver(g, c.jx, c.jy, side, inv_side, D, q, k, primk, ok, nk);
                    rel_vec(c.oj, ok, c.dzj, w);
                    make_ray(ok, w, c.hj, primk, 1.0f - 1e-4f, r);
                }
                bool blocked;
                if (COUNT) {
                    blocked = traverse_wave_any_masked(bvh, r, 1.0f - 1e-4f, want, wnode[wave], wmask[wave], ws);
                } else {
                    TRay rr[1] = {r};
                    const bool wr[1] = {want};
                    bool br[1];
                    traverse_wave_any<1>(bvh, rr, 1.0f - 1e-4f, wr, br, wnode[wave], ws, entry);
                    blocked = br[0];
                }
                if (want && !blocked) atomicOr(&wbits[wave][b * words + (q >> 5)], 1u << (q & 31));
            }
            wave_sync();
            for (int b = done; b < upto; ++b) {
                const RunCand &c = wcand[wave][b];
                if constexpr (kEntry) {
                    // the candidate's words as a wave-uniform base plus a
                    // 32-bit lane offset; the empty asm keeps the compiler
                    // from hoisting a per-lane 64-bit address out of the run
                    // loop, which this form (the largest) had to spill at the
                    // register bound: 8 bytes per lane stored once per wave,
                    // 25 MB of writes per 1080p AO launch.  (The other forms
                    // keep it in a register; given the same code, shadows
                    // measured 4% slower.)
                    const int jx = __builtin_amdgcn_readfirstlane(c.jx), jy = __builtin_amdgcn_readfirstlane(c.jy);
                    uint32_t *dst = bits + ((int64_t)jy * g.w + jx) * words;
                    int w0 = lane;
                    asm volatile("" : "+v"(w0));
                    for (int w = w0; w < words; w += 64) dst[w] = wbits[wave][b * words + w];
                } else {
                    const int64_t j = (int64_t)c.jy * g.w + c.jx;
                    for (int w = lane; w < words; w += 64) bits[j * words + w] = wbits[wave][b * words + w];
                }
            }
            done = upto;
            count = 0;
            wave_sync();  // the list is read before it is refilled
        };
        for (int b = 0; b < nrun; ++b) {
            // room for this candidate's pairs in the list (walked first,
            // before this candidate's data is loaded, so that nothing of it
            // lives across the walk)
            if (count + npairs - 1 > kMaxPairs) flush(b);
            // list x and the position in it of candidate c0 + b (scalar)
            uint32_t off = c0 + (uint32_t)b, base = 8 * kCountStride;
#pragma unroll
            for (int x = 0; x < 7; ++x) {
                const uint32_t n = lists[x * kCountStride];
                if (off >= n) {
                    off -= n;
                    base += per_xcd;
                } else {
                    break;
                }
            }
            const int64_t j = __builtin_amdgcn_readfirstlane((int)lists[base + off]);
            const int jy = (int)((uint32_t)j / (uint32_t)g.w), jx = (int)j - jy * g.w;
            const uint32_t hj = occ.hit[j];
            float xj[3], nj[3], oj[3], dzj[3], nzj[3];
            load3(g.pos, j, xj);
            load3(g.nrm, j, nj);
            offset_point(xj, nj, oj);
            load3(occ.dz, j, dzj);
            load3(occ.nz, j, nzj);
            // this candidate's segments: z_j = o_j + dz_j and this lane's receivers
            float clo[3], chi[3];
            for (int a = 0; a < 3; ++a) clo[a] = chi[a] = oj[a] + dzj[a];
            if (lane == 0) {
                RunCand &c = wcand[wave][b];
                for (int a = 0; a < 3; ++a) {
                    c.oj[a] = oj[a];
                    c.dzj[a] = dzj[a];
                }
                c.jx = jx;
                c.jy = jy;
                c.hj = hj;
                // z_j is its own first hit
                atomicOr(&wbits[wave][b * words + (qself >> 5)], 1u << (qself & 31));
            }
            // the receivers with positive density, listed in q order
            for (int qb = 0; qb < npairs; qb += 64) {
                const int q = qb + lane;
                bool want = false;
                int64_t k;
                uint32_t primk;
                float ok[3], nk[3];
                bool member = q < npairs;
                if (GROUP && member) {
                    // k = j + (q % side - D, q / side - D) in j's group (a negative
                    // coordinate shifts to a negative group index: never j's)
                    const int qy = small_div(q, inv_side);
                    const int kx = jx + (q - qy * side) - D, ky = jy + qy - D;
                    member = (kx >> lgw) == (jx >> lgw) && (ky >> lgh) == (jy >> lgh);
                }
                if (member && pair_receiver(g, jx, jy, side, inv_side, D, q, k, primk, ok, nk) && k != j) {
                    float w[3];
                    rel_vec(oj, ok, dzj, w);
                    float p;
                    if (MODE == OCR_AO) {
                        p = dens_ao(w, nk, nzj, R2);
                    } else {
                        p = dens_light(w, nk, recv_of(ok, L), nzj, L);
                    }
                    want = p > 0.0f;
                    if (want && kEntry) {
                        for (int a = 0; a < 3; ++a) {
                            clo[a] = fminf(clo[a], ok[a]);
                            chi[a] = fmaxf(chi[a], ok[a]);
                        }
                    }
                }
                const unsigned long long m = __ballot(want);
                if (want) wq[wave][count + __popcll(m & below)] = (uint16_t)((b << 11) | q);
                count += __popcll(m);
            }
            if (kEntry) {
                // into the run's box (wave-uniform: scalar registers)
                for (int a = 0; a < 3; ++a) {
                    slo[a] = uniform_f(fminf(slo[a], wave_fmin(clo[a])));
                    shi[a] = uniform_f(fmaxf(shi[a], wave_fmax(chi[a])));
                }
            }
        }
        flush(nrun);
    }
    if (COUNT && lane == 0) {
        atomicAdd((unsigned long long *)&stats[0], (unsigned long long)ws.walks);
        atomicAdd((unsigned long long *)&stats[1], (unsigned long long)ws.nodes);
        atomicAdd((unsigned long long *)&stats[2], (unsigned long long)ws.box_tests);
        atomicAdd((unsigned long long *)&stats[3], (unsigned long long)ws.tri_tests);
        atomicAdd((unsigned long long *)&stats[4], (unsigned long long)ws.segments);
    }
}

template <int MODE, class LT = LightF>
__global__ __launch_bounds__(kBlock) void sample_kernel(GBufView g, LT L, uint32_t sd, uint32_t sample, float *o_out,
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
            LightF Lc;
            pick_light((uint32_t)px, (uint32_t)py, sample, sd, L, o, y, Lc);
            d[0] = y[0] - o[0];
            d[1] = y[1] - o[1];
            d[2] = y[2] - o[2];
            k = shadow_traced(n, o, d, Lc) ? 0 : 1;
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

// Blocks for tile_of_block: 8 XCDs x whole runs of kTileRun tiles covering
// ceil(ntiles / 8) tiles each, so every tile has a block.
static inline int grid_for(int ntiles) {
    const int per = (ntiles + 7) / 8;
    return 8 * ((per + kTileRun - 1) / kTileRun) * kTileRun;
}

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

hipError_t launch_trace_count(const DeviceBVH &bvh, const GBufView &g, int mode, float R, const LightF &L,
                              uint32_t seed32, uint32_t sample, const OccView &out, uint64_t *stats, hipStream_t st) {
    int tiles_x;
    int nt = ntiles_for(g, tiles_x);
    dim3 grid(grid_for(nt)), block(kBlock);
    if (mode == OCR_AO)
        hipLaunchKernelGGL(trace_count_kernel<OCR_AO>, grid, block, 0, st, bvh, g, R, L, seed32, sample, out, tiles_x,
                           nt, stats);
    else
        hipLaunchKernelGGL(trace_count_kernel<OCR_SHADOW>, grid, block, 0, st, bvh, g, R, L, seed32, sample, out,
                           tiles_x, nt, stats);
    return hipGetLastError();
}

template <class LT>
static hipError_t launch_validate_t(const DeviceBVH &bvh, const GBufView &g, const OccView &occ, int mode, float R,
                                    const LT &L, const ocr_reuse_params &p, uint32_t *bits, uint64_t *stats,
                                    hipStream_t st) {
    const int D = pair_extent(p), words = pair_words(p);
    int tiles_x;
    int nt = ntiles_for(g, tiles_x);
    // the candidate lists live after the bits in the workspace; XCD x holds at most
    // per_xcd = ceil(ntiles / 8) tiles of 256 pixels
    uint32_t *lists = bits + (size_t)g.w * g.h * words;
    const uint32_t per_xcd = (uint32_t)((nt + 7) / 8) * (uint32_t)kBlock;
    hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(kBlock), 0, st, lists);
    const int per_band = (nt + 7) / 8;
    hipLaunchKernelGGL(compact_kernel, dim3(8 * ((per_band + kCompactTiles - 1) / kCompactTiles)), dim3(kBlock), 0, st,
                       g, occ, lists, per_xcd, tiles_x, nt);
    // oversubscribed grid: a multiple of 8 blocks (one share per XCD), 48 per
    // CU (of 4096-16384 blocks, 12288 measured fastest: 1080p shadow
    // validation 0.54 -> 0.50 ms against 8192, AO unchanged)
    dim3 grid(12288), block(kBlock);
    int gw = 0, gh = 0;
    if (p.pattern == OCR_GROUP) group_dims(p.group_n, gw, gh);
    const int lgw = gw == 4 ? 2 : (gw == 2 ? 1 : 0), lgh = gh == 2 ? 1 : 0;
#define OCR_VAL(M, C, G)                                                                                        \
    hipLaunchKernelGGL((validate_window_kernel<M, C, LT, G>), grid, block, 0, st, bvh, g, occ, R * R, L, D, words, \
                       bits, lists, per_xcd, stats, lgw, lgh)
#define OCR_VAL_M(M, G)               \
    do {                              \
        if (stats) OCR_VAL(M, true, G); \
        else OCR_VAL(M, false, G);      \
    } while (0)
    if (p.pattern == OCR_WINDOW) {
        if (mode == OCR_AO) OCR_VAL_M(OCR_AO, false);
        else OCR_VAL_M(OCR_SHADOW, false);
    } else {
        if (mode == OCR_AO) OCR_VAL_M(OCR_AO, true);
        else OCR_VAL_M(OCR_SHADOW, true);
    }
#undef OCR_VAL_M
#undef OCR_VAL
    return hipGetLastError();
}

hipError_t launch_validate(const DeviceBVH &bvh, const GBufView &g, const OccView &occ, int mode, float R,
                           const LightF &L, const ocr_reuse_params &p, uint32_t *bits, uint64_t *stats,
                           hipStream_t st) {
    return launch_validate_t(bvh, g, occ, mode, R, L, p, bits, stats, st);
}

// several lights (shadows only)
hipError_t launch_validate_lights(const DeviceBVH &bvh, const GBufView &g, const OccView &occ, const LightSetF &L,
                                  const ocr_reuse_params &p, uint32_t *bits, uint64_t *stats, hipStream_t st) {
    return launch_validate_t(bvh, g, occ, OCR_SHADOW, 1.0f, L, p, bits, stats, st);
}

// one light sampled from the bilinear emitter density (shadows)
hipError_t launch_trace_bilinear(const DeviceBVH &bvh, const GBufView &g, const LightBilinF &L, uint32_t seed32,
                                 uint32_t sample, const OccView &out, hipStream_t st) {
    int tiles_x;
    int nt = ntiles_for(g, tiles_x);
    dim3 grid(grid_for(nt)), block(kBlock);
    hipLaunchKernelGGL((trace_kernel<OCR_SHADOW, LightBilinF>), grid, block, 0, st, bvh, g, 1.0f, L, seed32, sample,
                       out, tiles_x, nt);
    return hipGetLastError();
}

hipError_t launch_samples_bilinear(const GBufView &g, const LightBilinF &L, uint32_t seed32, uint32_t sample,
                                   float *o, float *d, uint8_t *kind, hipStream_t st) {
    int64_t n = (int64_t)g.w * g.h;
    dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    hipLaunchKernelGGL((sample_kernel<OCR_SHADOW, LightBilinF>), grid, block, 0, st, g, L, seed32, sample, o, d,
                       kind);
    return hipGetLastError();
}

hipError_t launch_trace_lights(const DeviceBVH &bvh, const GBufView &g, const LightSetF &L, uint32_t seed32,
                               uint32_t sample, const OccView &out, hipStream_t st) {
    int tiles_x;
    int nt = ntiles_for(g, tiles_x);
    dim3 grid(grid_for(nt)), block(kBlock);
    hipLaunchKernelGGL((trace_shadow_wave_kernel<LightSetF>), grid, block, 0, st, bvh, g, L, seed32, sample, out,
                       tiles_x, nt);
    return hipGetLastError();
}

}  // namespace ocr
