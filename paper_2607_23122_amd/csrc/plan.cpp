// Batched schedule (plan): many views in one persistent trace launch and one
// persistent reuse launch, recorded once into a HIP graph and replayed.
// Views whose reuse is not the sliding window (fixed groups) are reused by
// the per-view kernel inside the same graph; OCR_UNBIASED views get their
// per-view validation between the two batched launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "api_internal.hpp"
#include "batch.hpp"

using namespace ocr;

struct ocr_plan {
    int device = 0;
    int nviews = 0;
    std::vector<ocr_view_desc> desc;
    std::vector<BatchView> hv;
    std::vector<size_t> ws_bytes;
    void *mem = nullptr;
    size_t mem_bytes = 0;
    BatchView *d_views = nullptr;
    uint32_t *d_tfirst = nullptr, *d_ttx = nullptr, *d_rfirst = nullptr, *d_qstart = nullptr, *d_ctr = nullptr;
    std::vector<uint32_t> h_qstart = std::vector<uint32_t>(18, 0u);
    std::vector<int> unb_views, grp_views;
    int64_t pixels = 0, trace_items = 0, reuse_items = 0;
    size_t reuse_lds = 0;
    int cus = 256, trace_bpc = 1, reuse_bpc = 1;
    ocr_plan_tuning tun{};
    int tuned = 0, candidates = 0, from_cache = 0;
    double tune_ms = 0.0, best_trace_ms = 0.0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kTiles[5][2] = {{8, 8}, {16, 8}, {16, 16}, {32, 8}, {32, 16}};

bool valid_tile(int w, int h) {
    for (auto &t : kTiles)
        if (t[0] == w && t[1] == h) return true;
    return false;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Split [0, total) into 8 contiguous ranges; q[0..8] are the bounds.
void split8(uint64_t total, uint32_t *q) {
    for (int x = 0; x <= 8; ++x) q[x] = (uint32_t)(total * (uint64_t)x / 8u);
}

// Trace tables for tile (tw, th): per-view first item and tiles per row.
void trace_tables(ocr_plan *p, int tw, int th, std::vector<uint32_t> &first, std::vector<uint32_t> &tx) {
    first.assign(p->nviews + 1, 0u);
    tx.assign(p->nviews, 0u);
    uint64_t acc = 0;
    for (int v = 0; v < p->nviews; ++v) {
        const ocr_gbuffer &g = p->desc[v].gbuf;
        first[v] = (uint32_t)acc;
        tx[v] = (uint32_t)((g.width + tw - 1) / tw);
        acc += (uint64_t)tx[v] * (uint64_t)((g.height + th - 1) / th);
    }
    first[p->nviews] = (uint32_t)acc;
    p->trace_items = (int64_t)acc;
    split8(acc, p->h_qstart.data());
}

hipError_t upload_trace_tables(ocr_plan *p, int tw, int th) {
    std::vector<uint32_t> first, tx;
    trace_tables(p, tw, th, first, tx);
    hipError_t e = hipMemcpy(p->d_tfirst, first.data(), first.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_ttx, tx.data(), tx.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_qstart, p->h_qstart.data(), 18 * 4, hipMemcpyHostToDevice);
    return e;
}

int grid_of(int cus, int bpc, int64_t items_per_block_unit) {
    int64_t g = (int64_t)cus * bpc;
    if (items_per_block_unit < g) g = items_per_block_unit;
    g = ((g + 7) / 8) * 8;
    return (int)std::max<int64_t>(g, 8);
}

hipError_t enqueue_trace(ocr_plan *p, hipStream_t st) {
    hipError_t e = launch_batch_reset(p->d_ctr, st);
    if (e != hipSuccess) return e;
    // one wave per item, four waves per block
    int grid = grid_of(p->cus, p->trace_bpc, (p->trace_items + 3) / 4);
    return launch_batch_trace(p->d_views, p->d_tfirst, p->d_ttx, p->nviews, p->d_qstart, p->d_ctr, p->tun.tile_w,
                              p->tun.tile_h, p->tun.packing, grid, st);
}

hipError_t enqueue_all(ocr_plan *p, hipStream_t st) {
    hipError_t e = enqueue_trace(p, st);
    if (e != hipSuccess) return e;
    for (int v : p->unb_views) {
        const BatchView &V = p->hv[v];
        // the light effects validate the shadow pairs
        e = launch_validate(V.bvh, V.g, V.occ, V.mode == OCR_AO ? OCR_AO : OCR_SHADOW, V.R, V.L, p->desc[v].params,
                            const_cast<uint32_t *>(V.bits), nullptr, st);
        if (e != hipSuccess) return e;
    }
    for (int v : p->grp_views) {
        const BatchView &V = p->hv[v];
        e = launch_reuse(V.g, V.occ, V.mode, V.R, V.L, p->desc[v].params, V.bits, V.out, st, V.scale);
        if (e != hipSuccess) return e;
    }
    if (p->reuse_items > 0) {
        int grid = grid_of(p->cus, p->reuse_bpc, p->reuse_items);
        e = launch_batch_reuse(p->d_views, p->d_rfirst, p->nviews, p->d_qstart, p->d_ctr, p->reuse_lds, grid, st);
    }
    return e;
}

void destroy_graph(ocr_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// Time the trace phase for the current knobs: one warm-up, then the median of 3.
hipError_t time_trace(ocr_plan *p, hipStream_t st, double &ms) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    std::vector<float> t;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(a, st);
        if (e == hipSuccess) e = enqueue_trace(p, st);
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float x = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&x, a, b);
        if (rep > 0) t.push_back(x);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e == hipSuccess) {
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
    }
    return e;
}

ocr_status autotune(ocr_plan *p, hipStream_t st) {
    auto t0 = std::chrono::steady_clock::now();
    double best = 1e30;
    ocr_plan_tuning best_t = p->tun;
    int n = 0;
    for (auto &tile : kTiles) {
        for (int pack = OCR_PACK_ROW; pack <= OCR_PACK_MORTON; ++pack) {
            // an 8x8 tile is one pass of 64 lanes: every packing is the same
            if (tile[0] == 8 && tile[1] == 8 && pack != OCR_PACK_ROW) continue;
            p->tun.tile_w = tile[0];
            p->tun.tile_h = tile[1];
            p->tun.packing = pack;
            hipError_t e = upload_trace_tables(p, tile[0], tile[1]);
            double ms = 0.0;
            if (e == hipSuccess) e = time_trace(p, st, ms);
            if (e != hipSuccess) return hip_fail(e, "autotune");
            ++n;
            if (ms < best) {
                best = ms;
                best_t = p->tun;
            }
        }
    }
    p->tun = best_t;
    hipError_t e = upload_trace_tables(p, best_t.tile_w, best_t.tile_h);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    p->tuned = 1;
    p->candidates = n;
    p->best_trace_ms = best;
    p->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return OCR_OK;
}

// Autotuner choices, kept per (device architecture, view-set shape) for the
// life of the process and, when the environment names a file in
// OCR_TUNE_CACHE, across processes (one line per choice: architecture,
// shape hash, tile width and height, packing).  The shape is what the
// trace's speed depends on: every view's size, effect, reuse parameters and
// scene (its triangle and node counts and depth).
std::mutex g_tune_mu;
std::map<std::pair<std::string, uint64_t>, ocr_plan_tuning> g_tune;
bool g_tune_loaded = false;

uint64_t fnv(uint64_t h, int64_t v) {
    for (int b = 0; b < 8; ++b) {
        h ^= (uint64_t)(v >> (8 * b)) & 0xFFu;
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t shape_hash(const ocr_view_desc *views, int n) {
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, n);
    for (int v = 0; v < n; ++v) {
        const ocr_view_desc &d = views[v];
        for (int64_t x : {(int64_t)d.gbuf.width, (int64_t)d.gbuf.height, (int64_t)d.mode,
                          (int64_t)d.params.pattern, (int64_t)d.params.radius, (int64_t)d.params.group_n,
                          (int64_t)d.params.estimator, d.bvh->info.ntris, d.bvh->info.nnodes,
                          (int64_t)d.bvh->info.depth})
            h = fnv(h, x);
    }
    return h;
}

std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.empty() ? "unknown" : a.substr(0, a.find(':'));
}

// (with g_tune_mu held)
void load_tune_file() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("OCR_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char arch[64];
    uint64_t shape = 0;
    int tw = 0, th = 0, pack = 0;
    while (std::fscanf(f, "%63s %" SCNx64 " %d %d %d", arch, &shape, &tw, &th, &pack) == 5)
        if (valid_tile(tw, th) && pack >= OCR_PACK_ROW && pack <= OCR_PACK_MORTON)
            g_tune[{arch, shape}] = ocr_plan_tuning{tw, th, pack, 1};
    std::fclose(f);
}

bool cached_tuning(const std::string &arch, uint64_t shape, ocr_plan_tuning &t) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_tune_file();
    auto it = g_tune.find({arch, shape});
    if (it == g_tune.end()) return false;
    t = it->second;
    return true;
}

void store_tuning(const std::string &arch, uint64_t shape, const ocr_plan_tuning &t) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_tune_file();
    g_tune[{arch, shape}] = t;
    const char *path = std::getenv("OCR_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "%s %" PRIx64 " %d %d %d\n", arch.c_str(), shape, t.tile_w, t.tile_h, t.packing);
        std::fclose(f);
    }
}

void free_plan(ocr_plan *p) {
    destroy_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

}  // namespace

extern "C" {

ocr_status ocr_plan_create(const ocr_view_desc *views, int32_t nviews, const ocr_plan_tuning *tuning, void *stream,
                           ocr_plan **out) {
    if (!out) return fail(OCR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!views || nviews < 1 || nviews > 4096) return fail(OCR_ERR_INVALID_ARG, "need 1..4096 views, got %d", nviews);
    if (tuning) {
        if (!valid_tile(tuning->tile_w, tuning->tile_h))
            return fail(OCR_ERR_INVALID_ARG, "tile %dx%d not one of 8x8, 16x8, 16x16, 32x8, 32x16", tuning->tile_w,
                        tuning->tile_h);
        if (tuning->packing < OCR_PACK_ROW || tuning->packing > OCR_PACK_MORTON)
            return fail(OCR_ERR_INVALID_ARG, "packing %d out of range", tuning->packing);
    }
    std::vector<BatchView> hv(nviews);
    std::vector<size_t> wsb(nviews, 0);
    int64_t pixels = 0;
    for (int v = 0; v < nviews; ++v) {
        const ocr_view_desc &d = views[v];
        if (!d.bvh) return fail(OCR_ERR_INVALID_ARG, "view %d: bvh is NULL", v);
        ocr_status st = check_gbuf(&d.gbuf);
        if (st) return fail(st, "view %d: %s", v, ocr_last_error());
        if ((st = check_params(&d.params))) return fail(st, "view %d: %s", v, ocr_last_error());
        if (d.params.accumulate || d.params.validated)
            return fail(OCR_ERR_INVALID_ARG, "view %d: accumulate and validated must be 0 in a plan", v);
        if (!d.out) return fail(OCR_ERR_INVALID_ARG, "view %d: out is NULL", v);
        BatchView &B = hv[v];
        std::memset(&B, 0, sizeof B);
        if (d.mode < OCR_AO || d.mode > OCR_DIRECT_ILLUMINATION)
            return fail(OCR_ERR_INVALID_ARG, "view %d: mode %d out of range", v, d.mode);
        // the light effects trace shadow records (uniformly sampled lights)
        const int32_t tmode = d.mode == OCR_AO ? OCR_AO : OCR_SHADOW;
        if ((st = check_effect(tmode, d.ao_radius, &d.light, B.L))) return fail(st, "view %d: %s", v, ocr_last_error());
        if (d.mode == OCR_DIRECT_ILLUMINATION && !(std::isfinite(d.radiance) && d.radiance >= 0.0f &&
                                                   std::isfinite(d.albedo) && d.albedo >= 0.0f))
            return fail(OCR_ERR_INVALID_ARG, "view %d: radiance %g and albedo %g must be finite and >= 0", v,
                        (double)d.radiance, (double)d.albedo);
        B.scale = d.mode == OCR_DIRECT_ILLUMINATION
                      ? (float)((double)d.albedo * (double)d.radiance / 3.14159265358979323846)
                      : 1.0f;
        B.bvh = d.bvh->dev;
        B.g = view(&d.gbuf);
        B.R = d.mode == OCR_AO ? d.ao_radius : 1.0f;
        B.R2 = B.R * B.R;
        B.sd = fold_seed(d.seed);
        B.sample = d.sample;
        B.mode = d.mode;
        B.estimator = d.params.estimator;
        B.radius = d.params.radius;
        B.dark_guard = (d.params.estimator == OCR_BIASED && d.params.dark_guard) ? 1 : 0;
        B.words = pair_words(d.params);
        B.r_tiles_x = (d.gbuf.width + kWTX - 1) / kWTX;
        B.out = d.out;
        wsb[v] = ocr_workspace_bytes(d.gbuf.width, d.gbuf.height, &d.params);
        pixels += (int64_t)d.gbuf.width * d.gbuf.height;
    }

    ocr_plan *p = new (std::nothrow) ocr_plan;
    if (!p) return fail(OCR_ERR_OOM, "plan allocation failed");
    p->nviews = nviews;
    p->desc.assign(views, views + nviews);
    p->pixels = pixels;
    p->tun = tuning ? *tuning : ocr_plan_tuning{16, 16, OCR_PACK_BLOCK8, 1};
    if (!tuning) p->tun.use_graph = 1;

    // reuse work: window tiles of window and no-reuse views; fixed groups go per view
    std::vector<uint32_t> rfirst(nviews + 1, 0u);
    uint64_t racc = 0;
    for (int v = 0; v < nviews; ++v) {
        const ocr_view_desc &d = views[v];
        rfirst[v] = (uint32_t)racc;
        const bool grp = d.params.estimator != OCR_NOREUSE && d.params.pattern == OCR_GROUP;
        if (grp) p->grp_views.push_back(v);
        else racc += (uint64_t)((d.gbuf.width + kWTX - 1) / kWTX) * (uint64_t)((d.gbuf.height + kWTY - 1) / kWTY);
        if (d.params.estimator == OCR_UNBIASED) p->unb_views.push_back(v);
        if (!grp && d.params.estimator != OCR_NOREUSE)
            p->reuse_lds = std::max(p->reuse_lds, batch_reuse_lds(d.params.radius, d.mode,
                                                                  d.params.estimator == OCR_UNBIASED, hv[v].words));
    }
    rfirst[nviews] = (uint32_t)racc;
    p->reuse_items = (int64_t)racc;
    split8(racc, p->h_qstart.data() + 9);

    // one device allocation: views, tables, queue counters, records, workspaces
    size_t off = 0;
    const size_t o_views = off;
    off += align256(sizeof(BatchView) * nviews);
    const size_t o_tfirst = off;
    off += align256(4 * (nviews + 1));
    const size_t o_ttx = off;
    off += align256(4 * nviews);
    const size_t o_rfirst = off;
    off += align256(4 * (nviews + 1));
    const size_t o_q = off;
    off += align256(4 * 18);
    const size_t o_ctr = off;
    off += align256(4 * kQueueWords);
    std::vector<size_t> o_rec(nviews), o_ws(nviews);
    for (int v = 0; v < nviews; ++v) {
        const size_t px = (size_t)views[v].gbuf.width * views[v].gbuf.height;
        o_rec[v] = off;
        off += align256(12 * px) + align256(12 * px) + align256(4 * px);
        o_ws[v] = off;
        off += align256(wsb[v]);
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->mem, off);
    if (e != hipSuccess) {
        free_plan(p);
        return e == hipErrorOutOfMemory ? fail(OCR_ERR_OOM, "plan needs %zu device bytes", off)
                                        : hip_fail(e, "plan allocation");
    }
    p->mem_bytes = off;
    char *base = (char *)p->mem;
    p->d_views = (BatchView *)(base + o_views);
    p->d_tfirst = (uint32_t *)(base + o_tfirst);
    p->d_ttx = (uint32_t *)(base + o_ttx);
    p->d_rfirst = (uint32_t *)(base + o_rfirst);
    p->d_qstart = (uint32_t *)(base + o_q);
    p->d_ctr = (uint32_t *)(base + o_ctr);
    for (int v = 0; v < nviews; ++v) {
        const size_t px = (size_t)views[v].gbuf.width * views[v].gbuf.height;
        char *r = base + o_rec[v];
        hv[v].occ.dz = (float *)r;
        hv[v].occ.nz = (float *)(r + align256(12 * px));
        hv[v].occ.hit = (uint32_t *)(r + 2 * align256(12 * px));
        hv[v].bits = wsb[v] ? (const uint32_t *)(base + o_ws[v]) : nullptr;
    }
    p->hv = hv;
    p->ws_bytes = wsb;

    int dev_cus = 0;
    if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && dev_cus > 0)
        p->cus = dev_cus;
    p->trace_bpc = batch_trace_blocks_per_cu();
    if (p->reuse_items > 0) {
        p->reuse_bpc = batch_reuse_blocks_per_cu(std::max<size_t>(p->reuse_lds, 16));
        if (p->reuse_bpc < 1) {
            free_plan(p);
            return fail(OCR_ERR_UNSUPPORTED, "reuse needs %zu bytes of LDS per block", p->reuse_lds);
        }
    }

    hipStream_t st = (hipStream_t)stream;
    e = hipMemcpy(p->d_views, hv.data(), sizeof(BatchView) * nviews, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_rfirst, rfirst.data(), 4 * (nviews + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = upload_trace_tables(p, p->tun.tile_w, p->tun.tile_h);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "plan upload");
    }
    if (!tuning) {
        // a view set of this shape tuned before on this architecture takes
        // its choice; otherwise time every setting and keep the fastest
        const std::string arch = device_arch(p->device);
        const uint64_t shape = shape_hash(views, nviews);
        ocr_plan_tuning t;
        if (cached_tuning(arch, shape, t)) {
            p->tun = t;
            p->tuned = 1;
            p->from_cache = 1;
            e = upload_trace_tables(p, t.tile_w, t.tile_h);
            if (e != hipSuccess) {
                free_plan(p);
                return hip_fail(e, "plan upload");
            }
        } else {
            ocr_status s2 = autotune(p, st);
            if (s2) {
                free_plan(p);
                return s2;
            }
            store_tuning(arch, shape, p->tun);
        }
    }
    if (p->tun.use_graph) {
        e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
        if (e != hipSuccess) {
            free_plan(p);
            return hip_fail(e, "plan stream");
        }
    }
    *out = p;
    return OCR_OK;
}

ocr_status ocr_plan_launch(ocr_plan *p, void *stream) {
    if (!p) return fail(OCR_ERR_INVALID_ARG, "plan is NULL");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (!p->tun.use_graph) {
        e = enqueue_all(p, st);
        return e == hipSuccess ? OCR_OK : hip_fail(e, "plan launch");
    }
    if (!p->exec) {
        e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        hipError_t e2 = enqueue_all(p, p->cap);
        e = hipStreamEndCapture(p->cap, &p->graph);
        if (e2 != hipSuccess || e != hipSuccess) {
            destroy_graph(p);
            return hip_fail(e2 != hipSuccess ? e2 : e, "graph capture");
        }
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            destroy_graph(p);
            return hip_fail(e, "graph instantiate");
        }
    }
    e = hipGraphLaunch(p->exec, st);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "graph launch");
}

ocr_status ocr_plan_get_info(const ocr_plan *p, ocr_plan_info *info) {
    if (!p || !info) return fail(OCR_ERR_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->nviews = p->nviews;
    info->pixels = p->pixels;
    info->trace_items = p->trace_items;
    info->reuse_items = p->reuse_items;
    info->device_bytes = (int64_t)p->mem_bytes;
    info->tuning = p->tun;
    info->tuned = p->tuned;
    info->candidates = p->candidates;
    info->tune_ms = p->tune_ms;
    info->best_trace_ms = p->best_trace_ms;
    info->from_cache = p->from_cache;
    return OCR_OK;
}

ocr_status ocr_plan_get_records(const ocr_plan *p, int32_t v, ocr_occluders *out) {
    if (!p || !out) return fail(OCR_ERR_INVALID_ARG, "NULL argument");
    if (v < 0 || v >= p->nviews) return fail(OCR_ERR_INVALID_ARG, "view %d out of range", v);
    out->dz = p->hv[v].occ.dz;
    out->nz = p->hv[v].occ.nz;
    out->hit = p->hv[v].occ.hit;
    return OCR_OK;
}

ocr_status ocr_plan_free(ocr_plan *p) {
    if (!p) return OCR_OK;
    // the plan's memory is freed either way; a failed wait is reported
    const hipError_t e = hipDeviceSynchronize();
    free_plan(p);
    return e == hipSuccess ? OCR_OK : hip_fail(e, "device synchronize before freeing the plan");
}

}  // extern "C"
