// Sliding-window occluder-domain MIS reuse of one target tile (Sec. 4.2-4.4;
// steps 2-3 of App. D / App. H), shared by the per-frame reuse kernel and the
// batched schedule.
//
// For a target i with reuse set S(i):
//   B_i = sum_{j in S(i), hit_j} [p_i(j) > 0 and P_i(j) > 0] p_i(j) / P_i(j),
//   P_i(j) = sum_{k in S(i)} p_k(j),
// p = the pair density (validated by the first-hit bits when unbiased).
//
// P_i(j) depends on both i and j, but only through the pair densities p_k(j)
// with k - j in [-2R, 2R]^2, each needed by every target whose window holds
// both.  So each candidate j's (4R+1)^2 densities are evaluated once, every
// P_i(j) for the (2R+1)^2 targets around j is formed as box sums (row sums,
// then column sums), and p_i(j)/P_i(j) is scattered to the targets.  A block
// owns a 16x16 target tile and stages the receivers of the tile plus an
// R-pixel halo in LDS; the scattered terms are summed in LDS as 32.32
// fixed-point integers, which makes the sum independent of the order in which
// waves arrive (bitwise reproducible) at ~2^-33 absolute error per term.
// For R = 1..3 a lane takes one receiver row of one candidate (its densities
// in registers, its row sums to LDS) and then one (candidate, target) pair;
// other radii take one wave per candidate.  Both sum in the same order, so
// they give the same bits.
#pragma once
#include "density.hpp"
#include "lights.hpp"
#include "ocr_common.hpp"
#include "solid_angle.hpp"

namespace ocr {

constexpr int kRBlock = 256;
// A candidate with at most this many positive densities in its rectangle takes
// the sparse path of the scatter.
constexpr int kSparse = 8;

__device__ inline void ld3(const float *p, int64_t i, float v[3]) {
    v[0] = p[3 * i];
    v[1] = p[3 * i + 1];
    v[2] = p[3 * i + 2];
}

__device__ inline float finish(int mode, bool valid, float B, float F, bool dark, float prev, int accumulate) {
    float v;
    if (mode == OCR_AO) v = valid ? 1.0f - B : 1.0f;
    else v = valid ? (dark ? 0.0f : F - B) : 0.0f;
    return accumulate ? prev + v : v;
}

// The no-reuse estimate of pixel gi (S(i) = {i}).  AO: 1 - [hit]; area
// shadows of a uniformly sampled light: [unblocked].  The solid-angle and
// direct-illumination quantities, and any light sampled from the bilinear
// density, take the N = 1 case of their MIS estimators: the unshadowed term
// minus C(x_i, z_i) for a hit whose own density is positive (the ratio p/p
// is 1).
template <int MODE, class LT>
__device__ inline float noreuse_value(const GBufView &g, const OccView &occ, const LT &L, int64_t gi, float scale) {
    // (both ids read together; a background pixel's hit id is never used)
    const uint32_t prim = g.prim[gi], hit0 = occ.hit[gi];
    const bool valid = prim != OCR_HIT_MISS;
    if constexpr (MODE == OCR_AO) {
        return (!valid || hit0 == OCR_HIT_MISS) ? 1.0f : 0.0f;
    } else if constexpr (MODE == OCR_SHADOW && !kBilinear<LT>) {
        return (valid && hit0 == OCR_HIT_MISS) ? 1.0f : 0.0f;
    } else {
        if (!valid) return 0.0f;
        float x[3], n[3], o[3];
        ld3(g.pos, gi, x);
        ld3(g.nrm, gi, n);
        offset_point(x, n, o);
        float Bg = 0.0f;
        const uint32_t hit = hit0;
        if (hit < OCR_HIT_SELF) {
            float dz[3], nz[3];
            ld3(occ.dz, gi, dz);
            ld3(occ.nz, gi, nz);
            const auto rk = recv_of(o, L);
            if (dens_light(dz, n, rk, nz, L) > 0.0f) {
                Bg = 1.0f;
                if constexpr (MODE == kDI) Bg = di_pair_g(dz, n, rk.hk, L);
                else if constexpr (MODE == kShadowSA) Bg = sa_pair_g(dz, rk.hk, L);
                if constexpr (kBilinear<LT>) Bg *= inv_bilinear_q(dz, rk, L);
            }
        }
        if constexpr (MODE == kDI) return di_estimate(o, n, L, Bg, scale);
        else if constexpr (MODE == kShadowSA) return sa_estimate(o, n, L, Bg);
        else return front_light(o, n, L) - Bg;
    }
}

// Radii the row-task body handles (compiled per radius); others take the
// per-candidate body.
__host__ __device__ constexpr bool row_body_radius(int R) { return R >= 1 && R <= 3; }

// LDS layout of the window kernel for radius R (dynamic shared memory).
struct WinLayout {
    int RWX, RWY, cells, side, dens, hsum, words;
    size_t o_off, n_off, sh_off, valid_off, miss_off, list_off, B_off, wave_off, total;
};

__host__ __device__ constexpr size_t lds_take(size_t &off, size_t bytes) {
    size_t at = off;
    off += (bytes + 15) & ~(size_t)15;
    return at;
}

// nrecv: floats of a receiver's light terms (kRecvFloats of the light type).
__host__ __device__ constexpr WinLayout win_layout(int R, int mode, bool unb, int words, int nrecv = 3) {
    WinLayout l{};
    l.RWX = kWTX + 2 * R;
    l.RWY = kWTY + 2 * R;
    l.cells = l.RWX * l.RWY;
    l.side = 4 * R + 1;
    l.dens = l.side * l.side;
    l.hsum = l.side * (2 * R + 1) > 2 * kSparse ? l.side * (2 * R + 1) : 2 * kSparse;
    l.words = words;
    size_t off = 0;
    l.B_off = lds_take(off, sizeof(unsigned long long) * kWTX * kWTY);
    l.o_off = lds_take(off, sizeof(float) * 3 * l.cells);
    l.n_off = lds_take(off, sizeof(float) * 3 * l.cells);
    l.sh_off = lds_take(off, mode != OCR_AO ? sizeof(float) * nrecv * l.cells : 0);
    l.valid_off = lds_take(off, l.cells);
    l.miss_off = lds_take(off, l.cells);
    l.list_off = lds_take(off, 4 * sizeof(int) + sizeof(uint16_t) * l.cells);
    // per-wave scratch: the per-candidate body's densities and box sums (the
    // row-task body keeps its sums in registers)
    const int per_wave = row_body_radius(R) ? 0 : l.dens + l.hsum;
    l.wave_off = lds_take(off, sizeof(float) * (kRBlock / 64) * per_wave);
    l.total = off;
    return l;
}

// The scattered term of target cell kc: p_i(j) / P_i(j) times the factor
// C(x_i, z_j) of the estimator, g_ij under the solid-angle definition
// (kShadowSA), gd_ij for direct illumination (kDI), and divided by q_i(y'_ij)
// for a light sampled from the bilinear density; clamped below 2^31 so that
// the 32.32 fixed-point sum cannot overflow (the factor reaches that size only
// within ~1e-5 of the light).
template <int MODE, class LT>
__device__ inline float weighted_term(float ratio, const float *s_o, const float *s_n, const float *s_sh, int CELLS,
                                      int kc, const float oj[3], const float dzj[3], const LT &L) {
    const float oi[3] = {s_o[kc], s_o[CELLS + kc], s_o[2 * CELLS + kc]};
    float w[3];
    rel_vec(oj, oi, dzj, w);
    float gf = 1.0f;
    if constexpr (MODE == kDI) {
        const float ni[3] = {s_n[kc], s_n[CELLS + kc], s_n[2 * CELLS + kc]};
        gf = di_pair_g(w, ni, s_sh[kc], L);
    } else if constexpr (MODE == kShadowSA) {
        gf = sa_pair_g(w, s_sh[kc], L);
    }
    if constexpr (kBilinear<LT>) {
        float v[6];
        for (int a = 0; a < 6; ++a) v[a] = s_sh[a * CELLS + kc];
        gf *= inv_bilinear_q(w, recv_load(v, L), L);
    }
    return fminf(ratio * gf, 0x1p31f);
}

// The targets of tile cells [R, R + kWTX) x [R, R + kWTY) (staged
// coordinates) that candidate cell (cx, cy) reaches, [tx0, tx0 + ntx) x
// [ty0, ty0 + nty), and the receivers they need, [tx0 - R, tx0 + ntx + R) x
// [ty0 - R, ty0 + nty + R).
struct CandRect {
    int tx0, ty0, ntx, nty;
};
__device__ inline CandRect cand_rect(int cx, int cy, int R) {
    CandRect q;
    q.tx0 = max(cx - R, R);
    q.ty0 = max(cy - R, R);
    q.ntx = min(cx + R, R + kWTX - 1) - q.tx0 + 1;
    q.nty = min(cy + R, R + kWTY - 1) - q.ty0 + 1;
    return q;
}

// DPP control of the whole-wave shift that gives each lane the value of the
// previous lane (wave_shr:1).
constexpr int kDppPrevLane = 0x138;

// v of lane - 1 (whole-wave DPP shift; lane 0, which has no source lane, gets
// 0 through bound_ctrl).  With full row and bank masks and bound_ctrl set, the
// compiler folds the move into the instruction that uses it.
__device__ inline float from_prev_lane(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), kDppPrevLane, 0xF, 0xF, true));
}

// Candidates of a staged tile with the row-task body (window radius R = 1..3,
// a template parameter so that a receiver row's 4R + 1 densities stay in
// registers).  The waves of the block claim batches of consecutive entries of
// the tile's candidate list in turn from one shared cursor (a compare-and-swap
// in LDS), a batch being the leading candidates whose receiver rows fit in 64
// lanes, the rows of a candidate on consecutive lanes; so only the tile's last
// batch is partly empty, not one per wave.  A lane takes one receiver row of one
// candidate j: the densities p_k(j) of the row's receivers, then the row's
// box sums over each window of 2R + 1 of them, H[t] = sum_e p(t + e) in e
// order, all in registers.  For each target column t, the window sums over
// rows, P_i(j) = sum of H over the 2R + 1 rows of target row r's window in
// row order, are folded through the lanes by cross-lane moves (no memory) and
// end on the lane of the window's last row, r + 2R, which takes p_i(j) from
// lane r + R and scatters p_i(j) / P_i(j) as the per-candidate body does.
// The sums run in the same order as that body's, so the estimates are the
// same bits.
template <int MODE, bool UNB, class LT, int R>
__device__ inline void tile_row_candidates(const WinLayout &lay, unsigned char *smem, const GBufView &g,
                                           const OccView &occ, float R2, const LT &L,
                                           const uint32_t *__restrict__ bits, int words, int tx, int ty) {
    constexpr int TW = 2 * R + 1, SIDE = 4 * R + 1, D = 2 * R;
    constexpr int TX = kWTX, TY = kWTY, RW = kWTX + 2 * R, CELLS = RW * (kWTY + 2 * R);
    // The staged normals and light terms follow the positions directly
    // (3 * CELLS floats each, a multiple of 16 bytes), so all the receiver
    // values a density reads sit at constant offsets from one LDS address.
    constexpr WinLayout kLay = win_layout(R, MODE, UNB, 1, kRecvFloats<LT>);
    static_assert(kLay.cells == CELLS && kLay.n_off == kLay.o_off + 3 * CELLS * sizeof(float) &&
                      (MODE == OCR_AO || kLay.sh_off == kLay.n_off + 3 * CELLS * sizeof(float)),
                  "receiver arrays are contiguous");
    const float inv_rw = 1.0f / (float)RW;
    unsigned long long *s_B = reinterpret_cast<unsigned long long *>(smem + lay.B_off);
    const float *s_o = reinterpret_cast<const float *>(smem + lay.o_off);
    const float *s_n = s_o + 3 * CELLS;
    const float *s_sh = s_n + 3 * CELLS;
    int *s_count = reinterpret_cast<int *>(smem + lay.list_off);
    const uint16_t *s_list = reinterpret_cast<const uint16_t *>(smem + lay.list_off + 4 * sizeof(int));
    const int lane = threadIdx.x & 63;
    const int x0 = tx * TX - R, y0 = ty * TY - R;
    // s_count[0]: candidates listed; s_count[1]: the shared cursor (entries
    // claimed), zero at the tile's start
    const int end = s_count[0];
    for (;;) {
        const int cur = __builtin_amdgcn_readfirstlane(__atomic_load_n(&s_count[1], __ATOMIC_RELAXED));
        if (cur >= end) break;
        // candidate lanes: lane k holds candidate cur + k and its receiver
        // rows; the batch is the leading candidates whose rows fit
        const int ci = cur + lane;
        int c = 0, hd = 0;
        if (ci < end) {
            c = s_list[ci];
            const int cy = small_div(c, inv_rw), cx = c - __mul24(cy, RW);
            hd = cand_rect(cx, cy, R).nty + 2 * R;
        }
        const int rows_inc = wave_incl_scan(hd);
        const int nb = __popcll(wave_ballot(ci < end && rows_inc <= 64));
        const int rows_total = __builtin_amdgcn_readlane(rows_inc, nb - 1);
        const int rows_exc = rows_inc - hd;
        // claim the batch; if another wave moved the cursor first, form the
        // next batch from where it now stands (some wave succeeds each round)
        int won = 0;
        if (lane == 0) won = atomicCAS(&s_count[1], cur, cur + nb) == cur;
        if (!__builtin_amdgcn_readfirstlane(won)) continue;

        // this lane's candidate and receiver row
        int k = 0;
        for (int m = 0; m < nb; ++m) k += lane >= __builtin_amdgcn_readlane(rows_inc, m) ? 1 : 0;
        k = min(k, nb - 1);
        const int cl = __shfl(c, k), rs = __shfl(rows_exc, k);
        const int cy = small_div(cl, inv_rw), cx = cl - __mul24(cy, RW);
        const CandRect q = cand_rect(cx, cy, R);
        const int row = lane - rs;
        const bool has_row = lane < rows_total;
        const int64_t gj = (int64_t)(y0 + cy) * g.w + (x0 + cx);
        const float oj[3] = {s_o[cl], s_o[CELLS + cl], s_o[2 * CELLS + cl]};
        float dzj[3] = {0.f, 0.f, 0.f};
        float p[SIDE];
#pragma unroll
        for (int e = 0; e < SIDE; ++e) p[e] = 0.0f;
        if (has_row) {
            const int WD = q.ntx + 2 * R;
            const int kx0 = q.tx0 - R, ky = q.ty0 - R + row;
            float nzj[3];
            ld3(occ.dz, gj, dzj);
            ld3(occ.nz, gj, nzj);
            // unbiased: the row's validation bits, bit e for receiver kx0 + e
            uint32_t rowbits = 0xFFFFFFFFu;
            if (UNB) {
                const int qb = __mul24(ky - cy + D, SIDE) + (kx0 - cx + D);
                const int w0 = qb >> 5;
                const uint32_t lo = bits[gj * words + w0];
                const uint32_t hi = w0 + 1 < words ? bits[gj * words + w0 + 1] : 0u;
                rowbits = (uint32_t)((((unsigned long long)hi << 32) | lo) >> (qb & 31));
            }
            const int kcb = __mul24(ky, RW) + kx0;
#pragma unroll
            for (int e = 0; e < SIDE; ++e) {
                if (e < WD && ((rowbits >> e) & 1u)) {
                    const int kc = kcb + e;
                    const float ok[3] = {s_o[kc], s_o[CELLS + kc], s_o[2 * CELLS + kc]};
                    const float nk[3] = {s_n[kc], s_n[CELLS + kc], s_n[2 * CELLS + kc]};
                    float w[3];
                    rel_vec(oj, ok, dzj, w);
                    if constexpr (MODE == OCR_AO) {
                        p[e] = dens_ao(w, nk, nzj, R2);
                    } else {
                        float v[kRecvFloats<LT>];
                        for (int a = 0; a < kRecvFloats<LT>; ++a) v[a] = s_sh[a * CELLS + kc];
                        p[e] = dens_light(w, nk, recv_load(v, L), nzj, L);
                    }
                }
            }
        }
        // P_i(j) for target row tr = row - 2R, column t: the box sums of rows
        // tr .. row (lanes lane - 2R .. lane, all of this candidate when
        // row >= 2R), summed in row order.  The fold runs upwards through the
        // lanes, G_e(lane) = G_(e-1)(lane - 1) + H(lane), so that after 2R
        // steps the lane of row `row` holds the window that ends at it, and
        // each step is one add with a shifted operand; p_i(j) comes from row
        // tr + R.  Every lane takes part in the moves; the lanes of rows
        // 2R .. 2R + nty - 1 scatter for the candidate's nty target rows.
        const int tr = row - D;
        const bool target_row = has_row && tr >= 0;
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            // (the sums start from their first term rather than from 0: the
            // same values, since no density is -0)
            float h = p[t];
#pragma unroll
            for (int e = 1; e < TW; ++e) h += p[t + e];
            float P = h;
#pragma unroll
            for (int e = 1; e < TW; ++e) P = from_prev_lane(P) + h;
            float pij = p[t + R];
#pragma unroll
            for (int e = 0; e < R; ++e) pij = from_prev_lane(pij);
            if (target_row && t < q.ntx && pij > 0.0f && P > 0.0f) {
                float term = pij * __builtin_amdgcn_rcpf(P);
                if constexpr (MODE >= kShadowSA || kBilinear<LT>) {
                    term = weighted_term<MODE>(term, s_o, s_n, s_sh, CELLS,
                                               __mul24(q.ty0 + tr, RW) + (q.tx0 + t), oj, dzj, L);
                }
                atomicAdd(&s_B[(q.ty0 + tr - R) * TX + (q.tx0 + t - R)],
                          (unsigned long long)rintf(term * 4294967296.0f));
            }
        }
    }
    (void)TY;
}

// One kWTX x kWTY target tile (tx, ty) of the sliding-window estimator; every
// thread of the block calls it.  `smem` holds win_layout(R, ...).total bytes.
template <int MODE, bool UNB, class LT = LightF>
__device__ inline void reuse_window_tile(unsigned char *smem, const GBufView &g, const OccView &occ, float R2,
                                         const LT &L, const uint32_t *__restrict__ bits, int words, int R,
                                         int dark_guard, int accumulate, float *out, int tx, int ty,
                                         float scale = 1.0f) {
    const WinLayout lay = win_layout(R, MODE, UNB, words, kRecvFloats<LT>);
    const int TX = kWTX, TY = kWTY, RW = lay.RWX, CELLS = lay.cells, D = 2 * R, SIDE = lay.side, TW = 2 * R + 1;
    const float inv_rw = 1.0f / (float)RW;
    unsigned long long *s_B = reinterpret_cast<unsigned long long *>(smem + lay.B_off);
    float *s_o = reinterpret_cast<float *>(smem + lay.o_off);    // [3][cells]
    float *s_n = reinterpret_cast<float *>(smem + lay.n_off);    // [3][cells]
    float *s_sh = reinterpret_cast<float *>(smem + lay.sh_off);  // [kRecvFloats][cells]
    uint8_t *s_valid = smem + lay.valid_off;
    uint8_t *s_miss = smem + lay.miss_off;
    int *s_count = reinterpret_cast<int *>(smem + lay.list_off);
    uint16_t *s_list = reinterpret_cast<uint16_t *>(smem + lay.list_off + 4 * sizeof(int));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *w_dens = reinterpret_cast<float *>(smem + lay.wave_off) + wave * (lay.dens + lay.hsum);
    float *w_h = w_dens + lay.dens;

    const int x0 = tx * TX - R, y0 = ty * TY - R;
    const int tid = threadIdx.x;
    if (tid == 0) s_count[0] = s_count[1] = 0;
    for (int t = tid; t < TX * TY; t += kRBlock) s_B[t] = 0ull;
    __syncthreads();

    // Stage receivers (o, n, shadow terms), validity, misses, validation
    // bits, and compact the cells whose ray found an occluder.
    for (int c = tid; c < CELLS; c += kRBlock) {
        const int cyy = small_div(c, inv_rw);
        int gx = x0 + (c - __mul24(cyy, RW)), gy = y0 + cyy;
        bool inside = gx >= 0 && gx < g.w && gy >= 0 && gy < g.h;
        int64_t gi = inside ? (int64_t)gy * g.w + gx : 0;
        bool valid = inside && g.prim[gi] != OCR_HIT_MISS;
        float o[3] = {0.f, 0.f, 0.f}, n[3] = {0.f, 0.f, 0.f};
        uint32_t hit = OCR_HIT_MISS;
        if (valid) {
            float x[3];
            ld3(g.pos, gi, x);
            ld3(g.nrm, gi, n);
            offset_point(x, n, o);
            hit = occ.hit[gi];
        }
        for (int a = 0; a < 3; ++a) {
            s_o[a * CELLS + c] = o[a];
            s_n[a * CELLS + c] = n[a];
        }
        if (MODE != OCR_AO) {
            // the receiver's light terms (its point, for several lights)
            float v[kRecvFloats<LT>] = {};
            if (valid) recv_store(recv_of(o, L), v);
            for (int a = 0; a < kRecvFloats<LT>; ++a) s_sh[a * CELLS + c] = v[a];
        }
        s_valid[c] = valid;
        s_miss[c] = valid && hit == OCR_HIT_MISS;
        if (valid && hit < OCR_HIT_SELF) s_list[atomicAdd(s_count, 1)] = (uint16_t)c;
    }
    __syncthreads();

    if (R == 1) {
        tile_row_candidates<MODE, UNB, LT, 1>(lay, smem, g, occ, R2, L, bits, words, tx, ty);
    } else if (R == 2) {
        tile_row_candidates<MODE, UNB, LT, 2>(lay, smem, g, occ, R2, L, bits, words, tx, ty);
    } else if (R == 3) {
        tile_row_candidates<MODE, UNB, LT, 3>(lay, smem, g, occ, R2, L, bits, words, tx, ty);
    } else {
        // Other radii: one wave per candidate j.
        const int ncand = *s_count;
        for (int li = wave; li < ncand; li += kRBlock / 64) {
            const int c = __builtin_amdgcn_readfirstlane((int)s_list[li]);
            const int cy = small_div(c, inv_rw), cx = c - __mul24(cy, RW);
            const int64_t gj = (int64_t)(y0 + cy) * g.w + (x0 + cx);
            float oj[3] = {s_o[c], s_o[CELLS + c], s_o[2 * CELLS + c]};
            float dzj[3], nzj[3];
            ld3(occ.dz, gj, dzj);
            ld3(occ.nz, gj, nzj);
            // The targets of this tile that j reaches are the cells [tx0, tx1] x
            // [ty0, ty1] (staged coordinates; the tile is [R, R + TX) x [R, R + TY));
            // they need the receivers [tx0 - R, tx1 + R] x [ty0 - R, ty1 + R], a
            // WD x HD rectangle inside the staged region (13 x 13 at R = 3 for a
            // candidate whose targets are all in the tile, less in the halo).
            const int tx0 = max(cx - R, R), tx1 = min(cx + R, R + TX - 1);
            const int ty0 = max(cy - R, R), ty1 = min(cy + R, R + TY - 1);
            const int ntx = tx1 - tx0 + 1, nty = ty1 - ty0 + 1;
            const int WD = ntx + 2 * R, HD = nty + 2 * R;
            const int kx0 = tx0 - R, ky0 = ty0 - R;
            // (hardware reciprocals: small_div stays exact with a 1-ulp inverse
            // for the quotients below, all < 2^12)
            const float inv_wd = __builtin_amdgcn_rcpf((float)WD), inv_ntx = __builtin_amdgcn_rcpf((float)ntx);
            const int nq = WD * HD;
            // (1) densities p_k(j) over the rectangle, row stride SIDE; every lane
            // runs every pass so that the count of positive densities is uniform.
            // Shadow candidates have a few positive densities at most (the light
            // subtends a narrow cone); AO candidates most often have dozens.
            constexpr bool kSparsePath = MODE != OCR_AO;
            int npos = 0;
            int *e_code = reinterpret_cast<int *>(w_h);  // positive entries, q order
            float *e_p = w_h + kSparse;
            for (int q0 = 0; q0 < nq; q0 += 64) {
                const int q = q0 + lane;
                float p = 0.0f;
                int qy = 0, qx = 0;
                if (q < nq) {
                    // (index products by 24-bit multiplies: full rate, all operands < 2^23)
                    qy = small_div(q, inv_wd);
                    qx = q - __mul24(qy, WD);
                    const int kx = kx0 + qx, ky = ky0 + qy;
                    const int kc = __mul24(ky, RW) + kx;
                    // unbiased: candidate j's validation bit for the receiver at
                    // offset k - j first.  It is set only where the validation
                    // found the same density positive (and the segment free), so
                    // a pair without it contributes 0 whatever its density, and a
                    // round with no bit set skips the densities altogether
                    // (shadow candidates have a few positive pairs, clustered).
                    bool need = true;
                    if (UNB) {
                        const int qb = __mul24(ky - cy + D, SIDE) + (kx - cx + D);
                        const uint32_t wv = bits[gj * words + (qb >> 5)];
                        need = (wv >> (qb & 31)) & 1u;
                    }
                    if (need) {
                        float ok[3] = {s_o[kc], s_o[CELLS + kc], s_o[2 * CELLS + kc]};
                        float nk[3] = {s_n[kc], s_n[CELLS + kc], s_n[2 * CELLS + kc]};
                        float w[3];
                        rel_vec(oj, ok, dzj, w);
                        if (MODE == OCR_AO) {
                            p = dens_ao(w, nk, nzj, R2);
                        } else {
                            float v[kRecvFloats<LT>];
                            for (int a = 0; a < kRecvFloats<LT>; ++a) v[a] = s_sh[a * CELLS + kc];
                            p = dens_light(w, nk, recv_load(v, L), nzj, L);
                        }
                    }
                    w_dens[__mul24(qy, SIDE) + qx] = p;
                }
                if (!kSparsePath) continue;
                const unsigned long long pm = __ballot(p > 0.0f);
                if (npos < kSparse) {
                    // keep the first kSparse positive entries for the sparse path
                    const int at = npos + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(pm >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)pm, 0u));
                    if (p > 0.0f && at < kSparse) {
                        e_code[at] = (qy << 8) | qx;
                        e_p[at] = p;
                    }
                }
                npos += (int)__popcll(pm);
            }
            wave_sync();
            if (kSparsePath && npos <= kSparse) {
                // (2') Few positive densities (most shadow candidates): P_i(j) from
                // the positive entries alone.  Lane e takes entry e; the sums run
                // over the rows in order and within a row over the columns in
                // order, the grouping of the box sums below, which only add zeros
                // besides (exact), so both paths give the same bits.
                int my_code = 0;
                float my_p = 0.0f;
                if (lane < npos) {
                    my_code = e_code[lane];
                    my_p = e_p[lane];
                }
                const int my_y = my_code >> 8, my_x = my_code & 255;
                const bool tgt = lane < npos && my_x >= R && my_x < R + ntx && my_y >= R && my_y < R + nty;
                if (__ballot(tgt) != 0ull) {
                    float P = 0.0f, h = 0.0f;
                    int row = -1;
                    for (int m = 0; m < npos; ++m) {
                        const int cm = __builtin_amdgcn_readlane(my_code, m);
                        const float pv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_p), m));
                        const int ym = cm >> 8, xm = cm & 255;
                        if (ym != row) {
                            P += h;
                            h = 0.0f;
                            row = ym;
                        }
                        if (abs(ym - my_y) <= R && abs(xm - my_x) <= R) h += pv;
                    }
                    P += h;
                    if (tgt) {
                        float term = my_p * __builtin_amdgcn_rcpf(P);
                        if constexpr (MODE >= kShadowSA || kBilinear<LT>)
                            term = weighted_term<MODE>(term, s_o, s_n, s_sh, CELLS, __mul24(ky0 + my_y, RW) + (kx0 + my_x),
                                                       oj, dzj, L);
                        atomicAdd(&s_B[(ky0 + my_y - R) * TX + (kx0 + my_x - R)],
                                  (unsigned long long)rintf(term * 4294967296.0f));
                    }
                }
            } else {
                // (2) row box sums H[row][t] = sum_{e < 2R+1} p(row, t + e), t < ntx
                for (int q = lane; q < HD * ntx; q += 64) {
                    const int row = small_div(q, inv_ntx), t2 = q - __mul24(row, ntx);
                    const float *pr = w_dens + __mul24(row, SIDE) + t2;
                    float h = 0.0f;
                    // unrolled so the LDS reads issue together; the additions keep their order
    #pragma unroll 4
                    for (int e = 0; e < TW; ++e) h += pr[e];
                    w_h[__mul24(row, TW) + t2] = h;
                }
                wave_sync();
                // (3) target i = (tx0 + t2, ty0 + r2): P_i(j) is the column box sum of H
                for (int q = lane; q < nty * ntx; q += 64) {
                    const int r2 = small_div(q, inv_ntx), t2 = q - __mul24(r2, ntx);
                    const float *ph = w_h + __mul24(r2, TW) + t2;
                    float P = 0.0f;
    #pragma unroll 4
                    for (int e = 0; e < TW; ++e) P += ph[__mul24(e, TW)];
                    const float pij = w_dens[__mul24(r2 + R, SIDE) + (t2 + R)];
                    if (pij > 0.0f && P > 0.0f) {
                        float term = pij * __builtin_amdgcn_rcpf(P);
                        if constexpr (MODE >= kShadowSA || kBilinear<LT>)
                            term = weighted_term<MODE>(term, s_o, s_n, s_sh, CELLS, __mul24(ty0 + r2, RW) + (tx0 + t2), oj,
                                                       dzj, L);
                        atomicAdd(&s_B[(ty0 + r2 - R) * TX + (tx0 + t2 - R)],
                                  (unsigned long long)rintf(term * 4294967296.0f));
                    }
                }
            }
            wave_sync();
        }
    }
    __syncthreads();

    // one lane per target
    for (int t = tid; t < TX * TY; t += kRBlock) {
        const int ix = t % TX, iy = t / TX;
        const int px = tx * TX + ix, py = ty * TY + iy;
        if (px >= g.w || py >= g.h) continue;
        const int c = __mul24(iy + R, RW) + (ix + R);
        const bool valid = s_valid[c];
        float B = (float)((double)s_B[t] * 0x1p-32);
        float F = 1.0f;
        bool dark = false;
        if (MODE != OCR_AO && valid) {
            float o[3] = {s_o[c], s_o[CELLS + c], s_o[2 * CELLS + c]};
            float n[3] = {s_n[c], s_n[CELLS + c], s_n[2 * CELLS + c]};
            if constexpr (MODE == kShadowSA) {
                // F_Omega - (Area / Omega_A) B, as F - B below
                F = sa_estimate(o, n, L, B);
                B = 0.0f;
            } else if constexpr (MODE == kDI) {
                // (rho L_e / pi) (E - Area B), as F - B below
                F = di_estimate(o, n, L, B, scale);
                B = 0.0f;
            } else {
                F = front_light(o, n, L);
            }
            if (dark_guard) {
                int misses = 0;
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) misses += s_miss[c + dy * RW + dx];
                dark = misses == 0;
            }
        }
        const int64_t gi = (int64_t)py * g.w + px;
        out[gi] = finish(MODE, valid, B, F, dark, accumulate ? out[gi] : 0.0f, accumulate);
    }
}


}  // namespace ocr
