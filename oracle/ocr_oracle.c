/*
 * CPU oracle for occlusion-point reuse -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this file's library.  It shares no code, header, table or helper with
 * the GPU library, and it imports nothing from it.
 *
 * What it computes, and where the paper defines it:
 *   - the no-reuse AO and shadow estimators (Sec. 3.2 Eq. ao-mc-estimator,
 *     Sec. 3.3 Eq. shadow-mc-estimator);
 *   - first-hit occluder records (Sec. 4.2 Eq. occ-first-hit; App. D and
 *     App. H, step 1 of both algorithms);
 *   - the induced occluder densities p_AO (Sec. 4.3 Eq. ao-pdf with the
 *     Jacobian of Eq. ao-jacobian) and p_Sh (Sec. 4.4 Eq. shadow-pdf with the
 *     Jacobian of Eq. shadow-jacobian evaluated at the light re-intersection
 *     y'(x,z));
 *   - the balance-heuristic MIS combination (Sec. 4.2 Eqs. generic-mis-weight
 *     and generic-mis-estimator-simplified) in its unbiased form (Eqs.
 *     ao-unbiased-estimator, shadow-estimator; App. D and App. H, steps 2-3)
 *     and its biased form (Eqs. ao-biased-estimator, shadow-biased-estimator)
 *     with the dark-region guard of Sec. 4.4;
 *   - accumulation over samples (final line of both algorithms);
 *   - FP64 quadrature references of Eqs. ao-hemisphere and shadow-area;
 *   - the paper's simple reuse baselines of Sec. 6: final-value filtering
 *     (Filter (N) for AO; for shadows light-sample reuse without validation,
 *     Light (N), which the paper notes reduces to the same average) and
 *     light-sample reuse with visibility re-evaluation (Light (NU));
 *   - shadows of several rectangular lights (the paper shows two lights
 *     but gives no formulation; reading: the visible fraction of the total
 *     emitting area, a light chosen per sample with probability A_l / A_tot
 *     and the induced density summed over the lights);
 *   - occluder-domain direct illumination (App. on it: Eq.
 *     reapp-di-occluder-domain-compact with the MIS estimator of Eq.
 *     reapp-di-general-mis-estimator and factor of Eq.
 *     reapp-di-general-mis-factor) for a Lambertian receiver under a
 *     uniform one-sided emitter, its unshadowed term from Lambert's polygon
 *     formula, and its quadrature reference;
 *   - shadows under the solid-angle definition (App. on that definition:
 *     Eq. reapp-shadow-definition-solid-angle, the MIS estimator of Eq.
 *     reapp-shadow-solid-angle-estimator with the factor C_Omega of Eq.
 *     reapp-shadow-solid-angle-mis-factor), with the emitter's solid angle
 *     computed exactly, and its quadrature reference.
 *
 * Readings where the paper is silent:
 * receiver point o = x + 2^-16 (1 + max|x|) n and the receiver's own
 * triangle ignored by its rays; candidates and receivers of a target are the
 * valid pixels of its reuse set (a clipped (2r+1)^2 window, or a fixed
 * image-aligned group of N pixels); MIS denominators sum over the target's
 * own set; the shadow target is F_i - B_i where F_i is the exact fraction of
 * the light in front of the receiver's tangent plane, with the front-side
 * support added to p_Sh; the one-sided light faces normalize(e_u x e_v).
 *
 * FP32 vs FP64: a GPU in FP32 cannot reproduce FP64 decisions that sit on a
 * threshold.  Every such decision is classified here: a trace is "grazing"
 * when any triangle lies within 2^-19 L of the ray inside the relevant t
 * range's tolerance, and a pair density is "ambiguous" when one of its
 * support tests sits within a narrow band of its threshold.  Ambiguous
 * densities are enumerated (both outcomes) so that the comparison accepts
 * either.  Grazing traces are only flagged: a comparison that finds a
 * different hit on a flagged ray leaves out the targets whose reuse set
 * holds it.
 */
#include "ocr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define GRAZE_REL 0x1p-19     /* edge / end-point band for traces, relative to L */
/* Bands around FP32-decided thresholds, each a generous multiple of the
 * FP32 rounding error of the quantity the GPU compares (a few ulps):      */
#define RADIUS_BAND 0x1p-17   /* |x - z| against R, relative to R           */
#define FRONT_BAND 0x1p-17    /* cosine of x->z with n_x against 0          */
#define LIGHT_BAND 0x1p-14    /* y' against the rectangle's edges (units of the
                                 edge length) and s against 1; y' carries the
                                 rounding of o - c, up to ~1e-6 of the edge  */
#define COS_BAND 0x1p-18      /* a clamped cosine reaching zero             */
#define VALID_ETA 1e-4        /* validation segments stop at t = 1 - eta */
#define MAX_AMBIG 3

/* ------------------------------------------------------------------------ */
/* Small FP64 vector helpers                                                */
/* ------------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *r) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double len3(const double *a) { return sqrt(dot3(a, a)); }
static void f2d(const float *a, double *r) { r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; }

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: pcg4d (Jarzynski and Olano, JCGT 2020).    */
/* ------------------------------------------------------------------------ */
static void pcg4d(uint32_t v[4]) {
    for (int i = 0; i < 4; ++i) v[i] = v[i] * 1664525u + 1013904223u;
    v[0] += v[1] * v[3];
    v[1] += v[2] * v[0];
    v[2] += v[0] * v[1];
    v[3] += v[1] * v[2];
    for (int i = 0; i < 4; ++i) v[i] ^= v[i] >> 16;
    v[0] += v[1] * v[3];
    v[1] += v[2] * v[0];
    v[2] += v[0] * v[1];
    v[3] += v[1] * v[2];
}

uint32_t orc_pcg4d_first(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t *out4) {
    uint32_t v[4] = {a, b, c, d};
    pcg4d(v);
    memcpy(out4, v, sizeof v);
    return v[0];
}

static uint32_t seed32(uint64_t s) { return (uint32_t)s ^ (uint32_t)(s >> 32); }
static float unit24(uint32_t h) { return (float)(h >> 8) * 0x1p-24f; }

/* ------------------------------------------------------------------------ */
/* FP32 sample specification (both sides reproduce it bit for bit).         */
/* Compiled with -ffp-contract=off: every + and * below rounds on its own;  */
/* fmaf is used only where written.                                         */
/* ------------------------------------------------------------------------ */

/* Receiver point o = x + eps n with eps = 2^-16 (1 + max_c |x_c|). */
static void offset_point(const float x[3], const float n[3], float o[3]) {
    float m = fmaxf(fabsf(x[0]), fmaxf(fabsf(x[1]), fabsf(x[2])));
    float eps = (1.0f + m) * 0x1p-16f;
    for (int c = 0; c < 3; ++c) o[c] = fmaf(eps, n[c], x[c]);
}

/* Cosine-weighted hemisphere direction (Eq. ao-direction-pdf) by Malley's
 * method: a uniform point (alpha, beta) of the unit disc by rejection, lifted
 * to gamma = sqrt(1 - alpha^2 - beta^2) along n, in the orthonormal basis of
 * Duff et al. (JCGT 2017). */
static void ao_direction(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const float n[3], float w[3]) {
    float al = 0.0f, be = 0.0f, q = 0.0f;
    for (uint32_t a = 0; a < 16u; ++a) {
        uint32_t h[4] = {px, py, s, sd + a * 0x9E3779B9u};
        pcg4d(h);
        float ta = 2.0f * unit24(h[0]) - 1.0f;
        float tb = 2.0f * unit24(h[1]) - 1.0f;
        float tq = fmaf(tb, tb, ta * ta);
        if (tq < 1.0f) {
            al = ta;
            be = tb;
            q = tq;
            break;
        }
    }
    float g = sqrtf(1.0f - q);
    float sign = copysignf(1.0f, n[2]);
    float a = -1.0f / (sign + n[2]);
    float b = n[0] * n[1] * a;
    float t[3] = {1.0f + sign * n[0] * n[0] * a, sign * b, -sign * n[0]};
    float bb[3] = {b, sign + n[1] * n[1] * a, -n[1]};
    for (int c = 0; c < 3; ++c) w[c] = (al * t[c] + be * bb[c]) + g * n[c];
}

/* Uniform point on the rectangle (Eq. shadow-light-pdf): y = c + (u0-1/2) e_u + (u1-1/2) e_v. */
static void light_point(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const float *L, float y[3]) {
    uint32_t h[4] = {px, py, s, sd};
    pcg4d(h);
    float a = unit24(h[0]) - 0.5f;
    float b = unit24(h[1]) - 0.5f;
    for (int c = 0; c < 3; ++c) y[c] = fmaf(b, L[6 + c], fmaf(a, L[3 + c], L[c]));
}

/* Light k of the parameters (k < max(nlights, 1)). */
static const float *light_k(const orc_params *p, int k) { return k == 0 ? p->light : p->more_lights + 9 * (k - 1); }
static int num_lights(const orc_params *p) { return p->nlights > 1 ? p->nlights : 1; }

/* FP32 area |e_u x e_v| of a light, as the sample specification computes it. */
static float light_area32(const float *L) {
    float nl0 = L[4] * L[8] - L[5] * L[7], nl1 = L[5] * L[6] - L[3] * L[8], nl2 = L[3] * L[7] - L[4] * L[6];
    return sqrtf(fmaf(nl2, nl2, fmaf(nl1, nl1, nl0 * nl0)));
}

/* Several lights: the light of a sample is chosen with probability
 * A_l / A_tot, so that the point is uniform over the union of the lights:
 * with u2 = unit24(h[2]) of the same hash, the first l whose running FP32 sum
 * C_l = A_0 + ... + A_l exceeds u2 * A_tot (the last light if rounding leaves
 * none); the point on it then uses h[0], h[1] exactly as for one light.  For
 * one light this is light_point. */
static int light_point_multi(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const orc_params *p, float y[3]) {
    int K = num_lights(p);
    uint32_t h[4] = {px, py, s, sd};
    pcg4d(h);
    int l = 0;
    if (K > 1) {
        float A[4], tot = 0.0f;
        for (int k = 0; k < K; ++k) {
            A[k] = light_area32(light_k(p, k));
            tot = tot + A[k];
        }
        float u = unit24(h[2]) * tot, C = 0.0f;
        l = K - 1;
        for (int k = 0; k < K; ++k) {
            C = C + A[k];
            if (u < C) {
                l = k;
                break;
            }
        }
    }
    const float *L = light_k(p, l);
    float a = unit24(h[0]) - 0.5f;
    float b = unit24(h[1]) - 0.5f;
    for (int c = 0; c < 3; ++c) y[c] = fmaf(b, L[6 + c], fmaf(a, L[3 + c], L[c]));
    return l;
}

/* General emitter-area density p_A(y | x) (App., general area-domain
 * sampling density): besides the uniform density 1 / Area, the bilinear
 * density of a receiver point o.  Its corner weights are the shape of the
 * solid-angle density cos(theta_y) / |o - y|^2 at the four corners, i.e.
 * 1 / |o - y_k|^3 (cos(theta_y) = h / |o - y| with the same height h for every
 * point of the rectangle), and over the rectangle it interpolates them
 * bilinearly in the light coordinates (a, b).  It depends on the receiver, so
 * reuse evaluates it at every receiver of a candidate.
 *
 * FP32 sample specification.  Corners k = 0..3 at (a_k, b_k) = (-1/2,-1/2),
 * (1/2,-1/2), (-1/2,1/2), (1/2,1/2); |o - y_k|^2 clamped below at 2^-40; the
 * weights divided by their maximum. */
static void bilinear_weights32(const float *L, const float o[3], float w[4]) {
    float m = 0.0f;
    for (int k = 0; k < 4; ++k) {
        float ak = (k & 1) ? 0.5f : -0.5f, bk = (k & 2) ? 0.5f : -0.5f, d[3];
        for (int c = 0; c < 3; ++c) d[c] = o[c] - fmaf(bk, L[6 + c], fmaf(ak, L[3 + c], L[c]));
        float d2 = fmaxf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])), 0x1p-40f);
        w[k] = 1.0f / (d2 * sqrtf(d2));
        m = fmaxf(m, w[k]);
    }
    for (int k = 0; k < 4; ++k) w[k] = w[k] / m;
}

/* Inverse of the CDF of the density proportional to (1 - t) e0 + t e1 on
 * [0, 1] (e0, e1 >= 0): the root in [0, 1] of (e1 - e0) t^2 + 2 e0 t =
 * xi (e0 + e1), in the form without cancellation,
 * t = xi (e0 + e1) / (e0 + sqrt((1 - xi) e0^2 + xi e1^2)). */
static float sample_linear32(float xi, float e0, float e1) {
    float r = sqrtf((1.0f - xi) * (e0 * e0) + xi * (e1 * e1));
    float den = e0 + r;
    if (!(den > 0.0f)) return 0.0f;
    float t = xi * (e0 + e1) / den;
    return fminf(t, 1.0f);
}

/* A point from the bilinear density of o: v (= b + 1/2) from its marginal,
 * linear between the corner sums w_0 + w_1 (v = 0) and w_2 + w_3 (v = 1), with
 * h[1]; then u (= a + 1/2) from the conditional at that v, linear between the
 * edge weights interpolated at v, with h[0]; the point as for uniform
 * sampling. */
static void light_point_bilinear(uint32_t px, uint32_t py, uint32_t s, uint32_t sd, const float *L,
                                 const float o[3], float y[3]) {
    uint32_t h[4] = {px, py, s, sd};
    pcg4d(h);
    float w[4];
    bilinear_weights32(L, o, w);
    float tv = sample_linear32(unit24(h[1]), w[0] + w[1], w[2] + w[3]);
    float f0 = (1.0f - tv) * w[0] + tv * w[2];
    float f1 = (1.0f - tv) * w[1] + tv * w[3];
    float tu = sample_linear32(unit24(h[0]), f0, f1);
    float a = tu - 0.5f, b = tv - 0.5f;
    for (int c = 0; c < 3; ++c) y[c] = fmaf(b, L[6 + c], fmaf(a, L[3 + c], L[c]));
}

/* kind: 0 traced, 1 no trace (below the tangent plane, or receiver on the
 * back side of the one-sided light), 2 background pixel. */
static int make_sample(int32_t W, const float *pos, const float *nrm, const uint32_t *prim, const orc_params *p,
                       int32_t px, int32_t py, float o[3], float dir[3]) {
    int64_t i = (int64_t)py * W + px;
    if (prim[i] == ORC_MISS) return 2;
    const float *x = pos + 3 * i, *n = nrm + 3 * i;
    offset_point(x, n, o);
    uint32_t sd = seed32(p->seed);
    if (p->mode == 0) {
        ao_direction((uint32_t)px, (uint32_t)py, p->sample, sd, n, dir);
        return 0;
    }
    float y[3];
    const float *L = p->light;
    if (p->light_pdf == 1) light_point_bilinear((uint32_t)px, (uint32_t)py, p->sample, sd, L, o, y);
    else L = light_k(p, light_point_multi((uint32_t)px, (uint32_t)py, p->sample, sd, p, y));
    for (int c = 0; c < 3; ++c) dir[c] = y[c] - o[c];
    float front = fmaf(n[2], dir[2], fmaf(n[1], dir[1], n[0] * dir[0]));
    float nl[3] = {L[4] * L[8] - L[5] * L[7], L[5] * L[6] - L[3] * L[8], L[3] * L[7] - L[4] * L[6]};
    float lit = fmaf(nl[2], o[2] - L[2], fmaf(nl[1], o[1] - L[1], nl[0] * (o[0] - L[0])));
    if (!(front > 0.0f) || !(lit > 0.0f)) return 1;
    return 0;
}

void orc_samples(int32_t W, int32_t H, const float *pos, const float *nrm, const uint32_t *prim,
                 const orc_params *p, int32_t x0, int32_t y0, int32_t x1, int32_t y1, float *o, float *dir,
                 uint8_t *kind) {
    (void)H;
    for (int32_t py = y0; py < y1; ++py)
        for (int32_t px = x0; px < x1; ++px) {
            int64_t i = (int64_t)py * W + px;
            float oo[3] = {0, 0, 0}, dd[3] = {0, 0, 0};
            kind[i] = (uint8_t)make_sample(W, pos, nrm, prim, p, px, py, oo, dd);
            memcpy(o + 3 * i, oo, sizeof oo);
            memcpy(dir + 3 * i, dd, sizeof dd);
        }
}

/* ------------------------------------------------------------------------ */
/* Scene, FP64 triangle probe, brute force and uniform-grid candidate sets. */
/* ------------------------------------------------------------------------ */
struct orc_scene {
    int64_t nt;
    double *v;       /* nt * 9 */
    uint8_t *degen;  /* zero-area triangles are never hit */
    int32_t use_grid;
    double lo[3], hi[3], cell[3];
    int32_t n[3];
    int64_t *cstart;
    uint32_t *crefs;
};

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

orc_scene *orc_scene_create(const float *V, int64_t nv, const uint32_t *F, int64_t nt, int32_t use_grid) {
    orc_scene *s = (orc_scene *)calloc(1, sizeof *s);
    s->nt = nt;
    s->v = (double *)malloc(sizeof(double) * 9 * (size_t)(nt > 0 ? nt : 1));
    s->degen = (uint8_t *)calloc((size_t)(nt > 0 ? nt : 1), 1);
    for (int64_t t = 0; t < nt; ++t) {
        for (int k = 0; k < 3; ++k) {
            uint32_t vi = F[3 * t + k];
            if ((int64_t)vi >= nv) vi = 0;
            for (int c = 0; c < 3; ++c) s->v[9 * t + 3 * k + c] = V[3 * (int64_t)vi + c];
        }
        double e1[3], e2[3], nn[3];
        sub3(s->v + 9 * t + 3, s->v + 9 * t, e1);
        sub3(s->v + 9 * t + 6, s->v + 9 * t, e2);
        cross3(e1, e2, nn);
        s->degen[t] = dot3(nn, nn) == 0.0;
    }
    s->use_grid = use_grid;
    if (!use_grid || nt == 0) return s;
    double vol = 1.0, ext[3];
    for (int c = 0; c < 3; ++c) { s->lo[c] = 1e300; s->hi[c] = -1e300; }
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) {
                double x = s->v[9 * t + 3 * k + c];
                if (x < s->lo[c]) s->lo[c] = x;
                if (x > s->hi[c]) s->hi[c] = x;
            }
    for (int c = 0; c < 3; ++c) {
        double pad = 1e-3 * (1.0 + fabs(s->lo[c]) + fabs(s->hi[c]));
        s->lo[c] -= pad;
        s->hi[c] += pad;
        ext[c] = s->hi[c] - s->lo[c];
        vol *= ext[c];
    }
    double h = cbrt(vol / (2.0 * (double)nt));
    for (int c = 0; c < 3; ++c) {
        s->n[c] = clampi((int)ceil(ext[c] / h), 1, 1024);
        s->cell[c] = ext[c] / s->n[c];
    }
    int64_t nc = (int64_t)s->n[0] * s->n[1] * s->n[2];
    s->cstart = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    /* Each triangle is binned by its bounding box grown by a margin, so a
     * ray passing within the grazing band of it visits one of its cells. */
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t t = 0; t < nt; ++t) {
            int c0[3], c1[3];
            for (int c = 0; c < 3; ++c) {
                double lo = 1e300, hi = -1e300;
                for (int k = 0; k < 3; ++k) {
                    double x = s->v[9 * t + 3 * k + c];
                    if (x < lo) lo = x;
                    if (x > hi) hi = x;
                }
                double m = 1e-4 * s->cell[c];
                c0[c] = clampi((int)floor((lo - m - s->lo[c]) / s->cell[c]), 0, s->n[c] - 1);
                c1[c] = clampi((int)floor((hi + m - s->lo[c]) / s->cell[c]), 0, s->n[c] - 1);
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) {
                        int64_t ci = ((int64_t)z * s->n[1] + y) * s->n[0] + x;
                        if (pass == 0) s->cstart[ci + 1]++;
                        else s->crefs[s->cstart[ci]++] = (uint32_t)t;
                    }
        }
        if (pass == 0) {
            for (int64_t c = 0; c < nc; ++c) s->cstart[c + 1] += s->cstart[c];
            s->crefs = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(s->cstart[nc] + 1));
        } else {
            for (int64_t c = nc; c > 0; --c) s->cstart[c] = s->cstart[c - 1];
            s->cstart[0] = 0;
        }
    }
    return s;
}

void orc_scene_free(orc_scene *s) {
    if (!s) return;
    free(s->v);
    free(s->degen);
    free(s->cstart);
    free(s->crefs);
    free(s);
}

int64_t orc_scene_grid_cells(const orc_scene *s) {
    return s->use_grid ? (int64_t)s->n[0] * s->n[1] * s->n[2] : 0;
}

/* Growable list of candidate triangle ids for one query. */
typedef struct {
    uint32_t *ids;
    int64_t n, cap;
} idlist;

static void idl_push(idlist *l, uint32_t id) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 256;
        l->ids = (uint32_t *)realloc(l->ids, sizeof(uint32_t) * (size_t)l->cap);
    }
    l->ids[l->n++] = id;
}

/* Candidate set for the segment o + t d, t in [0, tmax]: every triangle whose
 * (grown) box shares a grid cell with the segment, or all triangles. */
static void candidates(const orc_scene *s, const double o[3], const double d[3], double tmax, idlist *out) {
    out->n = 0;
    if (!s->use_grid) {
        for (int64_t t = 0; t < s->nt; ++t) idl_push(out, (uint32_t)t);
        return;
    }
    double t0 = 0.0, t1 = tmax * (1.0 + 1e-9) + 1e-12;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) {
            if (o[c] < s->lo[c] || o[c] > s->hi[c]) return;
            continue;
        }
        double ta = (s->lo[c] - o[c]) / d[c], tb = (s->hi[c] - o[c]) / d[c];
        if (ta > tb) { double q = ta; ta = tb; tb = q; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (t0 > t1) return;
    int cc[3], step[3];
    double tnext[3], tdel[3];
    for (int c = 0; c < 3; ++c) {
        double x = o[c] + t0 * d[c];
        cc[c] = clampi((int)floor((x - s->lo[c]) / s->cell[c]), 0, s->n[c] - 1);
        if (d[c] > 0) {
            step[c] = 1;
            tnext[c] = (s->lo[c] + (cc[c] + 1) * s->cell[c] - o[c]) / d[c];
            tdel[c] = s->cell[c] / d[c];
        } else if (d[c] < 0) {
            step[c] = -1;
            tnext[c] = (s->lo[c] + cc[c] * s->cell[c] - o[c]) / d[c];
            tdel[c] = -s->cell[c] / d[c];
        } else {
            step[c] = 0;
            tnext[c] = 1e300;
            tdel[c] = 1e300;
        }
    }
    for (;;) {
        int64_t ci = ((int64_t)cc[2] * s->n[1] + cc[1]) * s->n[0] + cc[0];
        for (int64_t r = s->cstart[ci]; r < s->cstart[ci + 1]; ++r) idl_push(out, s->crefs[r]);
        int ax = tnext[0] < tnext[1] ? (tnext[0] < tnext[2] ? 0 : 2) : (tnext[1] < tnext[2] ? 1 : 2);
        if (tnext[ax] > t1) break;
        cc[ax] += step[ax];
        if (cc[ax] < 0 || cc[ax] >= s->n[ax]) break;
        tnext[ax] += tdel[ax];
    }
}

/* Plane parameter t of the ray at the triangle's plane and the signed
 * distance (inside > 0) of that point from the triangle's boundary, plus the
 * query's length scale L = max_v |v - o|. */
typedef struct {
    int ok;
    double t, dist, L;
} probe_t;

static probe_t probe(const orc_scene *s, uint32_t id, const double o[3], const double d[3]) {
    probe_t r = {0, 0.0, 0.0, 0.0};
    if (s->degen[id]) return r;
    const double *a = s->v + 9 * (int64_t)id, *b = a + 3, *c = a + 6;
    double e1[3], e2[3], n[3], ao[3], bo[3], co[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, n);
    double nn = len3(n);
    sub3(a, o, ao);
    sub3(b, o, bo);
    sub3(c, o, co);
    r.L = fmax(len3(ao), fmax(len3(bo), len3(co)));
    double den = dot3(n, d);
    if (den == 0.0) return r;
    r.t = dot3(n, ao) / den;
    double p[3] = {o[0] + r.t * d[0], o[1] + r.t * d[1], o[2] + r.t * d[2]};
    const double *vs[3] = {a, b, c};
    double best = 1e300;
    for (int k = 0; k < 3; ++k) {
        const double *va = vs[k], *vb = vs[(k + 1) % 3];
        double e[3], pa[3], x[3];
        sub3(vb, va, e);
        sub3(p, va, pa);
        cross3(e, pa, x);
        double dk = dot3(x, n) / (len3(e) * nn);
        if (dk < best) best = dk;
    }
    r.dist = best;
    r.ok = 1;
    return r;
}

static void closest_one(const orc_scene *s, idlist *cand, const double o[3], const double d[3], double tmax,
                        int inclusive, uint32_t ign0, uint32_t ign1, uint32_t *tri, double *tout,
                        uint8_t *graze) {
    candidates(s, o, d, tmax, cand);
    double dl = len3(d);
    double bt = 0.0;
    uint32_t bid = ORC_MISS;
    for (int64_t q = 0; q < cand->n; ++q) {
        uint32_t id = cand->ids[q];
        if (id == ign0 || id == ign1) continue;
        probe_t pr = probe(s, id, o, d);
        if (!pr.ok || pr.dist < 0.0 || !(pr.t > 0.0)) continue;
        if (inclusive ? !(pr.t <= tmax) : !(pr.t < tmax)) continue;
        if (bid == ORC_MISS || pr.t < bt || (pr.t == bt && id < bid)) {
            bt = pr.t;
            bid = id;
        }
    }
    double tlim = bid == ORC_MISS ? tmax : bt;
    uint8_t g = 0;
    for (int64_t q = 0; q < cand->n && !g; ++q) {
        uint32_t id = cand->ids[q];
        if (id == ign0 || id == ign1) continue;
        probe_t pr = probe(s, id, o, d);
        if (!pr.ok) continue;
        double tp = GRAZE_REL * pr.L, tt = tp / dl;
        if (pr.t < -tt || pr.t > tlim + tt) continue;
        if (fabs(pr.dist) <= tp) { g = 1; break; }
        if (pr.dist < 0.0) continue;
        if (fabs(pr.t) <= tt || fabs(pr.t - tmax) <= tt) g = 1;
        if (bid != ORC_MISS && id != bid && fabs(pr.t - bt) <= tt) g = 1;
    }
    *tri = bid;
    *tout = bid == ORC_MISS ? 0.0 : bt;
    *graze = g;
}

static void any_one(const orc_scene *s, idlist *cand, const double o[3], const double d[3], double tmax,
                    uint32_t ign0, uint32_t ign1, uint8_t *blocked, uint8_t *graze) {
    candidates(s, o, d, tmax, cand);
    double dl = len3(d);
    int definite = 0, hit64 = 0, g = 0;
    for (int64_t q = 0; q < cand->n; ++q) {
        uint32_t id = cand->ids[q];
        if (id == ign0 || id == ign1) continue;
        probe_t pr = probe(s, id, o, d);
        if (!pr.ok) continue;
        double tp = GRAZE_REL * pr.L, tt = tp / dl;
        if (pr.t < -tt || pr.t > tmax + tt) continue;
        int near = fabs(pr.dist) <= tp;
        if (pr.dist >= 0.0 && pr.t > 0.0 && pr.t < tmax) hit64 = 1;
        if (!near && pr.dist > 0.0 && pr.t > tt && pr.t < tmax - tt) {
            definite = 1;
            break;
        }
        if (near || (pr.dist > 0.0 && (fabs(pr.t) <= tt || fabs(pr.t - tmax) <= tt))) g = 1;
    }
    *blocked = (uint8_t)(definite || hit64);
    *graze = (uint8_t)(!definite && g);
}

void orc_closest(const orc_scene *s, int64_t n, const double *o, const double *d, const double *tmax,
                 int32_t inclusive, const uint32_t *ign0, const uint32_t *ign1, uint32_t *tri, double *t,
                 uint8_t *graze) {
#pragma omp parallel
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i)
            closest_one(s, &cand, o + 3 * i, d + 3 * i, tmax[i], inclusive, ign0[i], ign1[i], tri + i, t + i,
                        graze + i);
        free(cand.ids);
    }
}

void orc_any(const orc_scene *s, int64_t n, const double *o, const double *d, const double *tmax,
             const uint32_t *ign0, const uint32_t *ign1, uint8_t *blocked, uint8_t *graze) {
#pragma omp parallel
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i)
            any_one(s, &cand, o + 3 * i, d + 3 * i, tmax[i], ign0[i], ign1[i], blocked + i, graze + i);
        free(cand.ids);
    }
}

/* ------------------------------------------------------------------------ */
/* First-hit records (step 1 of App. D and App. H).                        */
/* ------------------------------------------------------------------------ */
static void tri_normal(const orc_scene *s, uint32_t id, double n[3]) {
    const double *a = s->v + 9 * (int64_t)id;
    double e1[3], e2[3];
    sub3(a + 3, a, e1);
    sub3(a + 6, a, e2);
    cross3(e1, e2, n);
    double l = len3(n);
    n[0] /= l; n[1] /= l; n[2] /= l;
}

static void record_one(const orc_scene *s, idlist *cand, int32_t W, const float *pos, const float *nrm,
                       const uint32_t *prim, const orc_params *p, int32_t px, int32_t py, uint32_t *hit,
                       double *z, double *nz, uint8_t *graze) {
    int64_t i = (int64_t)py * W + px;
    float of[3], df[3];
    int kind = make_sample(W, pos, nrm, prim, p, px, py, of, df);
    graze[i] = 0;
    for (int c = 0; c < 3; ++c) { z[3 * i + c] = 0.0; nz[3 * i + c] = 0.0; }
    if (kind == 2) { hit[i] = ORC_MISS; return; }
    if (kind == 1) { hit[i] = ORC_SELF; return; }
    double o[3], d[3], t;
    f2d(of, o);
    f2d(df, d);
    uint32_t tri;
    /* AO: ray (o, omega), t in (0, R] (t_max = R, App. D).  Shadow: segment
     * o -> y, t in (0, 1) (t_max = |y - x|, App. H). */
    if (p->mode == 0) closest_one(s, cand, o, d, p->ao_radius, 1, prim[i], ORC_MISS, &tri, &t, graze + i);
    else closest_one(s, cand, o, d, 1.0, 0, prim[i], ORC_MISS, &tri, &t, graze + i);
    hit[i] = tri;
    if (tri == ORC_MISS) return;
    double n[3];
    tri_normal(s, tri, n);
    /* oriented hit normal: facing the ray's origin */
    if (dot3(n, d) > 0.0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    for (int c = 0; c < 3; ++c) {
        z[3 * i + c] = o[c] + t * d[c];
        nz[3 * i + c] = n[c];
    }
}

void orc_records(const orc_scene *s, int32_t W, int32_t H, const float *pos, const float *nrm,
                 const uint32_t *prim, const orc_params *p, int32_t x0, int32_t y0, int32_t x1, int32_t y1,
                 uint32_t *hit, double *z, double *nz, uint8_t *graze) {
    (void)H;
    int64_t w = x1 - x0, n = w * (int64_t)(y1 - y0);
#pragma omp parallel
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < n; ++q)
            record_one(s, &cand, W, pos, nrm, prim, p, x0 + (int32_t)(q % w), y0 + (int32_t)(q / w), hit, z, nz,
                       graze);
        free(cand.ids);
    }
}

/* ------------------------------------------------------------------------ */
/* Induced densities without the first-hit factor.                          */
/* Each density carries its FP64 value p, the value "ppass" it takes when   */
/* every support test sitting in its threshold band passes, whether such a  */
/* test exists (amb: the density is either ppass or 0), and whether the     */
/* value is not comparable at all (excl).                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double p, ppass;
    int amb, excl;
} dens_t;

/* Eq. (ao-pdf) with Occ dropped:
 *   (1/pi) <n_x, w_{x->z}> J_{Omega->S}(x,z) 1{|x - z| <= R},
 *   J_{Omega->S} = <n_z, w_{z->x}> / |x - z|^2           (Eq. ao-jacobian). */
static dens_t density_ao(const double o[3], const double n[3], const double z[3], const double nz[3], double R) {
    dens_t r = {0.0, 0.0, 0, 0};
    double w[3];
    sub3(z, o, w);
    double d2 = dot3(w, w);
    if (d2 == 0.0) return r;
    double d = sqrt(d2);
    double cos_x = dot3(n, w) / d;   /* <n_x, w_{x->z}> */
    double cos_z = -dot3(nz, w) / d; /* <n_z, w_{z->x}> */
    int fail = 0, amb = 0;
    if (fabs(d - R) <= RADIUS_BAND * R) amb = 1;
    else if (!(d <= R)) fail = 1;
    if (fabs(cos_x) <= COS_BAND) amb = 1;
    else if (!(cos_x > 0.0)) fail = 1;
    if (fabs(cos_z) <= COS_BAND) amb = 1;
    else if (!(cos_z > 0.0)) fail = 1;
    if (fail) return r;
    double J = fabs(cos_z) / d2;
    double g = (1.0 / PI) * fabs(cos_x) * J;
    r.ppass = g;
    r.amb = amb;
    r.p = (d <= R && cos_x > 0.0 && cos_z > 0.0) ? (1.0 / PI) * cos_x * (cos_z / d2) : 0.0;
    return r;
}

static void light_frame(const double *L, double c[3], double eu[3], double ev[3], double nl[3], double *area) {
    for (int k = 0; k < 3; ++k) { c[k] = L[k]; eu[k] = L[3 + k]; ev[k] = L[6 + k]; }
    cross3(eu, ev, nl);
    *area = len3(nl);
    nl[0] /= *area; nl[1] /= *area; nl[2] /= *area;
}

/* Eq. (shadow-pdf) with Occ dropped: (1/Area) J(x,z) chi_A(x,z), with the
 * Jacobian of Eq. (shadow-jacobian),
 *   J = <n_z, w_{z->x}> |x - y'|^2 / (<n_y, w_{y'->x}> |x - z|^2),
 * evaluated at y'(x,z), the point where the ray from x through z meets the
 * emitter; chi_A requires that point to lie beyond z on the emitting side
 * of the rectangle.  The front-side support <n_x, w_{x->z}> > 0 is added
 * because samples behind the tangent plane are accounted for exactly by F_i. */
static dens_t density_shadow(const double o[3], const double n[3], const double z[3], const double nz[3],
                             const double *L) {
    dens_t r = {0.0, 0.0, 0, 0};
    double c[3], eu[3], ev[3], nl[3], area;
    light_frame(L, c, eu, ev, nl, &area);
    double w[3];
    sub3(z, o, w);
    double d2 = dot3(w, w);
    if (d2 == 0.0) return r;
    double d = sqrt(d2);
    int fail = 0, amb = 0;
    double front = dot3(n, w) / d;
    if (fabs(front) <= FRONT_BAND) amb = 1;
    else if (!(front > 0.0)) fail = 1;
    double cos_y = -dot3(nl, w) / d; /* <n_y, w_{y'->x}> */
    if (!(cos_y > 0.0) && fabs(cos_y) > COS_BAND) return r;
    double co[3];
    sub3(c, o, co);
    double s = dot3(nl, co) / dot3(nl, w); /* y' = o + s w */
    double yp[3] = {o[0] + s * w[0], o[1] + s * w[1], o[2] + s * w[2]};
    double yc[3];
    sub3(yp, c, yc);
    double a = dot3(yc, eu) / dot3(eu, eu), b = dot3(yc, ev) / dot3(ev, ev);
    if (fabs(s - 1.0) <= LIGHT_BAND * fabs(s)) amb = 1;
    else if (!(s > 1.0)) fail = 1;
    if (fabs(fabs(a) - 0.5) <= LIGHT_BAND) amb = 1;
    else if (!(fabs(a) <= 0.5)) fail = 1;
    if (fabs(fabs(b) - 0.5) <= LIGHT_BAND) amb = 1;
    else if (!(fabs(b) <= 0.5)) fail = 1;
    /* a ray nearly parallel to the light's plane meets it far outside the
     * rectangle; only if it still lands on the light is the value unstable */
    if (!fail && fabs(cos_y) <= COS_BAND) {
        r.excl = 1;
        return r;
    }
    double cos_z = -dot3(nz, w) / d; /* <n_z, w_{z->x}> */
    if (fabs(cos_z) <= COS_BAND) amb = 1;
    else if (!(cos_z > 0.0)) fail = 1;
    if (fail) return r;
    double xy[3];
    sub3(o, yp, xy);
    double J = fabs(cos_z) * dot3(xy, xy) / (cos_y * d2);
    r.ppass = J / area;
    r.amb = amb;
    int pass = front > 0.0 && s > 1.0 && fabs(a) <= 0.5 && fabs(b) <= 0.5 && cos_z > 0.0;
    r.p = pass ? r.ppass : 0.0;
    return r;
}

/* Light coordinates (a, b) of y'(x, z): the ray from o through z meets the
 * light's plane at y' = c + a e_u + b e_v (the rectangle is |a|, |b| <= 1/2).
 * Returns 0 when the ray is parallel to the plane. */
static int yprime_coords(const double o[3], const double z[3], const double *L, double *a, double *b) {
    double c[3], eu[3], ev[3], nl[3], area, w[3], co[3];
    light_frame(L, c, eu, ev, nl, &area);
    sub3(z, o, w);
    sub3(c, o, co);
    double nw = dot3(nl, w);
    if (nw == 0.0) return 0;
    double s = dot3(nl, co) / nw;
    double yc[3] = {o[0] + s * w[0] - c[0], o[1] + s * w[1] - c[1], o[2] + s * w[2] - c[2]};
    *a = dot3(yc, eu) / dot3(eu, eu);
    *b = dot3(yc, ev) / dot3(ev, ev);
    return 1;
}

/* Area(A) p_A(y | x) of the bilinear density at light coordinates (a, b),
 * FP64: the bilinear interpolation over the unit square (u, v) = (a + 1/2,
 * b + 1/2) of the corner weights w_k = 1 / |o - y_k|^3 (|o - y_k|^2 clamped
 * below at 2^-40 as in the sampler), scaled by 4 / sum_k w_k so that its mean
 * over the rectangle, i.e. the integral of p_A, is 1. */
static double bilinear_q(const double o[3], const double *L, double a, double b) {
    double w[4], sum = 0.0;
    for (int k = 0; k < 4; ++k) {
        double ak = (k & 1) ? 0.5 : -0.5, bk = (k & 2) ? 0.5 : -0.5, d[3];
        for (int c = 0; c < 3; ++c) d[c] = o[c] - (L[c] + ak * L[3 + c] + bk * L[6 + c]);
        double d2 = dot3(d, d);
        if (d2 < 0x1p-40) d2 = 0x1p-40;
        w[k] = 1.0 / (d2 * sqrt(d2));
        sum += w[k];
    }
    double u = a + 0.5, v = b + 0.5;
    double bil = (1.0 - u) * (1.0 - v) * w[0] + u * (1.0 - v) * w[1] + (1.0 - u) * v * w[2] + u * v * w[3];
    return 4.0 * bil / sum;
}

/* q_x(y'(x, z)) = Area(A) p_A(y' | x) for the light density of the parameters
 * (1 for the uniform density). */
static double emitter_q(const orc_params *p, const double o[3], const double z[3]) {
    if (p->light_pdf != 1) return 1.0;
    double L[9], a, b;
    for (int q = 0; q < 9; ++q) L[q] = p->light[q];
    if (!yprime_coords(o, z, L, &a, &b)) return 1.0;
    return bilinear_q(o, L, a, b);
}

double orc_light_q(const double *o, const double *light, double a, double b) { return bilinear_q(o, light, a, b); }

double orc_density_ao(const double *o, const double *n, const double *z, const double *nz, double R) {
    return density_ao(o, n, z, nz, R).p;
}

double orc_density_shadow(const double *o, const double *n, const double *z, const double *nz,
                          const double *light) {
    return density_shadow(o, n, z, nz, light).p;
}

/* F_i: |A ∩ {y : <n, y - o> > 0}| / |A|, by clipping the rectangle polygon
 * against the receiver's tangent plane; 0 when the receiver is not on the
 * emitting side of the light's plane. */
static double front_fraction(const double o[3], const double n[3], const double *L, int *near_edge) {
    double c[3], eu[3], ev[3], nl[3], area;
    light_frame(L, c, eu, ev, nl, &area);
    double oc[3];
    sub3(o, c, oc);
    double side = dot3(nl, oc);
    if (near_edge) *near_edge = fabs(side) <= LIGHT_BAND * len3(oc);
    if (!(side > 0.0)) return 0.0;
    double P[4][3], Q[8][3];
    const double su[4] = {-0.5, 0.5, 0.5, -0.5}, sv[4] = {-0.5, -0.5, 0.5, 0.5};
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) P[k][a] = c[a] + su[k] * eu[a] + sv[k] * ev[a];
    int m = 0;
    for (int k = 0; k < 4; ++k) {
        const double *A = P[k], *B = P[(k + 1) % 4];
        double da[3], db[3];
        sub3(A, o, da);
        sub3(B, o, db);
        double fa = dot3(n, da), fb = dot3(n, db);
        if (fa > 0.0) { memcpy(Q[m++], A, sizeof(double) * 3); }
        if ((fa > 0.0) != (fb > 0.0)) {
            double t = fa / (fa - fb);
            for (int a = 0; a < 3; ++a) Q[m][a] = A[a] + t * (B[a] - A[a]);
            ++m;
        }
    }
    if (m < 3) return 0.0;
    double acc[3] = {0, 0, 0};
    for (int k = 1; k + 1 < m; ++k) {
        double e1[3], e2[3], x[3];
        sub3(Q[k], Q[0], e1);
        sub3(Q[k + 1], Q[0], e2);
        cross3(e1, e2, x);
        acc[0] += x[0]; acc[1] += x[1]; acc[2] += x[2];
    }
    return 0.5 * len3(acc) / area;
}

double orc_front_fraction(const double *o, const double *n, const double *light) {
    return front_fraction(o, n, light, NULL);
}

/* ------------------------------------------------------------------------ */
/* Solid-angle shadows.                                                     */
/* ------------------------------------------------------------------------ */

/* Solid angle of the triangle with vertices a, b, c (vectors from the
 * viewpoint), by the formula of Van Oosterom and Strackee (IEEE Trans.
 * Biomed. Eng. BME-30, 1983):
 *   tan(Omega / 2) = |a . (b x c)| / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|). */
static double tri_solid_angle(const double a[3], const double b[3], const double c[3]) {
    double bc[3];
    cross3(b, c, bc);
    double num = fabs(dot3(a, bc));
    double la = len3(a), lb = len3(b), lc = len3(c);
    double den = la * lb * lc + dot3(a, b) * lc + dot3(a, c) * lb + dot3(b, c) * la;
    return 2.0 * atan2(num, den);
}

/* Solid angle at o of a convex planar polygon Q[0..m), as a fan of
 * triangles from Q[0] (all of one orientation as seen from o). */
static double polygon_solid_angle(const double o[3], double Q[][3], int m) {
    double acc = 0.0;
    for (int k = 1; k + 1 < m; ++k) {
        double a[3], b[3], c[3];
        sub3(Q[0], o, a);
        sub3(Q[k], o, b);
        sub3(Q[k + 1], o, c);
        acc += tri_solid_angle(a, b, c);
    }
    return acc;
}

/* Omega_A(x), the solid angle the one-sided emitter subtends at o, and the
 * part of it in front of the receiver's tangent plane (the rectangle
 * clipped by <n, y - o> > 0); both 0 when o is not on the emitting side. */
static void emitter_solid_angles(const double o[3], const double n[3], const double *L, double *all,
                                 double *front, int *near_edge) {
    double c[3], eu[3], ev[3], nl[3], area;
    light_frame(L, c, eu, ev, nl, &area);
    double oc[3];
    sub3(o, c, oc);
    double side = dot3(nl, oc);
    if (near_edge) *near_edge = fabs(side) <= LIGHT_BAND * len3(oc);
    *all = 0.0;
    *front = 0.0;
    if (!(side > 0.0)) return;
    double P[4][3], Q[8][3];
    const double su[4] = {-0.5, 0.5, 0.5, -0.5}, sv[4] = {-0.5, -0.5, 0.5, 0.5};
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) P[k][a] = c[a] + su[k] * eu[a] + sv[k] * ev[a];
    *all = polygon_solid_angle(o, P, 4);
    int m = 0;
    for (int k = 0; k < 4; ++k) {
        const double *A = P[k], *B = P[(k + 1) % 4];
        double da[3], db[3];
        sub3(A, o, da);
        sub3(B, o, db);
        double fa = dot3(n, da), fb = dot3(n, db);
        if (fa > 0.0) { memcpy(Q[m++], A, sizeof(double) * 3); }
        if ((fa > 0.0) != (fb > 0.0)) {
            double t = fa / (fa - fb);
            for (int a = 0; a < 3; ++a) Q[m][a] = A[a] + t * (B[a] - A[a]);
            ++m;
        }
    }
    *front = m >= 3 ? polygon_solid_angle(o, Q, m) : 0.0;
}

/* C_Omega(x, z) = Area(A) / Omega_A(x) * <n_y', w_{y'->x}> / |x - y'|^2 at
 * the light crossing y'(x, z) of the ray from x through z (Eq.
 * reapp-shadow-solid-angle-mis-factor); 0 where that crossing does not
 * exist (the ray runs away from or parallel to the light's plane). */
static double sa_factor(const double o[3], const double z[3], const double *L, double omega_all) {
    double c[3], eu[3], ev[3], nl[3], area;
    light_frame(L, c, eu, ev, nl, &area);
    if (!(omega_all > 0.0)) return 0.0;
    double w[3], co[3];
    sub3(z, o, w);
    double nlw = dot3(nl, w);
    if (!(nlw < 0.0)) return 0.0;
    sub3(c, o, co);
    double s = dot3(nl, co) / nlw; /* y' = o + s w */
    double d = len3(w);
    double cos_y = -nlw / d;          /* <n_y', w_{y'->x}> */
    double r2 = s * s * d * d;        /* |x - y'|^2 */
    return area / omega_all * cos_y / r2;
}

/* ------------------------------------------------------------------------ */
/* Direct illumination (mode 3), in units of rho L_e / pi: for a Lambertian  */
/* receiver of albedo rho under a one-sided emitter of radiance L_e,         */
/* g(x, y) = (rho / pi) L_e cos+(n_x, w_{x->y}) <n_y, w_{y->x}> / |x - y|^2,   */
/* so the oracle's quantity is the visible irradiance of a unit-radiance     */
/* emitter, E_vis(x) = \int_A V cos+_x cos_y / |x - y|^2 dA.                  */
/* ------------------------------------------------------------------------ */

/* Irradiance at o (normal n) of a unit-radiance convex polygon Q[0..m) lying
 * in front of the tangent plane, by Lambert's formula:
 *   E = 1/2 |sum_k theta_k <n, (q_k x q_{k+1}) / |q_k x q_{k+1}|>|,
 * q_k = Q_k - o, theta_k the angle between q_k and q_{k+1}. */
static double lambert_polygon(const double o[3], const double n[3], double Q[][3], int m) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
        double a[3], b[3], c[3];
        sub3(Q[k], o, a);
        sub3(Q[(k + 1) % m], o, b);
        cross3(a, b, c);
        double lc = len3(c);
        if (lc == 0.0) continue;
        double th = atan2(lc, dot3(a, b));
        acc += th * dot3(n, c) / lc;
    }
    return 0.5 * fabs(acc);
}

/* U / (rho L_e / pi): the unshadowed term of Eq. reapp-di-unshadowed-term,
 * the irradiance of the part of the light in front of the tangent plane (0
 * for a receiver not on the emitting side). */
static double emitter_irradiance(const double o[3], const double n[3], const double *L, int *near_edge) {
    double c[3], eu[3], ev[3], nl[3], area;
    light_frame(L, c, eu, ev, nl, &area);
    double oc[3];
    sub3(o, c, oc);
    double side = dot3(nl, oc);
    if (near_edge) *near_edge = fabs(side) <= LIGHT_BAND * len3(oc);
    if (!(side > 0.0)) return 0.0;
    double P[4][3], Q[8][3];
    const double su[4] = {-0.5, 0.5, 0.5, -0.5}, sv[4] = {-0.5, -0.5, 0.5, 0.5};
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) P[k][a] = c[a] + su[k] * eu[a] + sv[k] * ev[a];
    int m = 0;
    for (int k = 0; k < 4; ++k) {
        const double *A = P[k], *B = P[(k + 1) % 4];
        double da[3], db[3];
        sub3(A, o, da);
        sub3(B, o, db);
        double fa = dot3(n, da), fb = dot3(n, db);
        if (fa > 0.0) { memcpy(Q[m++], A, sizeof(double) * 3); }
        if ((fa > 0.0) != (fb > 0.0)) {
            double t = fa / (fa - fb);
            for (int a = 0; a < 3; ++a) Q[m][a] = A[a] + t * (B[a] - A[a]);
            ++m;
        }
    }
    return m >= 3 ? lambert_polygon(o, n, Q, m) : 0.0;
}

/* C_DI(x, z) / (rho L_e / pi) = Area cos+_x <n_y', w_{y'->x}> / |x - y'|^2 at
 * the light crossing y' (Eq. reapp-di-general-mis-factor with p_A = 1/Area);
 * 0 where the crossing does not exist. */
static double di_factor(const double o[3], const double n[3], const double z[3], const double *L) {
    double c[3], eu[3], ev[3], nl[3], area;
    light_frame(L, c, eu, ev, nl, &area);
    double w[3], co[3];
    sub3(z, o, w);
    double nlw = dot3(nl, w);
    if (!(nlw < 0.0)) return 0.0;
    sub3(c, o, co);
    double s = dot3(nl, co) / nlw;
    double d = len3(w);
    double cos_x = dot3(n, w) / d;
    if (!(cos_x > 0.0)) return 0.0;
    double cos_y = -nlw / d;
    return area * cos_x * cos_y / (s * s * d * d);
}

double orc_emitter_irradiance(const double *o, const double *n, const double *light) {
    return emitter_irradiance(o, n, light, NULL);
}

double orc_di_factor(const double *o, const double *n, const double *z, const double *light) {
    return di_factor(o, n, z, light);
}

void orc_solid_angles(const double *o, const double *n, const double *light, double *out2) {
    emitter_solid_angles(o, n, light, &out2[0], &out2[1], NULL);
}

double orc_sa_factor(const double *o, const double *n, const double *z, const double *light) {
    double all, front;
    emitter_solid_angles(o, n, light, &all, &front, NULL);
    return sa_factor(o, z, light, all);
}

/* ------------------------------------------------------------------------ */
/* Reuse sets (Eq. reuse-group).                                            */
/* ------------------------------------------------------------------------ */
static void group_dims(int32_t N, int *gw, int *gh) {
    *gw = N == 8 ? 4 : (N >= 2 ? 2 : 1);
    *gh = N >= 4 ? 2 : 1;
}

/* Valid pixels of the reuse set of (ix, iy), in raster order. */
static int reuse_set(const orc_params *p, int32_t W, int32_t H, const uint32_t *prim, int ix, int iy,
                     int64_t *out) {
    int x0, x1, y0, y1, m = 0;
    if (p->estimator == 0) {
        x0 = ix; x1 = ix; y0 = iy; y1 = iy;
    } else if (p->pattern == 0) {
        x0 = ix - p->radius; x1 = ix + p->radius;
        y0 = iy - p->radius; y1 = iy + p->radius;
    } else {
        int gw, gh;
        group_dims(p->group_n, &gw, &gh);
        x0 = (ix / gw) * gw; x1 = x0 + gw - 1;
        y0 = (iy / gh) * gh; y1 = y0 + gh - 1;
    }
    for (int y = y0; y <= y1; ++y) {
        if (y < 0 || y >= H) continue;
        for (int x = x0; x <= x1; ++x) {
            if (x < 0 || x >= W) continue;
            int64_t j = (int64_t)y * W + x;
            if (prim[j] != ORC_MISS) out[m++] = j;
        }
    }
    return m;
}

static int max_offset(const orc_params *p) {
    if (p->pattern == 0) return 2 * p->radius;
    int gw, gh;
    group_dims(p->group_n, &gw, &gh);
    return (gw > gh ? gw : gh) - 1;
}

static int same_set_possible(const orc_params *p, int jx, int jy, int kx, int ky) {
    if (p->pattern == 0) return abs(jx - kx) <= 2 * p->radius && abs(jy - ky) <= 2 * p->radius;
    int gw, gh;
    group_dims(p->group_n, &gw, &gh);
    return jx / gw == kx / gw && jy / gh == ky / gh;
}

/* ------------------------------------------------------------------------ */
/* Estimators (Eqs. ao-unbiased-estimator / ao-biased-estimator,            */
/* shadow-estimator / shadow-biased-estimator; App. D and App. H).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_scene *s;
    int32_t W, H;
    const float *pos, *nrm;
    const uint32_t *prim;
    const orc_params *p;
    const uint32_t *hit;
    const double *z, *nz;
    const uint8_t *graze;
    /* first-hit validation table (unbiased): indexed by candidate pixel j in
     * the region [rx0,rx1) x [ry0,ry1) and offset (k - j) in [-D, D]^2 */
    int32_t rx0, ry0, rx1, ry1, D;
    uint8_t *occ; /* 0 not needed, 1 first hit, 2 blocked, 3 first hit (grazing), 4 blocked (grazing) */
} reuse_ctx;

static void receiver_point(const reuse_ctx *c, int64_t k, double o[3], double n[3]) {
    float of[3];
    offset_point(c->pos + 3 * k, c->nrm + 3 * k, of);
    f2d(of, o);
    f2d(c->nrm + 3 * k, n);
}

/* The light-frame area of light k (FP64). */
static double light_area64(const orc_params *p, int k) {
    double L[9], cc[3], eu[3], ev[3], nl[3], area;
    for (int q = 0; q < 9; ++q) L[q] = light_k(p, k)[q];
    light_frame(L, cc, eu, ev, nl, &area);
    return area;
}

static dens_t pair_density(const reuse_ctx *c, int64_t k, int64_t j) {
    double o[3], n[3];
    receiver_point(c, k, o, n);
    if (c->p->mode == 0) return density_ao(o, n, c->z + 3 * j, c->nz + 3 * j, c->p->ao_radius);
    int K = num_lights(c->p);
    if (K == 1) {
        double L[9];
        for (int q = 0; q < 9; ++q) L[q] = c->p->light[q];
        dens_t d = density_shadow(o, n, c->z + 3 * j, c->nz + 3 * j, L);
        if (c->p->light_pdf == 1 && d.ppass > 0.0) {
            /* a general emitter density (Eq. reapp-shadow-general-solid-angle-pdf):
             * p_A(y' | x) J chi_A = q_x(y') (1 / Area) J chi_A */
            double q = emitter_q(c->p, o, c->z + 3 * j);
            d.p *= q;
            d.ppass *= q;
        }
        return d;
    }
    /* several lights: the density of z over the union of the lights is the
     * area-weighted sum of the per-light densities, sum_l (A_l / A_tot) p_l */
    double A[4], tot = 0.0;
    for (int l = 0; l < K; ++l) tot += (A[l] = light_area64(c->p, l));
    dens_t r = {0.0, 0.0, 0, 0};
    for (int l = 0; l < K; ++l) {
        double L[9];
        for (int q = 0; q < 9; ++q) L[q] = light_k(c->p, l)[q];
        dens_t d = density_shadow(o, n, c->z + 3 * j, c->nz + 3 * j, L);
        r.p += A[l] / tot * d.p;
        r.ppass += A[l] / tot * d.ppass;
        r.amb |= d.amb;
        r.excl |= d.excl;
    }
    return r;
}

static uint8_t *occ_slot(const reuse_ctx *c, int64_t j, int64_t k) {
    int jx = (int)(j % c->W), jy = (int)(j / c->W), kx = (int)(k % c->W), ky = (int)(k / c->W);
    int64_t rw = c->rx1 - c->rx0, side = 2 * c->D + 1;
    int64_t jr = (int64_t)(jy - c->ry0) * rw + (jx - c->rx0);
    return c->occ + jr * side * side + (int64_t)(ky - jy + c->D) * side + (kx - jx + c->D);
}

/* First-hit validation, Eq. (occ-first-hit): z_j is the first hit from o_k
 * iff the segment o_k -> z_j is free over t in (0, 1 - eta), ignoring the
 * candidate's own triangle and the receiver's triangle. */
static void validate_all(reuse_ctx *c) {
    int64_t rw = c->rx1 - c->rx0, rh = c->ry1 - c->ry0, side = 2 * c->D + 1;
#pragma omp parallel
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < rw * rh; ++q) {
            int jx = c->rx0 + (int)(q % rw), jy = c->ry0 + (int)(q / rw);
            int64_t j = (int64_t)jy * c->W + jx;
            if (c->hit[j] >= ORC_SELF) continue;
            for (int dy = -c->D; dy <= c->D; ++dy)
                for (int dx = -c->D; dx <= c->D; ++dx) {
                    int kx = jx + dx, ky = jy + dy;
                    if (kx < c->rx0 || kx >= c->rx1 || ky < c->ry0 || ky >= c->ry1) continue;
                    if (dx == 0 && dy == 0) continue;
                    if (!same_set_possible(c->p, jx, jy, kx, ky)) continue;
                    int64_t k = (int64_t)ky * c->W + kx;
                    if (c->prim[k] == ORC_MISS) continue;
                    dens_t pd = pair_density(c, k, j);
                    if (!(pd.ppass > 0.0)) continue;
                    double o[3], n[3], w[3], tmax = 1.0 - VALID_ETA;
                    receiver_point(c, k, o, n);
                    sub3(c->z + 3 * j, o, w);
                    uint8_t blocked, g;
                    any_one(c->s, &cand, o, w, tmax, c->hit[j], c->prim[k], &blocked, &g);
                    c->occ[q * side * side + (int64_t)(dy + c->D) * side + (dx + c->D)] =
                        (uint8_t)((blocked ? 2 : 1) + (g ? 2 : 0));
                }
        }
        free(cand.ids);
    }
}

/* Effective density of candidate j at receiver k for the chosen estimator. */
static dens_t eff_density(const reuse_ctx *c, int64_t k, int64_t j) {
    dens_t d = pair_density(c, k, j);
    if (c->p->estimator != 2 || k == j) return d; /* Occ(x_j, z_j) = 1 */
    if (!(d.ppass > 0.0)) return d;
    uint8_t o = *occ_slot(c, j, k);
    if (o == 1) return d;
    if (o == 2) { dens_t z0 = {0.0, 0.0, 0, 0}; return z0; }
    /* grazing validation: the density is either its geometric value or 0 */
    d.amb = 1;
    if (o == 4) d.p = 0.0;
    return d;
}

#define MAXSET 289 /* (2*8+1)^2 */

typedef struct {
    int64_t S[MAXSET];
    int m;
    double *P;      /* m x m: P[a*m + b] = density of candidate S[b] at receiver S[a] */
    double *Ppass;
    double *Pv;     /* a variant of P (parity support) */
    int *amb;
    idlist cand;    /* tracer scratch (light-sample reuse) */
} target_buf;

/* Final-value filtering (Sec. 6, Filter (N); for shadows also Light (N),
 * light-sample reuse without visibility validation, which reduces to the
 * same average): the mean over the valid pixels j of S(i) of their
 * one-sample no-reuse estimates [the ray or segment of j is free]. */
static double eval_filter(const reuse_ctx *c, target_buf *t, int ix, int iy) {
    t->m = reuse_set(c->p, c->W, c->H, c->prim, ix, iy, t->S);
    double acc = 0.0;
    for (int a = 0; a < t->m; ++a) acc += c->hit[t->S[a]] == ORC_MISS ? 1.0 : 0.0;
    return acc / t->m;
}

/* Light-sample reuse with visibility re-evaluation (Sec. 6, Light (NU)):
 * target i re-traces the light sample y_j of every pixel j of S(i),
 *   Shadow_i = (1/|S(i)|) sum_j V(x_i, y_j),
 * unbiased because every y_j is uniform on the light independently of x_i.
 * V = 0 for a y_j behind the tangent plane of x_i or an x_i behind the
 * light (the FP32 tests of the sample specification, so that both sides
 * decide them identically), else 1 when the segment o_i -> y_j is free over
 * t in (0, 1), ignoring x_i's own triangle.  Grazing traces make the pair
 * ambiguous: up to three are enumerated, more make the target not
 * comparable. */
static void eval_light_reuse(const reuse_ctx *c, target_buf *t, int ix, int iy, double *value, uint8_t *nvar,
                             double *var) {
    const orc_params *p = c->p;
    int64_t i = (int64_t)iy * c->W + ix;
    t->m = reuse_set(p, c->W, c->H, c->prim, ix, iy, t->S);
    float o[3];
    const float *n = c->nrm + 3 * i, *L = p->light;
    offset_point(c->pos + 3 * i, n, o);
    uint32_t sd = seed32(p->seed);
    float nl[3] = {L[4] * L[8] - L[5] * L[7], L[5] * L[6] - L[3] * L[8], L[3] * L[7] - L[4] * L[6]};
    float lit = fmaf(nl[2], o[2] - L[2], fmaf(nl[1], o[1] - L[1], nl[0] * (o[0] - L[0])));
    int vis = 0, namb = 0, amb_vis[MAX_AMBIG];
    for (int a = 0; a < t->m; ++a) {
        int64_t j = t->S[a];
        float y[3], dir[3];
        light_point((uint32_t)(j % c->W), (uint32_t)(j / c->W), p->sample, sd, L, y);
        for (int q = 0; q < 3; ++q) dir[q] = y[q] - o[q];
        float front = fmaf(n[2], dir[2], fmaf(n[1], dir[1], n[0] * dir[0]));
        if (!(front > 0.0f) || !(lit > 0.0f)) continue;
        double od[3], dd[3];
        f2d(o, od);
        f2d(dir, dd);
        uint8_t blocked, g;
        any_one(c->s, &t->cand, od, dd, 1.0, c->prim[i], ORC_MISS, &blocked, &g);
        if (!blocked) ++vis;
        if (g) {
            if (namb < MAX_AMBIG) amb_vis[namb] = !blocked;
            ++namb;
        }
    }
    *value = (double)vis / t->m;
    if (namb > MAX_AMBIG) {
        *nvar = 0;
        return;
    }
    int nv = 1 << namb;
    for (int v = 0; v < nv; ++v) {
        int vv = vis;
        for (int q = 0; q < namb; ++q)
            if ((v >> q) & 1) vv += amb_vis[q] ? -1 : 1;
        var[v] = (double)vv / t->m;
    }
    *nvar = (uint8_t)nv;
}

/* The estimate's sum (App. D / App. H, step 3):
 *   B_i = sum_j [p_i(j) > 0 and P_i(j) > 0] C_ij p_i(j) / P_i(j),
 *   P_i(j) = sum_{k in S(i)} p_k(j),
 * over the set's densities Pm[a * m + b] = p_{S[a]}(z_{S[b]}) (receiver a,
 * candidate b), i = S[ia]; C_ij = cfac[b] (the solid-angle, direct-lighting
 * or emitter-density factor of the estimator), 1 when cfac is NULL. */
static double mis_sum(const reuse_ctx *c, const target_buf *t, const double *Pm, int ia, const double *cfac) {
    int m = t->m;
    double B = 0.0;
    for (int b = 0; b < m; ++b) {
        if (c->hit[t->S[b]] >= ORC_SELF) continue;
        double Pj = 0.0;
        for (int a = 0; a < m; ++a) Pj += Pm[a * m + b];
        double pij = Pm[ia * m + b];
        if (pij > 0.0 && Pj > 0.0) B += (cfac ? cfac[b] : 1.0) * (pij / Pj);
    }
    return B;
}

/* Parity support, not part of the estimator: the densities whose support
 * decision lies within FP32 rounding of its threshold (t->amb) may be
 * decided either way by an FP32 implementation.  Variant `mask` of the
 * matrix takes, for the q-th such density, its in-support value when bit q
 * is set and 0 otherwise. */
static void variant_matrix(const target_buf *t, const int *amb_idx, int namb, unsigned mask, double *Pv) {
    int m = t->m;
    for (int e = 0; e < m * m; ++e) {
        double v = t->P[e];
        if (t->amb[e]) {
            v = 0.0;
            for (int q = 0; q < namb; ++q)
                if (amb_idx[q] == e && ((mask >> q) & 1u)) v = t->Ppass[e];
        }
        Pv[e] = v;
    }
}

static void eval_target(const reuse_ctx *c, target_buf *t, int ix, int iy, double *value, uint8_t *nvar,
                        double *var) {
    int64_t i = (int64_t)iy * c->W + ix;
    const orc_params *p = c->p;
    *nvar = 0;
    *value = 0.0;
    if (c->prim[i] == ORC_MISS) {
        /* background pixel: no estimate is defined; the output convention is
         * 1 for AO (nothing occludes) and 0 for shadows (no lit surface) */
        *value = p->mode == 0 ? 1.0 : 0.0;
        var[0] = *value;
        *nvar = 1;
        return;
    }
    if (p->estimator == 3) {
        *value = eval_filter(c, t, ix, iy);
        var[0] = *value;
        *nvar = 1;
        return;
    }
    if (p->estimator == 4) {
        eval_light_reuse(c, t, ix, iy, value, nvar, var);
        return;
    }
    if (p->estimator == 0 && p->mode < 2 && p->light_pdf == 0) {
        /* Eqs. (ao-mc-estimator) and (shadow-mc-estimator), one sample:
         * V = 1 when the ray or segment is free.  (Solid-angle shadows take
         * the general path below with S(i) = {i}, and so do shadows sampled
         * from a general emitter density, whose one-sample weight is
         * 1 / (Area p_A(y' | x)).) */
        *value = c->hit[i] == ORC_MISS ? 1.0 : 0.0;
        var[0] = *value;
        *nvar = 1;
        return;
    }
    t->m = reuse_set(p, c->W, c->H, c->prim, ix, iy, t->S);
    int m = t->m, excluded = 0, ia = -1;
    for (int a = 0; a < m; ++a)
        if (t->S[a] == i) ia = a;
    int amb_idx[MAX_AMBIG + 1], namb = 0;
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            int e = a * m + b;
            t->P[e] = 0.0;
            t->Ppass[e] = 0.0;
            t->amb[e] = 0;
            int64_t j = t->S[b];
            if (c->hit[j] >= ORC_SELF) continue;
            dens_t d = eff_density(c, t->S[a], j);
            t->P[e] = d.p;
            t->Ppass[e] = d.ppass;
            t->amb[e] = d.amb;
            if (d.excl) excluded = 1;
            if (d.amb) {
                if (namb < MAX_AMBIG) amb_idx[namb] = e;
                ++namb;
            }
        }
    double F = 1.0;
    double cfac[MAXSET], *cf = NULL;
    if (p->mode == 1) {
        /* F_i; for several lights the area-weighted sum of the per-light
         * fractions (the front part of the union) */
        double o[3], n[3];
        receiver_point(c, i, o, n);
        int K = num_lights(p);
        double tot = 0.0, A[4];
        for (int l = 0; l < K; ++l) tot += (A[l] = light_area64(p, l));
        F = 0.0;
        for (int l = 0; l < K; ++l) {
            double L[9];
            int near;
            for (int q = 0; q < 9; ++q) L[q] = light_k(p, l)[q];
            double Fl = front_fraction(o, n, L, &near);
            if (near) excluded = 1;
            F += K == 1 ? Fl : A[l] / tot * Fl;
        }
    } else if (p->mode == 2) {
        /* Solid-angle definition: the visible fraction of Omega_A(x_i) is
         * F_Omega - B_i with F_Omega = Omega_front / Omega_A the part of the
         * emitter's solid angle in front of the tangent plane (the analogue
         * of F_i), and B_i weighted by C_Omega(x_i, z_j). */
        double o[3], n[3], L[9], all, front;
        int near;
        receiver_point(c, i, o, n);
        for (int q = 0; q < 9; ++q) L[q] = p->light[q];
        emitter_solid_angles(o, n, L, &all, &front, &near);
        if (near) excluded = 1;
        F = all > 0.0 ? front / all : 0.0;
        for (int b = 0; b < m; ++b)
            cfac[b] = c->hit[t->S[b]] < ORC_SELF ? sa_factor(o, c->z + 3 * t->S[b], L, all) : 0.0;
        cf = cfac;
    } else if (p->mode == 3) {
        /* Direct illumination (Eq. reapp-di-general-mis-estimator), in units
         * of rho L_e / pi: U - sum_j C_DI(x_i, z_j) p_i(j) / P_i(j). */
        double o[3], n[3], L[9];
        int near;
        receiver_point(c, i, o, n);
        for (int q = 0; q < 9; ++q) L[q] = p->light[q];
        F = emitter_irradiance(o, n, L, &near);
        if (near) excluded = 1;
        for (int b = 0; b < m; ++b)
            cfac[b] = c->hit[t->S[b]] < ORC_SELF ? di_factor(o, n, c->z + 3 * t->S[b], L) : 0.0;
        cf = cfac;
    }
    if (p->mode != 0 && p->light_pdf == 1) {
        /* a general emitter density: every estimator factor divides by
         * Area p_A(y'_ij | x_i) (C^gen of Eqs. reapp-shadow-general-solid-angle-mis-factor
         * and reapp-di-general-one-sample-blocked; 1 / (Area p_A) for the area
         * definition, whose factor is 1 under the uniform density) */
        double o[3], n[3];
        receiver_point(c, i, o, n);
        for (int b = 0; b < m; ++b) {
            int64_t j = t->S[b];
            double q = c->hit[j] < ORC_SELF ? emitter_q(p, o, c->z + 3 * j) : 1.0;
            cfac[b] = (cf ? cfac[b] : 1.0) / q;
        }
        cf = cfac;
    }
    /* Dark-region guard (Sec. 4.4, biased shadows): every sample of the set
     * blocked (an occluder hit, or no visible light sample at all). */
    int dark = 0;
    if (p->mode != 0 && p->estimator == 1 && p->dark_guard) {
        dark = 1;
        for (int a = 0; a < m; ++a)
            if (c->hit[t->S[a]] == ORC_MISS) dark = 0;
    }
    double B = mis_sum(c, t, t->P, ia, cf);
    *value = dark ? 0.0 : (p->mode == 0 ? 1.0 - B : F - B);
    /* admissible values of an FP32 implementation (parity support) */
    if (excluded || namb > MAX_AMBIG) return;
    int nv = 1 << namb;
    for (int v = 0; v < nv; ++v) {
        variant_matrix(t, amb_idx, namb, (unsigned)v, t->Pv);
        double Bv = mis_sum(c, t, t->Pv, ia, cf);
        var[v] = dark ? 0.0 : (p->mode == 0 ? 1.0 - Bv : F - Bv);
    }
    *nvar = (uint8_t)nv;
}

static void region_for(const orc_params *p, int32_t W, int32_t H, int32_t x0, int32_t y0, int32_t x1,
                       int32_t y1, int32_t *r) {
    if (p->estimator == 0) {
        r[0] = x0; r[1] = y0; r[2] = x1; r[3] = y1;
    } else if (p->pattern == 0) {
        r[0] = x0 - p->radius; r[1] = y0 - p->radius; r[2] = x1 + p->radius; r[3] = y1 + p->radius;
    } else {
        int gw, gh;
        group_dims(p->group_n, &gw, &gh);
        r[0] = (x0 / gw) * gw; r[1] = (y0 / gh) * gh;
        r[2] = ((x1 + gw - 1) / gw) * gw; r[3] = ((y1 + gh - 1) / gh) * gh;
    }
    if (r[0] < 0) r[0] = 0;
    if (r[1] < 0) r[1] = 0;
    if (r[2] > W) r[2] = W;
    if (r[3] > H) r[3] = H;
}

void orc_reuse(const orc_scene *s, int32_t W, int32_t H, const float *pos, const float *nrm,
               const uint32_t *prim, const orc_params *p, const uint32_t *hit, const double *z,
               const double *nz, const uint8_t *graze, int32_t x0, int32_t y0, int32_t x1, int32_t y1,
               double *value, uint8_t *nvar, double *var) {
    reuse_ctx c;
    memset(&c, 0, sizeof c);
    c.s = s; c.W = W; c.H = H; c.pos = pos; c.nrm = nrm; c.prim = prim; c.p = p;
    c.hit = hit; c.z = z; c.nz = nz; c.graze = graze;
    int32_t r[4];
    region_for(p, W, H, x0, y0, x1, y1, r);
    c.rx0 = r[0]; c.ry0 = r[1]; c.rx1 = r[2]; c.ry1 = r[3];
    c.D = max_offset(p);
    if (p->estimator == 2) {
        int64_t side = 2 * c.D + 1;
        c.occ = (uint8_t *)calloc((size_t)((int64_t)(c.rx1 - c.rx0) * (c.ry1 - c.ry0) * side * side), 1);
        validate_all(&c);
    }
    int64_t w = x1 - x0, n = w * (int64_t)(y1 - y0);
#pragma omp parallel
    {
        target_buf t;
        t.P = (double *)malloc(sizeof(double) * MAXSET * MAXSET);
        t.Ppass = (double *)malloc(sizeof(double) * MAXSET * MAXSET);
        t.Pv = (double *)malloc(sizeof(double) * MAXSET * MAXSET);
        t.amb = (int *)malloc(sizeof(int) * MAXSET * MAXSET);
        t.cand.ids = NULL;
        t.cand.n = 0;
        t.cand.cap = 0;
#pragma omp for schedule(dynamic, 32)
        for (int64_t q = 0; q < n; ++q) {
            int ix = x0 + (int)(q % w), iy = y0 + (int)(q / w);
            int64_t i = (int64_t)iy * W + ix;
            eval_target(&c, &t, ix, iy, value + i, nvar + i, var + 8 * i);
        }
        free(t.P);
        free(t.Ppass);
        free(t.Pv);
        free(t.amb);
        free(t.cand.ids);
    }
    free(c.occ);
}

/* Accumulation over samples (final line of App. D / App. H): the estimate
 * for M samples is the mean of the per-sample estimates. */
void orc_render(const orc_scene *s, int32_t W, int32_t H, const float *pos, const float *nrm,
                const uint32_t *prim, const orc_params *p, int32_t M, int32_t x0, int32_t y0, int32_t x1,
                int32_t y1, double *sum, double *sumsq) {
    int64_t npx = (int64_t)W * H;
    uint32_t *hit = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)npx);
    double *z = (double *)calloc((size_t)npx * 3, sizeof(double));
    double *nz = (double *)calloc((size_t)npx * 3, sizeof(double));
    uint8_t *g = (uint8_t *)calloc((size_t)npx, 1);
    double *val = (double *)calloc((size_t)npx, sizeof(double));
    uint8_t *nv = (uint8_t *)calloc((size_t)npx, 1);
    double *var = (double *)calloc((size_t)npx * 8, sizeof(double));
    int32_t r[4];
    region_for(p, W, H, x0, y0, x1, y1, r);
    orc_params q = *p;
    for (int64_t i = 0; i < npx; ++i) { sum[i] = 0.0; sumsq[i] = 0.0; hit[i] = ORC_MISS; }
    for (int32_t m = 0; m < M; ++m) {
        q.sample = p->sample + (uint32_t)m;
        orc_records(s, W, H, pos, nrm, prim, &q, r[0], r[1], r[2], r[3], hit, z, nz, g);
        orc_reuse(s, W, H, pos, nrm, prim, &q, hit, z, nz, g, x0, y0, x1, y1, val, nv, var);
        for (int32_t y = y0; y < y1; ++y)
            for (int32_t x = x0; x < x1; ++x) {
                int64_t i = (int64_t)y * W + x;
                sum[i] += val[i];
                sumsq[i] += val[i] * val[i];
            }
    }
    free(hit); free(z); free(nz); free(g); free(val); free(nv); free(var);
}

/* ------------------------------------------------------------------------ */
/* FP64 quadrature references.                                              */
/* ------------------------------------------------------------------------ */

/* AO(x) = (1/pi) \int V cos dw (Eq. ao-hemisphere).  Under the cosine
 * measure the hemisphere is the unit disc with (u, phi), u = r^2, uniform,
 * so the midpoint rule on an nstrata^2 grid of (u, phi) integrates it. */
double orc_ao_quadrature(const orc_scene *s, const double *o, const double *n, double R, uint32_t ign,
                         int32_t nstrata) {
    double nn[3] = {n[0], n[1], n[2]}, l = len3(nn);
    nn[0] /= l; nn[1] /= l; nn[2] /= l;
    double helper[3] = {1.0, 0.0, 0.0};
    if (fabs(nn[0]) > 0.9) { helper[0] = 0.0; helper[1] = 1.0; }
    double t1[3], t2[3];
    cross3(nn, helper, t1);
    l = len3(t1);
    t1[0] /= l; t1[1] /= l; t1[2] /= l;
    cross3(nn, t1, t2);
    double vis = 0.0;
#pragma omp parallel reduction(+ : vis)
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int32_t a = 0; a < nstrata; ++a) {
            double u = (a + 0.5) / nstrata, rr = sqrt(u), zc = sqrt(1.0 - u);
            for (int32_t b = 0; b < nstrata; ++b) {
                double ph = 2.0 * PI * (b + 0.5) / nstrata;
                double lx = rr * cos(ph), ly = rr * sin(ph), d[3];
                for (int c = 0; c < 3; ++c) d[c] = lx * t1[c] + ly * t2[c] + zc * nn[c];
                uint32_t tri;
                double t;
                uint8_t g;
                closest_one(s, &cand, o, d, R, 1, ign, ORC_MISS, &tri, &t, &g);
                if (tri == ORC_MISS) vis += 1.0;
            }
        }
        free(cand.ids);
    }
    return vis / ((double)nstrata * nstrata);
}

/* Shadow(x) = (1/Area) \int_A V(x,y) dmu(y) (Eq. shadow-area), with V = 0 for
 * light points behind the tangent plane and for a receiver behind the
 * one-sided light; midpoint rule on an ngrid^2 grid over the rectangle. */
double orc_shadow_quadrature(const orc_scene *s, const double *o, const double *n, const double *light,
                             uint32_t ign, int32_t ngrid) {
    double c[3], eu[3], ev[3], nl[3], area, oc[3];
    light_frame(light, c, eu, ev, nl, &area);
    sub3(o, c, oc);
    if (!(dot3(nl, oc) > 0.0)) return 0.0;
    double vis = 0.0;
#pragma omp parallel reduction(+ : vis)
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int32_t a = 0; a < ngrid; ++a)
            for (int32_t b = 0; b < ngrid; ++b) {
                double ua = (a + 0.5) / ngrid - 0.5, ub = (b + 0.5) / ngrid - 0.5, d[3];
                for (int q = 0; q < 3; ++q) d[q] = c[q] + ua * eu[q] + ub * ev[q] - o[q];
                if (!(dot3(n, d) > 0.0)) continue;
                uint8_t blocked, g;
                any_one(s, &cand, o, d, 1.0, ign, ORC_MISS, &blocked, &g);
                if (!blocked) vis += 1.0;
            }
        free(cand.ids);
    }
    return vis / ((double)ngrid * ngrid);
}

/* E_vis(x) = \int_A V cos+_x cos_y / |x - y|^2 dA (Eq. reapp-di-area-compact
 * in units of rho L_e / pi): midpoint rule on an ngrid^2 grid over the
 * rectangle; 0 for a receiver behind the one-sided light. */
double orc_di_quadrature(const orc_scene *s, const double *o, const double *n, const double *light, uint32_t ign,
                         int32_t ngrid) {
    double c[3], eu[3], ev[3], nl[3], area, oc[3];
    light_frame(light, c, eu, ev, nl, &area);
    sub3(o, c, oc);
    if (!(dot3(nl, oc) > 0.0)) return 0.0;
    double vis = 0.0;
    double dA = area / ((double)ngrid * ngrid);
#pragma omp parallel reduction(+ : vis)
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int32_t a = 0; a < ngrid; ++a)
            for (int32_t b = 0; b < ngrid; ++b) {
                double ua = (a + 0.5) / ngrid - 0.5, ub = (b + 0.5) / ngrid - 0.5, d[3];
                for (int q = 0; q < 3; ++q) d[q] = c[q] + ua * eu[q] + ub * ev[q] - o[q];
                double cx = dot3(n, d);
                if (!(cx > 0.0)) continue;
                uint8_t blocked, g;
                any_one(s, &cand, o, d, 1.0, ign, ORC_MISS, &blocked, &g);
                if (blocked) continue;
                double r2 = dot3(d, d);
                vis += cx * -dot3(nl, d) / (r2 * r2) * dA;
            }
        free(cand.ids);
    }
    return vis;
}

/* Shadow_Omega(x) = (1/Omega_A) \int_{Omega_A} V dw (Eq.
 * reapp-shadow-definition-solid-angle): the midpoint rule on an ngrid^2 grid
 * over the rectangle with each cell weighted by its solid angle
 * <n_y, w_{y->x}> dA / |x - y|^2, normalised by the sum of the weights; V = 0
 * behind the tangent plane, and 0 for a receiver behind the one-sided light. */
double orc_shadow_sa_quadrature(const orc_scene *s, const double *o, const double *n, const double *light,
                                uint32_t ign, int32_t ngrid) {
    double c[3], eu[3], ev[3], nl[3], area, oc[3];
    light_frame(light, c, eu, ev, nl, &area);
    sub3(o, c, oc);
    if (!(dot3(nl, oc) > 0.0)) return 0.0;
    double vis = 0.0, tot = 0.0;
#pragma omp parallel reduction(+ : vis, tot)
    {
        idlist cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int32_t a = 0; a < ngrid; ++a)
            for (int32_t b = 0; b < ngrid; ++b) {
                double ua = (a + 0.5) / ngrid - 0.5, ub = (b + 0.5) / ngrid - 0.5, d[3];
                for (int q = 0; q < 3; ++q) d[q] = c[q] + ua * eu[q] + ub * ev[q] - o[q];
                double r2 = dot3(d, d);
                double wgt = -dot3(nl, d) / sqrt(r2) / r2;
                tot += wgt;
                if (!(dot3(n, d) > 0.0)) continue;
                uint8_t blocked, g;
                any_one(s, &cand, o, d, 1.0, ign, ORC_MISS, &blocked, &g);
                if (!blocked) vis += wgt;
            }
        free(cand.ids);
    }
    return vis / tot;
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
