/*
 * Primary-visibility G-buffer writer for the seeded synthetic workloads.
 *
 * Fixture code: it turns a triangle scene and a pinhole camera into the
 * per-pixel shading point x, normal n_x and primitive id that the method
 * takes as input (the paper's notation of Sec. 3.1).  It is not part of the
 * method: neither the oracle nor the GPU library calls it, and its answers
 * are inputs to both.
 *
 * FP64 throughout: camera rays through pixel centres, closest hit over a
 * uniform grid of triangle bounding boxes, Moller-Trumbore intersection.
 * Output is stored as FP32; the normal is the geometric triangle normal
 * flipped to face the camera; background pixels get prim = 0xFFFFFFFF and
 * zero position/normal.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double lo[3], hi[3], cell[3], inv_cell[3];
    int32_t n[3];
    int64_t *start; /* ncells + 1 */
    uint32_t *refs;
} gb_grid;

static int64_t cidx(const gb_grid *g, int x, int y, int z) {
    return ((int64_t)z * g->n[1] + y) * g->n[0] + x;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void tri_box(const float *V, const uint32_t *F, int64_t t, double lo[3], double hi[3]) {
    for (int a = 0; a < 3; ++a) { lo[a] = 1e300; hi[a] = -1e300; }
    for (int k = 0; k < 3; ++k) {
        const float *p = V + 3 * (int64_t)F[3 * t + k];
        for (int a = 0; a < 3; ++a) {
            if (p[a] < lo[a]) lo[a] = p[a];
            if (p[a] > hi[a]) hi[a] = p[a];
        }
    }
}

static int grid_build(gb_grid *g, const float *V, int64_t nv, const uint32_t *F, int64_t nt) {
    for (int a = 0; a < 3; ++a) { g->lo[a] = 1e300; g->hi[a] = -1e300; }
    for (int64_t i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a) {
            if (V[3 * i + a] < g->lo[a]) g->lo[a] = V[3 * i + a];
            if (V[3 * i + a] > g->hi[a]) g->hi[a] = V[3 * i + a];
        }
    double ext[3], vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        g->lo[a] -= 1e-3; g->hi[a] += 1e-3;
        ext[a] = g->hi[a] - g->lo[a];
        vol *= ext[a];
    }
    double s = cbrt(vol / (2.0 * (double)(nt > 0 ? nt : 1)));
    for (int a = 0; a < 3; ++a) {
        int n = (int)ceil(ext[a] / s);
        g->n[a] = clampi(n, 1, 1024);
        g->cell[a] = ext[a] / g->n[a];
        g->inv_cell[a] = 1.0 / g->cell[a];
    }
    int64_t nc = (int64_t)g->n[0] * g->n[1] * g->n[2];
    g->start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    if (!g->start) return -1;
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t t = 0; t < nt; ++t) {
            double lo[3], hi[3];
            int c0[3], c1[3];
            tri_box(V, F, t, lo, hi);
            for (int a = 0; a < 3; ++a) {
                c0[a] = clampi((int)floor((lo[a] - g->lo[a]) * g->inv_cell[a]), 0, g->n[a] - 1);
                c1[a] = clampi((int)floor((hi[a] - g->lo[a]) * g->inv_cell[a]), 0, g->n[a] - 1);
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) {
                        int64_t c = cidx(g, x, y, z);
                        if (pass == 0) g->start[c + 1]++;
                        else g->refs[g->start[c]++] = (uint32_t)t;
                    }
        }
        if (pass == 0) {
            for (int64_t c = 0; c < nc; ++c) g->start[c + 1] += g->start[c];
            g->refs = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->start[nc] + 1));
            if (!g->refs) return -1;
        } else {
            /* undo the fill shift */
            for (int64_t c = nc; c > 0; --c) g->start[c] = g->start[c - 1];
            g->start[0] = 0;
        }
    }
    return 0;
}

/* Moller-Trumbore in FP64; returns t or -1 when there is no hit in (0, inf). */
static double mt_hit(const double o[3], const double d[3], const double a[3], const double b[3],
                     const double c[3]) {
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (fabs(det) < 1e-300) return -1.0;
    double inv = 1.0 / det;
    double s[3] = {o[0] - a[0], o[1] - a[1], o[2] - a[2]};
    double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) * inv;
    if (u < 0.0 || u > 1.0) return -1.0;
    double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return -1.0;
    double t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    return t > 0.0 ? t : -1.0;
}

static void load_v(const float *V, uint32_t i, double out[3]) {
    out[0] = V[3 * (int64_t)i]; out[1] = V[3 * (int64_t)i + 1]; out[2] = V[3 * (int64_t)i + 2];
}

/* Closest hit along (o,d) through the grid (Amanatides-Woo walk). */
static int64_t grid_cast(const gb_grid *g, const float *V, const uint32_t *F, const double o[3],
                         const double d[3], double *t_out) {
    double t0 = 0.0, t1 = 1e300;
    for (int a = 0; a < 3; ++a) {
        if (fabs(d[a]) < 1e-300) {
            if (o[a] < g->lo[a] || o[a] > g->hi[a]) return -1;
            continue;
        }
        double ta = (g->lo[a] - o[a]) / d[a], tb = (g->hi[a] - o[a]) / d[a];
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (t0 > t1) return -1;
    int c[3], step[3];
    double tnext[3], tdelta[3];
    for (int a = 0; a < 3; ++a) {
        double p = o[a] + t0 * d[a];
        c[a] = clampi((int)floor((p - g->lo[a]) * g->inv_cell[a]), 0, g->n[a] - 1);
        if (d[a] > 0) {
            step[a] = 1;
            tnext[a] = (g->lo[a] + (c[a] + 1) * g->cell[a] - o[a]) / d[a];
            tdelta[a] = g->cell[a] / d[a];
        } else if (d[a] < 0) {
            step[a] = -1;
            tnext[a] = (g->lo[a] + c[a] * g->cell[a] - o[a]) / d[a];
            tdelta[a] = -g->cell[a] / d[a];
        } else {
            step[a] = 0;
            tnext[a] = 1e300;
            tdelta[a] = 1e300;
        }
    }
    double best = 1e300;
    int64_t best_id = -1;
    for (;;) {
        int64_t ci = cidx(g, c[0], c[1], c[2]);
        for (int64_t r = g->start[ci]; r < g->start[ci + 1]; ++r) {
            uint32_t t = g->refs[r];
            double a[3], b[3], cc[3];
            load_v(V, F[3 * (int64_t)t], a);
            load_v(V, F[3 * (int64_t)t + 1], b);
            load_v(V, F[3 * (int64_t)t + 2], cc);
            double th = mt_hit(o, d, a, b, cc);
            if (th > 0.0 && (th < best || (th == best && (int64_t)t < best_id))) {
                best = th;
                best_id = t;
            }
        }
        int ax = tnext[0] < tnext[1] ? (tnext[0] < tnext[2] ? 0 : 2) : (tnext[1] < tnext[2] ? 1 : 2);
        if (best <= tnext[ax]) break;
        c[ax] += step[ax];
        if (c[ax] < 0 || c[ax] >= g->n[ax]) break;
        tnext[ax] += tdelta[ax];
    }
    *t_out = best;
    return best_id;
}

/*
 * Render a W x H G-buffer.  Camera basis (fwd, right, up) is orthonormal;
 * pixel (px,py) maps to fwd + sx*right + sy*up with
 * sx = (2(px+1/2)/W - 1) tan_half * W/H and sy = (1 - 2(py+1/2)/H) tan_half.
 */
int gb_render(const float *V, int64_t nv, const uint32_t *F, int64_t nt, const double *eye,
              const double *fwd, const double *right, const double *up, double tan_half, int32_t W,
              int32_t H, float *pos, float *nrm, uint32_t *prim) {
    gb_grid g;
    memset(&g, 0, sizeof g);
    if (grid_build(&g, V, nv, F, nt) != 0) return -1;
    double aspect = (double)W / (double)H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t py = 0; py < H; ++py) {
        for (int32_t px = 0; px < W; ++px) {
            double sx = (2.0 * (px + 0.5) / W - 1.0) * tan_half * aspect;
            double sy = (1.0 - 2.0 * (py + 0.5) / H) * tan_half;
            double d[3], len = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = fwd[a] + sx * right[a] + sy * up[a];
                len += d[a] * d[a];
            }
            len = sqrt(len);
            for (int a = 0; a < 3; ++a) d[a] /= len;
            double t;
            int64_t id = grid_cast(&g, V, F, eye, d, &t);
            int64_t p = (int64_t)py * W + px;
            if (id < 0) {
                prim[p] = 0xFFFFFFFFu;
                for (int a = 0; a < 3; ++a) { pos[3 * p + a] = 0.f; nrm[3 * p + a] = 0.f; }
                continue;
            }
            double a0[3], b0[3], c0[3];
            load_v(V, F[3 * id], a0);
            load_v(V, F[3 * id + 1], b0);
            load_v(V, F[3 * id + 2], c0);
            double e1[3] = {b0[0] - a0[0], b0[1] - a0[1], b0[2] - a0[2]};
            double e2[3] = {c0[0] - a0[0], c0[1] - a0[1], c0[2] - a0[2]};
            double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                           e1[0] * e2[1] - e1[1] * e2[0]};
            double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            double sgn = (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]) > 0 ? -1.0 : 1.0;
            prim[p] = (uint32_t)id;
            for (int a = 0; a < 3; ++a) {
                pos[3 * p + a] = (float)(eye[a] + t * d[a]);
                nrm[3 * p + a] = (float)(sgn * n[a] / nl);
            }
        }
    }
    free(g.start);
    free(g.refs);
    return 0;
}
