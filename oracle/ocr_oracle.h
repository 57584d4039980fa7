/*
 * CPU oracle for occlusion-point reuse.  TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the GPU library, and it shares no code with it.
 *
 * Everything is plain FP64 except the sample specification (receiver offset,
 * cosine-hemisphere direction, light point), which is defined as FP32
 * arithmetic so that the GPU can reproduce it bit for bit.
 *
 * Pixel arrays are row-major [H][W]; 3-vectors are interleaved [H][W][3].
 */
#ifndef OCR_ORACLE_H
#define OCR_ORACLE_H
#include <stdint.h>

#define ORC_MISS 0xFFFFFFFFu /* no occluder within the support */
#define ORC_SELF 0xFFFFFFFEu /* shadow sample below the tangent plane or receiver behind the light */

typedef struct {
    int32_t mode;       /* 0 ambient occlusion, 1 rectangular-light shadow (area definition),
                           2 rectangular-light shadow under the solid-angle definition,
                           3 direct illumination of a Lambertian receiver, in units of
                             rho L_e / pi (the visible irradiance of a unit-radiance light) */
    int32_t estimator;  /* 0 no reuse, 1 biased reuse, 2 unbiased reuse, 3 final-value filtering
                           (Filter (N) / Light (N)), 4 light-sample reuse re-traced (Light (NU), shadows) */
    int32_t pattern;    /* 0 sliding window of radius r, 1 fixed group of N pixels */
    int32_t radius;     /* window radius r */
    int32_t group_n;    /* group size N in {1,2,4,8} */
    int32_t dark_guard; /* biased shadow: all samples in the set blocked -> 0 */
    double ao_radius;   /* AO support radius R */
    float light[9];     /* centre, edge_u, edge_v (FP32 inputs) */
    uint64_t seed;
    uint32_t sample;    /* sample index s */
    int32_t light_pdf;  /* shadows, one light: 0 uniform emitter-area density, 1 bilinear density of
                           the receiver (corner weights 1 / |o - y_k|^3); estimators 0-2 */
    int32_t nlights;    /* shadows: number of rectangular lights (0 or 1: light[] only; up to 4) */
    float more_lights[3 * 9]; /* lights 1..nlights-1, as light[] */
} orc_params;

typedef struct orc_scene orc_scene;

orc_scene *orc_scene_create(const float *V, int64_t nv, const uint32_t *F, int64_t nt, int32_t use_grid);
void orc_scene_free(orc_scene *s);
int64_t orc_scene_grid_cells(const orc_scene *s);

/* Closest hit over t in (0, tmax] (inclusive) or (0, tmax) (exclusive). */
void orc_closest(const orc_scene *s, int64_t n, const double *o, const double *d, const double *tmax,
                 int32_t inclusive, const uint32_t *ign0, const uint32_t *ign1, uint32_t *tri, double *t,
                 uint8_t *graze);
/* Any hit over t in (0, tmax). */
void orc_any(const orc_scene *s, int64_t n, const double *o, const double *d, const double *tmax,
             const uint32_t *ign0, const uint32_t *ign1, uint8_t *blocked, uint8_t *graze);

/* FP32 sample specification for pixels of a region: origin o, direction
 * (AO: unit-ish omega; shadow: y - o) and kind (0 traced, 1 self-blocked /
 * unlit, 2 background). */
void orc_samples(int32_t W, int32_t H, const float *pos, const float *nrm, const uint32_t *prim,
                 const orc_params *p, int32_t x0, int32_t y0, int32_t x1, int32_t y1, float *o, float *dir,
                 uint8_t *kind);

/* First-hit records for pixels of a region (full-image arrays). */
void orc_records(const orc_scene *s, int32_t W, int32_t H, const float *pos, const float *nrm,
                 const uint32_t *prim, const orc_params *p, int32_t x0, int32_t y0, int32_t x1, int32_t y1,
                 uint32_t *hit, double *z, double *nz, uint8_t *graze);

/* Reuse estimate for the targets of a region.  Records must cover every
 * pixel of the targets' reuse sets.  nvar: 0 = not comparable (more than
 * three ambiguous threshold decisions, or a density on a grazing light
 * direction), else the number of admissible values written to var[8*i]. */
void orc_reuse(const orc_scene *s, int32_t W, int32_t H, const float *pos, const float *nrm,
               const uint32_t *prim, const orc_params *p, const uint32_t *hit, const double *z,
               const double *nz, const uint8_t *graze, int32_t x0, int32_t y0, int32_t x1, int32_t y1,
               double *value, uint8_t *nvar, double *var);

/* Area(A) p_A(y | x) of the bilinear emitter density of receiver point o at
 * light coordinates (a, b) of y. */
double orc_light_q(const double *o, const double *light, double a, double b);

/* Multi-sample accumulation over samples p->sample .. p->sample+M-1:
 * per-pixel sum and sum of squares of the per-sample estimates. */
void orc_render(const orc_scene *s, int32_t W, int32_t H, const float *pos, const float *nrm,
                const uint32_t *prim, const orc_params *p, int32_t M, int32_t x0, int32_t y0, int32_t x1,
                int32_t y1, double *sum, double *sumsq);

/* Induced densities of Eqs. (ao-pdf) and (shadow-pdf) without the
 * first-hit factor, exact normalisation (1/pi, 1/Area). */
double orc_density_ao(const double *o, const double *n, const double *z, const double *nz, double R);
double orc_density_shadow(const double *o, const double *n, const double *z, const double *nz,
                          const double *light);
/* Fraction of the light's area in front of the receiver's tangent plane. */
double orc_front_fraction(const double *o, const double *n, const double *light);
/* Solid angle of the whole one-sided light at o (out2[0]) and of its part in
 * front of the tangent plane (out2[1]); 0 behind the light. */
void orc_solid_angles(const double *o, const double *n, const double *light, double *out2);
/* C_Omega(o, z) of the solid-angle MIS estimator. */
double orc_sa_factor(const double *o, const double *n, const double *z, const double *light);
/* Irradiance of the unit-radiance light's part in front of the tangent plane
 * (the unshadowed direct-illumination term in units of rho L_e / pi). */
double orc_emitter_irradiance(const double *o, const double *n, const double *light);
/* C_DI(o, z) / (rho L_e / pi) of the direct-illumination MIS estimator. */
double orc_di_factor(const double *o, const double *n, const double *z, const double *light);
/* FP64 quadrature of the visible irradiance (direct illumination in units of rho L_e / pi). */
double orc_di_quadrature(const orc_scene *s, const double *o, const double *n, const double *light, uint32_t ign,
                         int32_t ngrid);

/* FP64 quadrature references of the AO integral (Eq. ao-hemisphere) and the
 * normalised shadow integral (Eq. shadow-area) at one receiver. */
double orc_ao_quadrature(const orc_scene *s, const double *o, const double *n, double R, uint32_t ign,
                         int32_t nstrata);
double orc_shadow_quadrature(const orc_scene *s, const double *o, const double *n, const double *light,
                             uint32_t ign, int32_t ngrid);
/* ... and of the solid-angle shadow (Eq. reapp-shadow-definition-solid-angle). */
double orc_shadow_sa_quadrature(const orc_scene *s, const double *o, const double *n, const double *light,
                                uint32_t ign, int32_t ngrid);

uint32_t orc_pcg4d_first(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t *out4);
int32_t orc_num_threads(void);
#endif
