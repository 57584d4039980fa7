/*
 * ocr.h -- C-ABI of the MI355X (gfx950) occlusion-point-reuse library.
 *
 * The library computes, per pixel of a G-buffer, radius-limited ambient
 * occlusion (Sec. 3.2, Eq. ao-hemisphere) or normalised rectangular-light
 * shadow visibility (Sec. 3.3, Eq. shadow-area) with one traced ray per
 * pixel and sample, and reuses neighbouring pixels' first-hit occluders
 * through the occluder-domain MIS estimators of Sec. 4 (Eqs.
 * ao-unbiased-estimator, ao-biased-estimator, shadow-estimator,
 * shadow-biased-estimator).
 *
 * Conventions common to every entry point:
 *   - Pointers marked "device" must be HIP device memory (hipMalloc or a
 *     torch CUDA tensor's data_ptr) on the current device; "host" pointers
 *     are ordinary host memory.  The caller owns every buffer it passes.
 *   - Per-frame calls only enqueue work on `stream` (a hipStream_t, NULL =
 *     the null stream).  They allocate nothing and never synchronise; the
 *     caller keeps buffers alive until the stream has passed the call.
 *   - Every call returns an ocr_status; on error the outputs are undefined
 *     and ocr_last_error() returns a thread-local description.  Nothing is
 *     thrown across the ABI.
 *   - Pixel arrays are row-major [height][width]; 3-vectors are interleaved
 *     float[height][width][3].  Row 0 is the top row.
 *   - Given the same inputs and seed every call produces bitwise identical
 *     outputs.
 */
#ifndef OCR_H
#define OCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ocr_status;
enum {
    OCR_OK = 0,
    OCR_ERR_INVALID_ARG = -1, /* a pointer, size or parameter is out of range */
    OCR_ERR_OOM = -2,         /* a library-owned allocation failed */
    OCR_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    OCR_ERR_UNSUPPORTED = -4, /* a valid request this build does not implement */
    OCR_ERR_BUDGET = -5,      /* a server request can never fit its memory budget */
    OCR_ERR_BUSY = -6         /* a server queue is full; retry later */
};

/* effect */
enum { OCR_AO = 0, OCR_SHADOW = 1 };
/* Effects a batched view or a served request can ask for besides OCR_AO and
 * OCR_SHADOW: shadows under the solid-angle definition
 * (ocr_reuse_shadow_solid_angle) and direct illumination
 * (ocr_reuse_direct_illumination); both trace shadow records.  The per-view
 * trace and validation entry points take OCR_AO and OCR_SHADOW only. */
enum { OCR_SHADOW_SOLID_ANGLE = 2, OCR_DIRECT_ILLUMINATION = 3 };
/* estimator: no reuse (Eqs. ao-mc-estimator / shadow-mc-estimator), biased
 * reuse (local first-hit consistency), unbiased reuse (first-hit validation) */
enum { OCR_NOREUSE = 0, OCR_BIASED = 1, OCR_UNBIASED = 2 };
/* reuse set S(i) of a target pixel i (Sec. 4.2, Eq. reuse-group):
 * OCR_WINDOW = the (2r+1)^2 pixels within Chebyshev distance r, clipped to
 * the image; OCR_GROUP = the fixed image-aligned group of N pixels holding i
 * (N = 1, 2, 4, 8 as 1x1, 2x1, 2x2, 4x2 tiles).  Background pixels are never
 * members. */
enum { OCR_WINDOW = 0, OCR_GROUP = 1 };

/* hit codes of an occluder record */
#define OCR_HIT_MISS 0xFFFFFFFFu /* no occluder within the support (or background pixel) */
#define OCR_HIT_SELF 0xFFFFFFFEu /* shadow sample behind the receiver's tangent plane, or
                                    receiver behind the light's emitting face: not traced */

/* Shading points (Sec. 3.1 notation: x and n_x per pixel).
 * pos, nrm: device float[h][w][3]; prim: device uint32[h][w], the triangle
 * index the pixel lies on, or 0xFFFFFFFF for background.  nrm is the unit
 * geometric normal facing the camera. */
typedef struct {
    const float *pos;
    const float *nrm;
    const uint32_t *prim;
    int32_t width, height;
} ocr_gbuffer;

/* Emitter-area sampling densities p_A(y | x) of a light (ocr_rect_light.pdf).
 *   OCR_LIGHT_UNIFORM:  1 / Area (Eq. shadow-light-pdf).
 *   OCR_LIGHT_BILINEAR: a general, receiver-dependent area density (App.,
 *     general area-domain sampling density): over the light coordinates
 *     (a, b) the bilinear interpolation of the corner weights 1 / |o - y_k|^3,
 *     the shape of the solid-angle density cos(theta_y) / |o - y|^2 at the
 *     corners, normalised to unit mass.  The occluder density becomes
 *     p_A(y' | x) J chi_A Occ and every estimator factor divides by
 *     Area p_A(y' | x).  Sampling is specified in FP32 (corner weights with
 *     |o - y_k|^2 clamped at 2^-40 and divided by their maximum; v = b + 1/2
 *     from its linear marginal with h[1], then u = a + 1/2 from the linear
 *     conditional with h[0], each by the inverse CDF
 *     t = xi (e0 + e1) / (e0 + sqrt((1 - xi) e0^2 + xi e1^2)), capped at 1).
 *     Taken by ocr_trace_occluders, ocr_sample_rays, ocr_validate_pairs (the
 *     validation does not depend on the density), ocr_reuse_shadow,
 *     ocr_reuse_shadow_solid_angle and ocr_reuse_direct_illumination; the
 *     other entry points that take lights return OCR_ERR_UNSUPPORTED for it. */
enum { OCR_LIGHT_UNIFORM = 0, OCR_LIGHT_BILINEAR = 1 };

/* One-sided rectangular emitter: the rectangle c + a e_u + b e_v,
 * |a|,|b| <= 1/2, emitting towards normalize(e_u x e_v).  e_u and e_v must be
 * orthogonal.  pdf: OCR_LIGHT_UNIFORM (0) or OCR_LIGHT_BILINEAR; other
 * values are OCR_ERR_INVALID_ARG. */
typedef struct {
    float center[3];
    float edge_u[3];
    float edge_v[3];
    int32_t pdf;
} ocr_rect_light;

/* First-hit occluder records (App. D / App. H, step 1), device buffers the
 * caller allocates:
 *   dz:  float[h][w][3]  hit point minus the ray origin o (o = x + eps n with
 *        eps = 2^-16 (1 + max_c |x_c|)), so z = o + dz;
 *   nz:  float[h][w][3]  unit geometric normal of the hit triangle, oriented
 *        towards the ray origin;
 *   hit: uint32[h][w]    index of the hit triangle in the scene's triangle
 *        array, or OCR_HIT_MISS / OCR_HIT_SELF.
 * dz and nz are written only where hit is a triangle index. */
typedef struct {
    float *dz;
    float *nz;
    uint32_t *hit;
} ocr_occluders;

/* Reuse configuration.
 *   pattern:    OCR_WINDOW or OCR_GROUP
 *   radius:     window radius r, 0..8 (OCR_WINDOW)
 *   group_n:    1, 2, 4 or 8 (OCR_GROUP)
 *   estimator:  OCR_NOREUSE, OCR_BIASED or OCR_UNBIASED
 *   dark_guard: biased shadows only: a target whose reuse set holds no
 *               unblocked sample gets 0 (Sec. 4.4)
 *   accumulate: 0 = write the estimate, 1 = add it to the output (sample
 *               accumulation; see ocr_scale)
 *   validated:  OCR_UNBIASED only: 1 = the workspace already holds this
 *               frame's validation bits (ocr_validate_pairs), 0 = the reuse
 *               call computes them first */
typedef struct {
    int32_t pattern;
    int32_t radius;
    int32_t group_n;
    int32_t estimator;
    int32_t dark_guard;
    int32_t accumulate;
    int32_t validated;
} ocr_reuse_params;

/* Library-owned acceleration structure over a triangle scene. */
typedef struct ocr_bvh ocr_bvh;

typedef struct {
    int64_t ntris;      /* triangles in the scene */
    int64_t nnodes;     /* 4-wide interior nodes */
    int32_t depth;      /* levels of 4-wide nodes */
    int32_t max_leaf;   /* largest leaf (triangles) */
    int64_t device_bytes;
    double build_ms;    /* host build time */
} ocr_bvh_info;

/* Build a 4-wide SAH bounding-volume hierarchy over a triangle scene and
 * upload it to the current device.  (The paper relies on a hardware
 * acceleration structure, Sec. 5; CDNA4 has no ray-tracing units, so the
 * library builds its own.)
 *   verts: host float[nverts][3]; tris: host uint32[ntris][3] vertex
 *   indices, each < nverts.  Triangle index t is its row in `tris`.
 *   stream: the upload is ordered on it and waited for before returning.
 * Synchronous.  Errors: OCR_ERR_INVALID_ARG (null pointers, nverts < 1,
 * ntris < 1 or >= 2^27, index out of range), OCR_ERR_OOM, OCR_ERR_HIP. */
ocr_status ocr_build_bvh(const float *verts, int64_t nverts, const uint32_t *tris, int64_t ntris,
                         void *stream, ocr_bvh **out);
ocr_status ocr_bvh_free(ocr_bvh *bvh);
ocr_status ocr_bvh_get_info(const ocr_bvh *bvh, ocr_bvh_info *info);

/* The hierarchy ocr_build_bvh uploads, built on the host only and copied to
 * caller memory for inspection (a structural check of the build); it makes
 * no HIP call, so it runs without a GPU.
 *   nodes: host buffer of node_capacity nodes of 128 bytes, or NULL to ask
 *     for the count only.  A node is float lo_x[4], hi_x[4], lo_y[4],
 *     hi_y[4], lo_z[4], hi_z[4] (the four child boxes), uint32 child[4],
 *     uint32 pad[4]; node 0 is the root.  child: 0xFFFFFFFF = empty slot;
 *     bit 31 clear = interior node index; bit 31 set = leaf of
 *     (bits 30..27) + 1 triangles starting at triangle (bits 26..0) of
 *     tri_data.
 *   tri_data: host float[3 * ntris][4] or NULL: the triangles in leaf order,
 *     three vertices each; the w word of the first vertex holds the
 *     triangle's row in `tris` (as uint32 bits).
 *   out_nnodes, out_depth: node count and depth (levels of nodes).
 * Errors: as ocr_build_bvh, and OCR_ERR_INVALID_ARG when nodes is given and
 * node_capacity is below the count (out_nnodes is set first). */
ocr_status ocr_build_bvh_host(const float *verts, int64_t nverts, const uint32_t *tris, int64_t ntris, void *nodes,
                              int64_t node_capacity, float *tri_data, int64_t *out_nnodes, int32_t *out_depth);

/* Step 1 of App. D (AO) / App. H (shadow): one sample per valid pixel with
 * the counter-based hash pcg4d(px, py, sample, seed32 + a*0x9E3779B9)
 * (Jarzynski and Olano, JCGT 2020; seed32 = low ^ high word of seed), then a
 * closest-hit trace:
 *   AO (mode OCR_AO): cosine-weighted direction (Eq. ao-direction-pdf, by
 *     Malley's method in the basis of Duff et al., JCGT 2017), ray
 *     t in (0, ao_radius];
 *   shadow (OCR_SHADOW): light point y from the light's emitter density
 *     (uniform, Eq. shadow-light-pdf, or bilinear: see OCR_LIGHT_BILINEAR),
 *     segment o -> y, t in (0, 1); not traced (OCR_HIT_SELF) when y is
 *     behind the receiver's tangent plane or the receiver is behind the
 *     light's emitting face.
 * The receiver's own triangle (prim) is never hit.  light is NULL for AO.
 * Errors: OCR_ERR_INVALID_ARG (null pointers, width or height < 1,
 * ao_radius not finite and > 0 for AO, degenerate or non-orthogonal light
 * edges for shadows), OCR_ERR_HIP. */
ocr_status ocr_trace_occluders(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, int32_t mode, float ao_radius,
                               const ocr_rect_light *light, uint64_t seed, uint32_t sample,
                               ocr_occluders *out, void *stream);

/* ocr_trace_occluders with the walks' work counted: the same records, and
 * adds the number of rays traced, BVH node visits, box tests (one per
 * non-empty child of a visited node), triangle tests and again the rays
 * traced to stats (device
 * uint64[5], caller-zeroed; the layout of ocr_validate_pairs' counts).  A
 * separate, slower kernel for work accounting (roofline figures), not for
 * frames.  Errors as ocr_trace_occluders, OCR_ERR_INVALID_ARG for a NULL
 * stats, and OCR_ERR_UNSUPPORTED for a light not sampled uniformly. */
ocr_status ocr_trace_occluders_counted(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, int32_t mode, float ao_radius,
                                       const ocr_rect_light *light, uint64_t seed, uint32_t sample,
                                       ocr_occluders *out, uint64_t *stats, void *stream);

/* The sample step alone (row A1 of the trace): for every pixel, the offset
 * receiver point o, the ray direction (AO: the cosine-weighted direction;
 * shadow: y - o for the light point y of the light's density) and its kind (0 traced,
 * 1 not traced -- shadow sample behind the tangent plane or receiver behind
 * the light, 2 background).  Bit-identical to what ocr_trace_occluders
 * traces.  origin, dir: device float[h][w][3]; kind: device uint8[h][w].
 * Errors as ocr_trace_occluders. */
ocr_status ocr_sample_rays(const ocr_gbuffer *gbuf, int32_t mode, const ocr_rect_light *light, uint64_t seed,
                           uint32_t sample, float *origin, float *dir, uint8_t *kind, void *stream);

/* Device workspace (bytes) ocr_reuse_ao / ocr_reuse_shadow need for a
 * w x h frame: the first-hit validation bits of the unbiased estimator
 * (one bit per receiver/candidate pair of a reuse set) and lists of the
 * candidate pixels (about 4 bytes per pixel); 0 for the
 * other estimators.  Returns 0 for invalid parameters. */
size_t ocr_workspace_bytes(int32_t width, int32_t height, const ocr_reuse_params *params);

/* First half of the unbiased estimators (Eq. occ-first-hit): for every
 * receiver k and candidate j of a common reuse set whose density at k is
 * positive, an any-hit segment from o_k towards z_j over t in (0, 1 - 1e-4),
 * ignoring z_j's triangle and k's own, decides whether z_j is the first hit
 * from x_k.  Writes one bit per pair into workspace (layout internal; size
 * from ocr_workspace_bytes with estimator OCR_UNBIASED).  mode, ao_radius and
 * light as for the trace.  stats: NULL, or device uint64[5] to which the
 * validation (window or groups) adds its useful work -- wave walks, node visits, the
 * box and triangle tests each segment needs on its own (a segment tests the
 * children of the nodes whose box it touches, and the triangles of the
 * leaves it reaches), and the segments traced.  With stats the validation runs a slower
 * work-accounting instantiation of the walk; the bits are the same.
 * Errors as ocr_reuse_ao. */
ocr_status ocr_validate_pairs(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ, int32_t mode,
                              float ao_radius, const ocr_rect_light *light, const ocr_reuse_params *params,
                              void *workspace, size_t workspace_bytes, uint64_t *stats, void *stream);

/* AO reuse (Sec. 4.3): out[i] = 1 - B_i with
 *   B_i = sum_{j in S(i), hit_j} [p(z_j|x_i) > 0 and P_i(j) > 0] p(z_j|x_i) / P_i(j),
 *   P_i(j) = sum_{k in S(i)} p(z_j|x_k),
 * p = p_AO of Eq. ao-pdf (biased: without the first-hit factor, Eq.
 * ao-biased-estimator; unbiased: with it, Eq. ao-unbiased-estimator, each
 * pair validated by an any-hit segment from x_k to z_j stopping 1e-4 short
 * of z_j).  OCR_NOREUSE gives out[i] = 1 - [hit_i].  Background pixels get 1.
 *   bvh: needed for OCR_UNBIASED (NULL allowed otherwise)
 *   occ: the records of ocr_trace_occluders(OCR_AO) for this G-buffer
 *   workspace: device, >= ocr_workspace_bytes() bytes (NULL if that is 0)
 *   out: device float[h][w]; raw, unclamped (Sec. 6).
 * Errors: OCR_ERR_INVALID_ARG, OCR_ERR_HIP. */
ocr_status ocr_reuse_ao(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ, float ao_radius,
                        const ocr_reuse_params *params, void *workspace, size_t workspace_bytes, float *out,
                        void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ocr_reuse_ao without the workspace argument.  The unbiased estimator's
 * validation bits and candidate lists live in a device array of the library
 * (64 MiB per device, held from the library's first use on that device until
 * the process ends); the call allocates nothing, and its results are those of
 * ocr_reuse_ao (the same kernels).
 *   Arguments, output and errors as ocr_reuse_ao, and OCR_ERR_INVALID_ARG
 *   when the frame needs more than 64 MiB of workspace (ocr_workspace_bytes;
 *   a 1920x1080 window of radius 3 needs 58 MB) or when params->validated is
 *   set (the validation runs within the call).
 * Every call on a device shares that device's array and leaves its contents
 * there: calls that overlap on one device (on different streams, or from
 * different threads) race; the caller orders them. */
ocr_status ocr_reuse_ao_noalloc(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                float ao_radius, const ocr_reuse_params *params, float *out, void *stream);

/* Shadow reuse (Sec. 4.4): out[i] = F_i - B_i with B_i as above for p_Sh of
 * Eq. shadow-pdf (Jacobian of Eq. shadow-jacobian at the light
 * re-intersection y'(x,z); support: y' on the rectangle beyond z, on the
 * emitting side, z in front of the receiver's tangent plane) and F_i the
 * exact fraction of the light in front of the receiver's tangent plane
 * (F_i = 1 for a receiver facing the whole light).  Biased with dark_guard:
 * 0 when no sample of S(i) is unblocked.  OCR_NOREUSE gives [hit_i is a
 * miss].  For a light sampled from the bilinear density the densities are
 * p_A(y' | x) J chi_A and each term p_i(j) / P_i(j) is divided by
 * Area p_A(y'_ij | x_i) (OCR_NOREUSE: F_i - 1 / (Area p_A) for a hit).
 * The records must be traced with the same light (density included).
 * Background pixels get 0.  Errors as ocr_reuse_ao. */
ocr_status ocr_reuse_shadow(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                            const ocr_rect_light *light, const ocr_reuse_params *params, void *workspace,
                            size_t workspace_bytes, float *out, void *stream);

/* Shadow reuse under the solid-angle definition (the appendix deriving the
 * occluder-domain form of Eq. reapp-shadow-definition-solid-angle): the
 * visible fraction of the solid angle Omega_A(x_i) that the light subtends,
 *   out[i] = F_Omega(x_i) - sum_j C_Omega(x_i, z_j) p_i(j) / P_i(j)
 * (Eq. reapp-shadow-solid-angle-estimator), with p, P, the validation and
 * the records exactly as for ocr_reuse_shadow (the light is still sampled
 * on its area: trace with OCR_SHADOW), the factor
 *   C_Omega(x, z) = Area / Omega_A(x) * <n_y', w_{y'->x}> / |x - y'|^2
 * for a uniformly sampled light, divided by Area p_A(y' | x) for one sampled
 * from the bilinear density (the density p_A(y' | x) J chi_A in p and P),
 * at the light crossing y' of the ray from x through z (Eq.
 * reapp-shadow-solid-angle-mis-factor), and F_Omega = Omega_front /
 * Omega_A, the part of the light's solid angle in front of the receiver's
 * tangent plane (1 for a receiver facing the whole light; solid angles
 * exact, by the formula of Van Oosterom and Strackee).  OCR_NOREUSE is the
 * N = 1 case: F_Omega - C_Omega(x_i, z_i) for a hit.  Biased with dark_guard:
 * 0 when no sample of S(i) is unblocked.  Background pixels and receivers
 * not on the light's emitting side get 0.  A single term is clamped below
 * 2^31 (reached only within ~1e-5 of the light).  Arguments, workspace and
 * errors as ocr_reuse_shadow. */
ocr_status ocr_reuse_shadow_solid_angle(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                        const ocr_rect_light *light, const ocr_reuse_params *params,
                                        void *workspace, size_t workspace_bytes, float *out, void *stream);

/* Shadows of several rectangular lights (up to 4).  The paper shows a
 * two-light result without giving its formulation; the quantity estimated
 * here is the visible fraction of the lights' total emitting area,
 *   sum_l (A_l / A_tot) Shadow_l(x_i),  A_l = |e_u x e_v| of light l.
 * ocr_trace_occluders_lights: as ocr_trace_occluders(OCR_SHADOW), except
 * that each sample first picks light l with probability A_l / A_tot (the
 * first l whose FP32 running sum A_0 + ... + A_l exceeds u2 A_tot, u2 the
 * third word of the sample's hash mapped as u0 and u1 are; the last light if
 * rounding leaves none), so that its point is uniform over the union of the
 * lights; one light gives exactly ocr_trace_occluders' samples and records.
 * ocr_reuse_shadow_lights: as ocr_reuse_shadow with the induced density of
 * an occluder summed over the lights (the area-weighted sum of the per-light
 * densities of Eq. shadow-pdf) and F_i the area-weighted front fraction.
 * lights: host array of nlights light descriptions (each checked as for one
 * light).  Errors as the single-light calls, and OCR_ERR_INVALID_ARG for a
 * NULL array or nlights outside [1, 4]. */
ocr_status ocr_trace_occluders_lights(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_rect_light *lights,
                                      int32_t nlights, uint64_t seed, uint32_t sample, ocr_occluders *out,
                                      void *stream);
ocr_status ocr_reuse_shadow_lights(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                   const ocr_rect_light *lights, int32_t nlights, const ocr_reuse_params *params,
                                   void *workspace, size_t workspace_bytes, float *out, void *stream);
/* ocr_validate_pairs for several lights (the pairs whose summed density is
 * positive); arguments, workspace, stats and errors as ocr_validate_pairs. */
ocr_status ocr_validate_pairs_lights(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                     const ocr_rect_light *lights, int32_t nlights, const ocr_reuse_params *params,
                                     void *workspace, size_t workspace_bytes, uint64_t *stats, void *stream);

/* Occluder-domain direct illumination (the appendix deriving Eq.
 * reapp-di-occluder-domain-compact) of a Lambertian receiver of albedo
 * `albedo` (rho) under the one-sided light emitting radiance `radiance`
 * (L_e) uniformly:
 *   out[i] = U(x_i) - sum_j C_DI(x_i, z_j) p_i(j) / P_i(j)
 * (Eq. reapp-di-general-mis-estimator) with p, P, the validation and the
 * records exactly as for ocr_reuse_shadow (trace with OCR_SHADOW: the light
 * is sampled on its area), C_DI(x, z) = Area g(x, y') for a uniformly sampled
 * light (g(x, y') / p_A(y' | x) for the bilinear density) and
 * g(x, y) = (rho / pi) L_e cos+(n_x, w_{x->y}) <n_y, w_{y->x}> / |x - y|^2
 * (Eq. reapp-di-general-mis-factor with p_A = 1 / Area), and U the unshadowed
 * term of Eq. reapp-di-unshadowed-term, computed exactly by Lambert's polygon
 * formula over the light clipped by the receiver's tangent plane.
 * OCR_NOREUSE is the N = 1 case: U - C_DI(x_i, z_i) for a hit.  Biased with
 * dark_guard: 0 when no sample of S(i) is unblocked.  Background pixels and
 * receivers not on the light's emitting side get 0.  Errors as
 * ocr_reuse_shadow, and OCR_ERR_INVALID_ARG for a negative or non-finite
 * radiance or albedo. */
ocr_status ocr_reuse_direct_illumination(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_occluders *occ,
                                         const ocr_rect_light *light, float radiance, float albedo,
                                         const ocr_reuse_params *params, void *workspace, size_t workspace_bytes,
                                         float *out, void *stream);

/* The paper's simple reuse baselines (Sec. 6), for quality comparisons.
 *
 * Final-value filtering (Filter (N) for AO; for shadows also Light (N),
 * light-sample reuse without visibility validation, which reduces to the same
 * average): out[i] = the mean of in[j] over the valid pixels j of S(i), the
 * window of radius params->radius or the group of params->group_n
 * (params->pattern; the estimator field is checked but unused); background
 * pixels keep in[i].  in: device float[h][w], typically the OCR_NOREUSE
 * estimate of ocr_reuse_ao / ocr_reuse_shadow; out: device float[h][w],
 * must not alias in (params->accumulate: out += the value).  Async on
 * `stream`.  Errors: OCR_ERR_INVALID_ARG (bad G-buffer or params, NULL or
 * aliased buffers), OCR_ERR_HIP. */
ocr_status ocr_filter_values(const ocr_gbuffer *gbuf, const ocr_reuse_params *params, const float *in, float *out,
                             void *stream);

/* Light-sample reuse with visibility re-evaluation (Light (NU), Sec. 6):
 * target i re-traces the light sample y_j (the sample of ocr_trace_occluders
 * with this seed and sample index) of every valid pixel j of S(i):
 *   out[i] = (1/|S(i)|) sum_j V(x_i, y_j),
 * unbiased because every y_j is uniform on the light.  V = 0 for a y_j behind
 * the tangent plane of x_i or an x_i behind the light (the sampler's FP32
 * tests), else 1 when the segment o_i -> y_j is free over t in (0, 1).  Costs
 * |S(i)| segments per pixel.  Background pixels get 0 (accumulate: += ).
 * Async on `stream`.  Errors: OCR_ERR_INVALID_ARG (NULL bvh or out, bad
 * G-buffer, params or light), OCR_ERR_HIP. */
ocr_status ocr_light_reuse_shadow(const ocr_bvh *bvh, const ocr_gbuffer *gbuf, const ocr_rect_light *light,
                                  uint64_t seed, uint32_t sample, const ocr_reuse_params *params, float *out,
                                  void *stream);

/* out[i] *= s for n floats (device); turns accumulated sums over M samples
 * into their mean (the final line of App. D / App. H). */
ocr_status ocr_scale(float *out, int64_t n, float s, void *stream);

/* ---------------------------------------------------------------------------
 * Batched schedule.  The paper runs one view per pass; a plan runs many views
 * of uneven size, over several scenes and mixed effects, as one persistent
 * trace launch and one persistent reuse launch over a (view, tile) work list,
 * recorded once into a HIP graph and replayed.  Each view's output is bitwise
 * identical to ocr_trace_occluders followed by the mode's per-view reuse entry
 * point (and, for OCR_UNBIASED, ocr_validate_pairs) with the same arguments: the schedule
 * changes only which lane or block computes a pixel, never its arithmetic.
 * ------------------------------------------------------------------------- */

/* One view of a plan.  All pointers are borrowed and must stay valid for the
 * plan's lifetime.
 *   bvh:       the view's scene
 *   gbuf:      device G-buffer (as for ocr_trace_occluders)
 *   mode:      OCR_AO, OCR_SHADOW, OCR_SHADOW_SOLID_ANGLE or
 *              OCR_DIRECT_ILLUMINATION (the last two trace shadow records)
 *   ao_radius, light, seed, sample: as for ocr_trace_occluders (light ignored
 *              for AO; uniformly sampled lights only, OCR_ERR_UNSUPPORTED
 *              for another density)
 *   params:    reuse configuration (accumulate and validated must be 0)
 *   out:       device float[h][w], the estimate (as for the per-view reuse
 *              entry point of the mode)
 *   radiance, albedo: direct illumination only (as
 *              ocr_reuse_direct_illumination) */
typedef struct {
    const ocr_bvh *bvh;
    ocr_gbuffer gbuf;
    int32_t mode;
    float ao_radius;
    ocr_rect_light light;
    uint64_t seed;
    uint32_t sample;
    ocr_reuse_params params;
    float *out;
    float radiance;
    float albedo;
} ocr_view_desc;

typedef struct ocr_plan ocr_plan;

/* Performance knobs of a plan (none changes a result).
 *   tile_w x tile_h: pixels one wavefront traces per work item (8x8, 16x8,
 *                    16x16, 32x8 or 32x16; tile_w*tile_h/64 rays per lane)
 *   packing:         order of a tile's pixels over lanes and passes:
 *                    0 row-major, 1 8x8 blocks, 2 Morton
 *   use_graph:       1 = record the schedule into a HIP graph on the first
 *                    launch and replay it; 0 = enqueue the kernels each time */
enum { OCR_PACK_ROW = 0, OCR_PACK_BLOCK8 = 1, OCR_PACK_MORTON = 2 };
typedef struct {
    int32_t tile_w, tile_h;
    int32_t packing;
    int32_t use_graph;
} ocr_plan_tuning;

typedef struct {
    int32_t nviews;
    int64_t pixels;           /* sum of w*h over views */
    int64_t trace_items;      /* (view, tile) work items of the trace launch */
    int64_t reuse_items;      /* (view, 16x16 tile) work items of the reuse launch */
    int64_t device_bytes;     /* records, workspaces and tables the plan owns */
    ocr_plan_tuning tuning;   /* the knobs in use */
    int32_t tuned;            /* 1 when the knobs came from the autotuner */
    int32_t candidates;       /* knob settings the autotuner timed */
    double tune_ms;           /* autotuner wall time */
    double best_trace_ms;     /* autotuner's time for the chosen trace knobs */
    int32_t from_cache;       /* 1 when an earlier plan of the same shape gave the knobs */
} ocr_plan_info;

/* Create a plan over `nviews` views (1..4096).  The plan allocates, once, the
 * occluder records of every view, the validation workspaces of OCR_UNBIASED
 * views and its work tables.  tuning: NULL = autotune (time every tile and
 * packing setting on these views with `stream` and keep the fastest; only
 * the plan's own records are written meanwhile), else use the given knobs.
 * An autotuned choice is kept for the process, keyed by the device
 * architecture and the view set's shape (each view's size, effect, reuse
 * parameters and scene size); a later plan of the same shape takes it
 * without timing (info.from_cache).  With the environment variable
 * OCR_TUNE_CACHE naming a file, choices are also read from and appended to
 * it, so they outlive the process.
 * Synchronous.  Errors: OCR_ERR_INVALID_ARG (any view argument that the
 * per-view calls would refuse, accumulate or validated set, bad knobs),
 * OCR_ERR_OOM, OCR_ERR_HIP. */
ocr_status ocr_plan_create(const ocr_view_desc *views, int32_t nviews, const ocr_plan_tuning *tuning, void *stream,
                           ocr_plan **out);
/* Enqueue one pass of every view on `stream`: reset the work queues, trace,
 * validate (OCR_UNBIASED views), reuse.  With use_graph the first call records
 * the graph (on a stream the plan owns) and every call replays it on
 * `stream`.  Allocates nothing after the first call.  Calls that overlap in
 * time on one plan race; one plan at a time per stream. */
ocr_status ocr_plan_launch(ocr_plan *plan, void *stream);
ocr_status ocr_plan_get_info(const ocr_plan *plan, ocr_plan_info *info);
/* The plan's occluder records of view v (device pointers the plan owns). */
ocr_status ocr_plan_get_records(const ocr_plan *plan, int32_t view, ocr_occluders *out);
/* Wait for the device, then free the plan's memory, graph and stream (freed
 * even when the wait fails; that failure is returned as OCR_ERR_HIP). */
ocr_status ocr_plan_free(ocr_plan *plan);

/* ---------------------------------------------------------------------------
 * Served loop: frame requests against resident scenes, admitted under an HBM
 * budget, run concurrently on a pool of stream slots (continuous batching:
 * a request is admitted as soon as a slot and memory are free, while others
 * are still on the device).  A request's result is bitwise identical to the
 * per-view calls with the same arguments, whatever else is in flight.
 * ------------------------------------------------------------------------- */
typedef struct ocr_server ocr_server;

/*   hbm_budget_bytes: device arena for per-request state (occluder records,
 *                     validation workspace, server-held outputs), allocated
 *                     once at creation (>= 4096)
 *   max_slots:        requests in flight at once (1..64), one stream each
 *   max_queue:        queued requests before submit returns OCR_ERR_BUSY
 *                     (0 = unbounded)
 *   poll_us:          completion polling interval of the worker (0 = 20)
 *   mock:             1 = no device work: each request "runs" for
 *                     mock_ns_per_pixel * w * h, for scheduler tests on a
 *                     machine without a GPU (no HIP call is made)
 *   fault_every:      fault injection for tests of failure handling: 0 = off;
 *                     k > 0 = every k-th admission finds its request's launch
 *                     failing with OCR_ERR_OOM after its memory was taken.
 *                     The request then completes with that status, holds no
 *                     arena memory and writes no output, and the server goes
 *                     on with the next one (the path any launch failure takes) */
typedef struct {
    size_t hbm_budget_bytes;
    int32_t max_slots;
    int32_t max_queue;
    int32_t poll_us;
    int32_t mock;
    double mock_ns_per_pixel;
    int32_t fault_every;
} ocr_server_options;

/* A frame request.  scene_id / view select a resident G-buffer.  mode:
 * OCR_AO, OCR_SHADOW, OCR_SHADOW_SOLID_ANGLE or OCR_DIRECT_ILLUMINATION (the
 * light may use either emitter density).  out: device float[h][w] to write, or
 * NULL to have the server keep the output in its arena (ocr_result.out) until
 * ocr_server_release.  arrival_ms: arrival time on the server clock
 * (ocr_server_now_ms), 0 = stamped at submission.  radiance, albedo: direct
 * illumination only (as ocr_reuse_direct_illumination). */
typedef struct {
    int32_t scene_id;
    int32_t view;
    int32_t mode;
    float ao_radius;
    ocr_rect_light light;
    uint64_t seed;
    uint32_t sample;
    ocr_reuse_params params;
    float *out;
    double arrival_ms;
    float radiance;
    float albedo;
} ocr_request;

typedef struct {
    uint64_t ticket;
    ocr_status status;
    int32_t width, height;
    float *out;          /* where the estimate is (device) */
    double arrival_ms;   /* server clock */
    double start_ms;     /* admitted and enqueued */
    double end_ms;       /* completion observed */
    double latency_ms;   /* end - arrival */
} ocr_result;

typedef struct {
    int64_t submitted, completed, refused, queued, in_flight;
    int64_t waited_for_memory;  /* admission attempts that found the head request too big for the free arena */
    int64_t peak_bytes, budget_bytes;
    int64_t max_in_flight;
    double p50_ms, p99_ms, mean_ms, max_ms;  /* arrival-to-completion latency of completed requests */
    double frames_per_s;                     /* completed / (last completion - first arrival) */
    int64_t failed;                          /* completed with an error status (counted in completed) */
} ocr_server_stats;

/* Create a server on the current device (mock: no device).  Starts one worker
 * thread.  Errors: OCR_ERR_INVALID_ARG, OCR_ERR_OOM (arena), OCR_ERR_HIP. */
ocr_status ocr_server_create(const ocr_server_options *opt, ocr_server **out);
/* Register a resident scene: its BVH and a pool of G-buffers (copied
 * descriptors; the device arrays are borrowed for the server's lifetime). */
ocr_status ocr_server_add_scene(ocr_server *s, const ocr_bvh *bvh, const ocr_gbuffer *views, int32_t nviews,
                                int32_t *scene_id);
/* Queue a request (first in, first out).  The server's streams do not wait
 * for other streams: the G-buffer and a caller-given output must be ready
 * (their producers finished) when the request is submitted.  Errors:
 * OCR_ERR_INVALID_ARG (as the per-view calls), OCR_ERR_BUDGET (its state can
 * never fit the arena), OCR_ERR_BUSY (queue full, or server stopping). */
ocr_status ocr_server_submit(ocr_server *s, const ocr_request *req, uint64_t *ticket);
/* Move up to `max` completed results to `out` (host), completion order. */
ocr_status ocr_server_poll(ocr_server *s, ocr_result *out, int32_t max, int32_t *n);
/* Give back a server-held output (request submitted with out == NULL). */
ocr_status ocr_server_release(ocr_server *s, uint64_t ticket);
/* Block until nothing is queued or in flight. */
ocr_status ocr_server_drain(ocr_server *s);
ocr_status ocr_server_get_stats(ocr_server *s, ocr_server_stats *st);
/* Milliseconds on the server clock (steady, shared by all servers). */
double ocr_server_now_ms(void);
/* Drain, stop the worker and free the arena and streams. */
ocr_status ocr_server_destroy(ocr_server *s);

/* Thread-local description of the last error on this thread ("" if none). */
const char *ocr_last_error(void);

/* Library version string. */
const char *ocr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OCR_H */
