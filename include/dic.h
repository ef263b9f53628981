/*
 * dic.h -- C ABI of the MI355X subset digital-image-correlation library.
 *
 * The library computes, for every point of interest (POI) of an image pair,
 *   1. the integer displacement that maximises the zero-normalised
 *      cross-correlation of Eq. (1) over a square search window (brute-force
 *      search, Sec. 2.1), and
 *   2. its sub-pixel refinement by inverse-compositional Gauss-Newton with a
 *      first-order (affine) shape function and bicubic interpolation of the
 *      deformed image (Sec. 2.2; Newton-Raphson, bilinear or cubic B-spline
 *      interpolation and a bicubic coefficient table by plan flags),
 * plus the adjoint of the ZNSSD criterion with respect to the warp parameters
 * and the deformed-image grey levels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Images   float32, row-major, pitch = width.  Pixel (r, c) has x = c, y = r
 *          and its grey level sits at that integer point (Sec. 2.2).  Images of
 *          all pairs live in two caller-owned device arenas, one for reference
 *          images and one for deformed images; each pair names its images by
 *          element offsets into them (the same arena may serve both).
 * POIs     int32 [N, 2] device array of integer centres (x, y), the POIs of
 *          pair k occupying rows [poi_offset, poi_offset + poi_count).
 * Subset   (2M+1) x (2M+1) pixels centred on the POI (Sec. 2.1), visited
 *          row-major; M = subset_radius.
 * Warp     p = (u, ux, uy, v, vx, vy) as float64 [N, 6]:
 *          x' = x0 + (1+ux) dx + uy dy + u,  y' = y0 + vx dx + (1+vy) dy + v.
 * Memory   The library never allocates device memory.  Every device buffer is
 *          allocated by the caller; the plan owns host metadata only (plus a
 *          captured HIP graph when DIC_FLAG_USE_GRAPH is set).
 * Streams  Every device-side call is asynchronous on the given stream
 *          (hipStream_t passed as void*, NULL = the default stream) and makes
 *          no allocation and no host synchronisation, so it can be captured.
 * Errors   Return codes only (dic_status_t); no exception crosses the ABI.
 *          dic_last_error() returns a thread-local message for the last
 *          failure.  Per-POI outcomes are reported through int32 status
 *          arrays using the DIC_POI_* codes.
 * Threads  A plan must not be used from two threads at the same time.
 */
#ifndef DIC_H_
#define DIC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dic_plan_s* dic_plan_t;
typedef void* dic_stream_t; /* a hipStream_t */

typedef enum {
  DIC_SUCCESS = 0,
  DIC_ERR_INVALID_ARGUMENT = -1,
  DIC_ERR_WORKSPACE_TOO_SMALL = -2,
  DIC_ERR_HIP = -3,
  DIC_ERR_UNSUPPORTED = -4,
  DIC_ERR_INTERNAL = -5,
  DIC_ERR_NOT_BOUND = -6
} dic_status_t;

/* Per-POI status codes. */
enum {
  DIC_POI_OK = 0,
  DIC_POI_NOT_CONVERGED = 1,      /* IC-GN hit max_iters; last p returned   */
  DIC_POI_OUT_OF_BOUNDS = 2,      /* a 4x4 interpolation neighbourhood left
                                     the image; last in-bounds p returned    */
  DIC_POI_ZERO_VARIANCE = 3,      /* flat reference (or deformed) subset    */
  DIC_POI_SINGULAR_HESSIAN = 4,   /* Cholesky pivot <= 1e-10 * diagonal     */
  DIC_POI_NO_VALID_CANDIDATE = 5, /* every search candidate inadmissible    */
  DIC_POI_NAN_INPUT = 6           /* NaN in the reference subset or in the
                                     interpolated deformed samples           */
};

typedef enum {
  DIC_FP32_BATCHED = 0, /* FP32 interpolation and correlation sums in short
                           per-lane blocks with a fixed reduction tree (no
                           Kahan compensation), FP64 for the sums that decide
                           means and statuses, bf16 matrix-core search
                           filter with an FP64 decision, LDS staging,
                           persistent batched launches; FP64 for the 6x6
                           factorisation/solve and warp composition         */
  DIC_FP64_PLAIN = 1    /* FP64 throughout, no staging, no compensation,
                           one launch per pair                               */
} dic_precision_t;

enum {
  DIC_FLAG_USE_GRAPH = 1u << 0,       /* dic_correlate captures and replays
                                         a HIP graph                         */
  DIC_FLAG_CACHE_REF_PREP = 1u << 1,  /* reuse the reference-side and
                                         deformed-side precomputations for
                                         the same image pointers until
                                         dic_plan_invalidate_reference()     */
  DIC_FLAG_DETERMINISTIC_BWD = 1u << 2, /* grad_def accumulated in a fixed
                                         order (no float atomics): 2^-40
                                         fixed-point integer sums per
                                         distinct deformed image, added to
                                         grad_def once.  Pairs must name
                                         the same deformed image (equal
                                         def_offset, width and height) or
                                         disjoint ones; dic_plan_create
                                         rejects partial overlaps with
                                         INVALID_ARGUMENT                    */
  DIC_FLAG_REFINE_NR = 1u << 3,       /* dic_correlate (and the autotuner)
                                         refine with Newton-Raphson instead
                                         of IC-GN                            */
  DIC_FLAG_INTERP_BILINEAR = 1u << 4, /* IC-GN and Newton-Raphson interpolate
                                         g bilinearly (Eq. (5), 2x2 taps,
                                         out of bounds when a 2x2
                                         neighbourhood leaves the image)
                                         instead of bicubically; FP32
                                         batched plans only; the ZNSSD
                                         adjoint rejects such plans         */
  DIC_FLAG_BICUBIC_LUT = 1u << 5,     /* IC-GN and Newton-Raphson evaluate
                                         the bicubic interpolant from a
                                         table of its 16 polynomial
                                         coefficients per pixel cell (the
                                         look-up tables of Sec. 2.2), built
                                         from each deformed image before the
                                         refinement (64 bytes per pixel of
                                         workspace), instead of from 4x4
                                         taps; same interpolant and bounds
                                         up to FP32 rounding.  FP32 batched
                                         plans only; exclusive with
                                         DIC_FLAG_INTERP_BILINEAR           */
  DIC_FLAG_INTERP_BSPLINE = 1u << 6   /* IC-GN and Newton-Raphson interpolate
                                         g with the cubic B-spline through
                                         its pixels (the spline
                                         interpolation of Sec. 2.2): the
                                         spline's coefficient image is
                                         computed from each deformed image
                                         before the refinement (mirror
                                         boundary, 8 bytes per pixel of
                                         workspace) and sampled with 4x4
                                         taps; same bounds as bicubic; an
                                         image with a non-finite pixel gives
                                         DIC_POI_NAN_INPUT at every POI the
                                         refinement reaches.  FP32 batched
                                         plans only; exclusive with
                                         DIC_FLAG_INTERP_BILINEAR and
                                         DIC_FLAG_BICUBIC_LUT; the ZNSSD
                                         adjoint rejects such plans         */
};

typedef struct {
  int32_t width;          /* pixels, >= 8                                     */
  int32_t height;         /* pixels, >= 8                                     */
  int32_t subset_radius;  /* M, 1 <= M <= 20                                  */
  int32_t search_radius;  /* S, 0 <= S <= 32                                  */
  int64_t ref_offset;     /* element offset of the reference image            */
  int64_t def_offset;     /* element offset of the deformed image             */
  int64_t poi_offset;     /* first POI row of this pair                       */
  int64_t poi_count;      /* number of POIs of this pair (may be 0)           */
} dic_pair_desc_t;

typedef struct {
  int32_t num_pairs;              /* >= 1                                     */
  const dic_pair_desc_t* pairs;   /* host array of num_pairs, copied          */
  int32_t precision;              /* dic_precision_t                          */
  int32_t max_iters;              /* IC-GN iteration cap, 1..200 (20)         */
  double conv_tol;                /* stop when |dp| < conv_tol, with
                                     |dp| = sqrt(du^2 + dv^2 + M^2 (dux^2 +
                                     duy^2 + dvx^2 + dvy^2)) (1e-3)           */
  uint32_t flags;                 /* DIC_FLAG_*                               */
} dic_plan_desc_t;

/* Tile and schedule choices; dic_plan_autotune() fills them by measurement.
 * Every choice gives bit-identical results. */
typedef struct {
  int32_t search_block;     /* integer-search form: 4 or 8 = vector-ALU form
                               with that many candidates per lane along du (a
                               workgroup has one lane per tile of the widest
                               window, at most 1024); 32 = matrix-core form
                               (bf16 filter, FP64 decision; radii up to 31,
                               2 x 2 candidate tiles beyond 16)             */
  int32_t search_occupancy; /* resident search workgroups per CU, 0 = as many
                               as registers and LDS allow, else 1..16        */
  int32_t icgn_waves;      /* waves (POIs in flight) per refinement workgroup
                              1..8 (IC-GN and Newton-Raphson)                 */
  int32_t icgn_slack;      /* extra pixels around the staged deformed patch,
                              0..16; kernels whose patch is sized for less
                              (subsets of 29 and 31 columns, and of 37 and
                              more) use at most 6.  It changes when a patch
                              is restaged, never the results                 */
} dic_tuning_t;

/* Validate a plan description and build the POI work list (host only, no
 * device call).  POIs of all pairs form one list ordered by decreasing
 * subset size so uneven pairs balance in one persistent launch (Sec. 2.3:
 * sub-images and whole pairs are independent).  Errors: INVALID_ARGUMENT for
 * null pointers or any field outside its stated range, overlapping or
 * non-contiguous POI ranges, or a POI count above 2^31 - 1. */
dic_status_t dic_plan_create(const dic_plan_desc_t* desc, dic_plan_t* out);

/* Bytes of device workspace the plan needs (gradients, per-POI reference
 * records, search templates, work list, counters). */
dic_status_t dic_plan_workspace_size(dic_plan_t plan, size_t* bytes);

/* Attach a caller-owned device workspace (>= dic_plan_workspace_size bytes,
 * 256-byte aligned) and upload the work list on `stream` (asynchronous).
 * Errors: WORKSPACE_TOO_SMALL, INVALID_ARGUMENT for a misaligned pointer,
 * HIP on a failed copy.  The workspace must outlive every later call. */
dic_status_t dic_plan_bind(dic_plan_t plan, void* workspace, size_t bytes,
                           dic_stream_t stream);

/* Read / override the tile and schedule choices (host only). */
dic_status_t dic_plan_get_tuning(dic_plan_t plan, dic_tuning_t* out);
dic_status_t dic_plan_set_tuning(dic_plan_t plan, const dic_tuning_t* in);

/* Time every tuning candidate on the given inputs and keep the fastest
 * (synchronises `stream`; must not be captured).  Choices are cached in the
 * JSON file named by the environment variable DIC_AUTOTUNE_CACHE when set.
 * The inputs are the same as dic_correlate's; outputs are scratch. */
dic_status_t dic_plan_autotune(dic_plan_t plan, const float* ref_images,
                               const float* def_images, const int32_t* poi_xy,
                               int32_t* uv_scratch, float* f_scratch,
                               int32_t* i_scratch, double* p_scratch,
                               dic_stream_t stream);

/* Mark the cached reference-side precomputation stale (host only). */
dic_status_t dic_plan_invalidate_reference(dic_plan_t plan);

/* Reference-side precomputation (Sec. 2.2: quantities IC-GN needs once per
 * subset): central-difference gradients of every reference image, and per
 * POI the subset mean and norm, steepest-descent sums, the Cholesky factor
 * of the Gauss-Newton Hessian and the search template.  Called implicitly by
 * the calls below unless DIC_FLAG_CACHE_REF_PREP holds a valid cache. */
dic_status_t dic_prepare_reference(dic_plan_t plan, const float* ref_images,
                                   const int32_t* poi_xy, dic_stream_t stream);

/* Deformed-side precomputation for the FP32 search: for every subset centre
 * of every deformed image, the exact (FP64) sums of g and g^2 over the
 * subset, so each candidate's normalisation is a lookup; with
 * DIC_FLAG_BICUBIC_LUT also the bicubic coefficient table, with
 * DIC_FLAG_INTERP_BSPLINE the B-spline coefficient image.  Called
 * implicitly by dic_integer_search / dic_correlate (the table by the
 * refinements) unless DIC_FLAG_CACHE_REF_PREP holds a valid cache for this
 * `def_images` pointer (then call it again, or dic_plan_invalidate_reference,
 * after changing the images in place).  A no-op for the FP64 plain form. */
dic_status_t dic_prepare_deformed(dic_plan_t plan, const float* def_images,
                                  dic_stream_t stream);

/* Brute-force integer search (Sec. 2.1, Eq. (1)).  For each POI evaluates
 * every candidate (du, dv) with |du - cu| <= S, |dv - cv| <= S, where (cu, cv)
 * is seed_uv[i] (int32 [N,2], nullable = (0,0)); a candidate whose subset
 * leaves the image or is flat (sum (g - gbar)^2 <= 1e-6 sum g^2) is skipped.
 * The winner is the smallest (dv, du), row-major, among candidates within
 * 1e-12 of the maximum coefficient.  The FP32 batched form first scores
 * every candidate approximately (bf16 matrix-core products with a rigorous
 * error bound for radii up to 31 and subsets up to 41 x 41, FP32 vector
 * sums otherwise), keeps every candidate whose bound still reaches the
 * maximum, and evaluates Eq. (1) for those in FP64 before the tie rule; the
 * winner and its FP64 coefficient (rounded to float) do not depend on the
 * form.  The FP64 plain form scores every candidate in FP64.
 * Outputs (device, length N): uv_out int32 [N,2] integer displacement,
 * zncc_out float [N] its coefficient, status_out int32 [N] DIC_POI_* (OK,
 * ZERO_VARIANCE, NO_VALID_CANDIDATE or NAN_INPUT; uv = (0,0) unless OK). */
dic_status_t dic_integer_search(dic_plan_t plan, const float* ref_images,
                                const float* def_images, const int32_t* poi_xy,
                                const int32_t* seed_uv, int32_t* uv_out,
                                float* zncc_out, int32_t* status_out,
                                dic_stream_t stream);

/* IC-GN sub-pixel refinement (Sec. 2.2).  Starts from p = (du, 0, 0, dv, 0, 0)
 * with (du, dv) = uv_init[i]; the gradient terms come from p_init (float64
 * [N,6], nullable) when given.  POIs whose status_in (nullable) is not OK are
 * skipped and keep that status.  Each iteration warps the subset, interpolates
 * the deformed image with Keys' cubic kernel (a = -1/2; bilinear, the
 * coefficient table or the cubic B-spline when a plan flag selects it), solves
 * H dp = -sum SD^T e with e = (f - fbar) - (df/dg)(g - gbar) and composes
 * W(p) <- W(p) W(dp)^-1; it stops when |dp| < conv_tol (OK) or after
 * max_iters (NOT_CONVERGED).  Outputs: p_out float64 [N,6], zncc_out float [N]
 * (Eq. (1) at the final p, NaN unless OK/NOT_CONVERGED), iters_out int32 [N],
 * status_out int32 [N]. */
dic_status_t dic_icgn_refine(dic_plan_t plan, const float* ref_images,
                             const float* def_images, const int32_t* poi_xy,
                             const int32_t* uv_init, const int32_t* status_in,
                             const double* p_init, double* p_out,
                             float* zncc_out, int32_t* iters_out,
                             int32_t* status_out, dic_stream_t stream);

/* Newton-Raphson sub-pixel refinement (Sec. 2.2: the alternative to IC-GN
 * whose quantities are recomputed at every iteration), on the ZNSSD
 * criterion with the first-order warp applied forward,
 * x_i = x0 + W(p) xi_i, and updated additively.  Each iteration interpolates
 * g and its gradient (Keys, a = -1/2, unless a plan flag selects bilinear,
 * the coefficient table or the B-spline) at the warped samples, forms
 * J_i = [gx, gx dx, gx dy, gy, gy dx, gy dy], Jc = J - mean(J), and takes
 *   dp = Hc^-1 sum Jc_i [(dg/df)(f_i - fbar) - ZNCC (g_i - gbar)],
 *   Hc = sum Jc_i^T Jc_i,
 * i.e. p <- p - H^-1 dC/dp with the exact gradient of ZNSSD and its
 * Gauss-Newton Hessian; a Cholesky pivot failure stops with
 * SINGULAR_HESSIAN (last p kept).  Arguments, outputs, stop rule and the
 * other statuses are those of dic_icgn_refine; the reference-side Hessian
 * of the plan's records is not used (a POI whose reference Hessian is
 * singular is refined). */
dic_status_t dic_nr_refine(dic_plan_t plan, const float* ref_images,
                           const float* def_images, const int32_t* poi_xy,
                           const int32_t* uv_init, const int32_t* status_in,
                           const double* p_init, double* p_out,
                           float* zncc_out, int32_t* iters_out,
                           int32_t* status_out, dic_stream_t stream);

/* Particle swarm integer search (Sec. 2.1, Eqs. 2-4) with the settings of
 * Sec. 5.2: 50 particles, at most 5 generations, stop once the swarm's best
 * coefficient reaches 0.995; acceleration coefficients c1 = c2 = 2 (not
 * given in the paper), inertia w(t) = 0.9 - t / 10 (Eq. 4).  With
 * modified = 1 every particle also evaluates the four neighbours of its
 * position and moves to the best of the five before the update (the
 * modified swarm with star search).  Positions and velocities are window
 * offsets from seed_uv[i] (nullable = (0,0)), initialised uniformly in
 * [-S, S]; a particle's coefficient is Eq. (1) at its rounded position
 * clipped to the window, candidates whose subset leaves the image, is not
 * finite or is flat having none; personal and swarm bests follow the
 * brute-force tie rule; velocities are clipped to [-S, S], positions to the
 * window.  swarm_random (device, float32 [N, 5, 50, 4], uniforms in [0, 1))
 * holds the swarm's random numbers: [i, 0, j] = (x, y of particle j's
 * position, x, y of its velocity) at initialisation, [i, t + 1, j] = (r1 for
 * x, r1 for y, r2 for x, r2 for y) of the update after generation t.  Each
 * coefficient is computed once per POI (a look-up table).  Outputs as
 * dic_integer_search (status NO_VALID_CANDIDATE when no evaluated position
 * had a coefficient), plus generations_out and evaluations_out (int32 [N],
 * nullable): generations run and distinct positions evaluated (at most 250,
 * or 1250 with modified = 1).  FP32 batched plans only (it reads the
 * deformed-side box sums); DIC_ERR_UNSUPPORTED otherwise. */
dic_status_t dic_pso_search(dic_plan_t plan, const float* ref_images,
                            const float* def_images, const int32_t* poi_xy,
                            const int32_t* seed_uv, const float* swarm_random,
                            int32_t modified, int32_t* uv_out, float* zncc_out,
                            int32_t* status_out, int32_t* generations_out,
                            int32_t* evaluations_out, dic_stream_t stream);

/* Search then refine in one call (the two entries above, in order; the
 * refinement is Newton-Raphson when the plan has DIC_FLAG_REFINE_NR).
 * zncc_int_out / status_int_out receive the search results (nullable).  With
 * DIC_FLAG_USE_GRAPH the enqueued work is captured once per distinct set of
 * pointers and replayed as a HIP graph afterwards. */
dic_status_t dic_correlate(dic_plan_t plan, const float* ref_images,
                           const float* def_images, const int32_t* poi_xy,
                           const int32_t* seed_uv, const double* p_init,
                           int32_t* uv_out, float* zncc_int_out,
                           int32_t* status_int_out, double* p_out,
                           float* zncc_out, int32_t* iters_out,
                           int32_t* status_out, dic_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search and refinement as dic_correlate, with the same arguments, outputs
 * and results, but the plan's workspace is a static device array of 64 MiB
 * inside the library (one per device, held until the process ends) instead of
 * a caller-bound one, so the plan need not be bound.  The call allocates
 * nothing: it uploads the plan's tables into the array, prepares both images
 * again (no cache), and runs every kernel in order on `stream` (no side
 * stream, no graph).  The plan's own binding, caches and graphs are left as
 * they were.  Errors: WORKSPACE_TOO_SMALL when dic_plan_workspace_size
 * exceeds 64 MiB (use dic_plan_bind and dic_correlate), INVALID_ARGUMENT for
 * a null required pointer, HIP when the array's address cannot be found.
 * Every call on one device shares its array and leaves its contents behind:
 * calls that overlap in time on one device (two streams, two threads) race
 * and must be ordered by the caller. */
dic_status_t dic_correlate_noalloc(dic_plan_t plan, const float* ref_images,
                                   const float* def_images, const int32_t* poi_xy,
                                   const int32_t* seed_uv, const double* p_init,
                                   int32_t* uv_out, float* zncc_int_out,
                                   int32_t* status_int_out, double* p_out,
                                   float* zncc_out, int32_t* iters_out,
                                   int32_t* status_out, dic_stream_t stream);

/* ZNSSD criterion and its adjoint.  For each POI with warp p (float64 [N,6],
 * forward-additive), C = sum_i (fhat_i - ghat_i)^2 with fhat = (f - fbar)/df
 * and ghat = (g - gbar)/dg, g interpolated at x0 + W(p) xi_i (= 2 - 2 ZNCC).
 * grad_c (float [N], nullable = ones) scales each POI's gradients.
 * Outputs (each nullable, skipped when NULL): c_out float [N];
 * grad_p float64 [N,6] = dC/dp (overwritten); grad_def float, same layout as
 * the deformed arena, receives += sum_i dC/dg_i w(tx) w(ty) at the 16 taps of
 * every sample.  POIs whose reference subset is flat, singular or NaN, or
 * whose samples leave the image, get C = NaN and zero gradients. */
dic_status_t dic_znssd_backward(dic_plan_t plan, const float* ref_images,
                                const float* def_images, const int32_t* poi_xy,
                                const double* p, const float* grad_c,
                                float* c_out, double* grad_p, float* grad_def,
                                dic_stream_t stream);

/* Sequence seeding: after a frame, for every POI whose status is OK copy its
 * p into p_seed (float64 [N,6]) and set seed_uv (int32 [N,2]) to
 * (rint(u), rint(v)); other POIs keep their previous seed (the last OK frame).
 * Pass p_seed as the next frame's p_init and seed_uv as its seed. */
dic_status_t dic_seed_update(dic_plan_t plan, const double* p, const int32_t* status,
                             int32_t* seed_uv, double* p_seed, dic_stream_t stream);

/* Host helper: POI grid x0 = m + k*step <= W-1-m (same for y), m = M+S+2,
 * row-major.  Writes min(count, capacity) rows of (x, y) into out_xy (host)
 * and the full count into *count. */
dic_status_t dic_poi_grid(int32_t width, int32_t height, int32_t subset_radius,
                          int32_t search_radius, int32_t step, int32_t* out_xy,
                          int64_t capacity, int64_t* count);

void dic_plan_destroy(dic_plan_t plan);
const char* dic_status_string(int32_t status);
const char* dic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DIC_H_ */
