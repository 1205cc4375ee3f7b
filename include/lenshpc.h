/*
 * lenshpc.h -- C ABI of the MI355X (gfx950) lens-gradient library.
 *
 * The library computes the data-parallel hot path of Lenstool-HPC
 * (Schaefer, Fourestey & Kneib, arXiv:2004.06352):
 *   - the deflection map alpha = grad psi, summed over every parametric
 *     potential at every grid point (Sec. 4.1, Eq. (10));
 *   - the second derivatives psi_xx, psi_xy, psi_yy at every grid point, the
 *     input of the kappa, gamma and mu maps (Sec. 2.4, Eqs. (7)-(9));
 *   - the chi^2 of many model samples, in the source plane (unlens, take the
 *     barycentre, Sec. 2.2, Fig. 3, Eq. (6)) or in the image plane by
 *     brute-force inversion of a triangulated grid (Sec. 2.3, Fig. 4;
 *     Sec. 4.2, Fig. 7).
 *
 * Mass model.  Every potential is a dPIE (Eliasdottir et al. 2007, the
 * reference the paper gives for its sub-halo parameters, Sec. 2.2): the
 * difference of two cored isothermal ellipsoids with core radius rcore and cut
 * radius rcut, convergence
 *     kappa = (b0/2) F [1/sqrt(rcore^2 + rho^2) - 1/sqrt(rcut^2 + rho^2)],
 *     F = rcut/(rcut - rcore),  rho^2 = x'^2/(1+eps)^2 + y'^2/(1-eps)^2,
 * in the frame (x', y') rotated by the position angle phi.  rcut = +inf gives
 * the cored isothermal ellipsoid; eps = 0, rcore = 0, rcut = +inf gives the
 * singular isothermal sphere, whose deflection has modulus b0 everywhere.
 * A potential with rcore = 0 contributes exactly zero at its own centre.
 *
 * Units: positions and radii in arcsec, angles in radians (counter-clockwise
 * from +x), b0 in arcsec at Dls/Ds = 1.  Deflections come out in arcsec,
 * second derivatives dimensionless; every map is multiplied by the Dls/Ds
 * (`dlsds`) passed with it.
 *
 * Layout.  Tables are structures of arrays: one array per parameter, entry k
 * of each array describes potential k.  Maps are row-major planes [ny][nx],
 * one plane per channel; grid point (i, j) is (x0 + i dx, y0 + j dy) and sits
 * at index j*nx + i.
 *
 * Memory.  Unless stated otherwise every array pointer is a DEVICE pointer on
 * the context's device, owned by the caller, and must stay valid until the
 * stream has passed the call.  The library owns only its context scratch
 * (derived tables, cached deflections, image slots, work queues), allocated on
 * demand up to the context's scratch limit and freed by lens_ctx_destroy.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Compute calls
 * are asynchronous on it, except that a context created with
 * LENS_CTX_CHECK_TABLES validates device-resident table contents before
 * launching and therefore synchronises `stream` once per call.
 *
 * Errors.  Functions return LENS_OK (0) or a negative status; a thread-local
 * message is available from lens_last_error().  An argument error is detected
 * before anything is launched and leaves every output untouched.  Device-side
 * content errors (a potential with eps outside [0, 1), rcore < 0,
 * rcore >= rcut, b0 < 0 or a NaN) are reported synchronously as LENS_EINVAL in
 * checked contexts; in unchecked contexts the affected outputs become NaN and
 * lens_ctx_status() reports LENS_EINVAL after the stream has passed the call.
 * Faults of the device runtime surface as LENS_EDEVICE.
 *
 * Threads.  A context may be used by one host thread at a time; several
 * contexts may share a device.  A context's scratch is reused by every call
 * on it, so calls on one context must not overlap on the device: give each
 * concurrently used stream its own context.
 *
 * Bounds.  Before launching, every device array argument is checked against
 * the allocation it lies in (hipMemGetAddressRange): an array that does not
 * fit is LENS_EINVAL.  Offsets read by kernels are clamped to the declared
 * sizes, so inconsistent offset contents cannot address outside the arrays.
 */
#ifndef LENSHPC_H
#define LENSHPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LENSHPC_ABI_VERSION 2

typedef int32_t lens_status_t;
#define LENS_OK 0
#define LENS_EINVAL (-1)       /* invalid argument or table content */
#define LENS_ENOMEM (-2)       /* device memory or the scratch limit exhausted */
#define LENS_EDEVICE (-3)      /* HIP runtime error or device fault */
#define LENS_EOVERFLOW (-4)    /* image slots overflowed (counts stay exact) */
#define LENS_EUNSUPPORTED (-5) /* valid request this build does not provide */

/* Evaluation precision of the map and chi^2 kernels.
 *   LENS_FP64        every step in FP64; FP64 outputs.
 *   LENS_FP32_ACC64  pixel offsets and rotation in FP64, each potential's
 *                    terms in FP32, the sum over potentials in FP64; maps are
 *                    stored as FP32, chi^2 as FP64.
 *   LENS_FP32_COMP32 as LENS_FP32_ACC64 but the sum over potentials is a
 *                    compensated (Neumaier) FP32 sum. */
typedef int32_t lens_precision_t;
#define LENS_FP64 0
#define LENS_FP32_ACC64 1
#define LENS_FP32_COMP32 2

typedef int32_t lens_chi2_mode_t;
#define LENS_CHI2_SOURCE 0 /* source-plane: scatter of unlensed images (Sec. 2.2) */
#define LENS_CHI2_IMAGE 1  /* image-plane: grid inversion + assignment (Sec. 2.3, 4.2) */

/* How lens_chi2_batch issues its work (the result does not depend on it).
 *   LENS_CHI2_PATH_PER_SAMPLE  one kernel launch per sample (reference path)
 *   LENS_CHI2_PATH_BATCHED     persistent kernels pulling samples from a
 *                              device work queue, a few launches per batch */
typedef int32_t lens_chi2_path_t;
#define LENS_CHI2_PATH_BATCHED 0
#define LENS_CHI2_PATH_PER_SAMPLE 1

/* Context flags */
#define LENS_CTX_CHECK_TABLES 1u /* validate table contents before each launch */

typedef struct lens_ctx lens_ctx_t;        /* opaque */
typedef struct lens_chi2_plan lens_chi2_plan_t; /* opaque */
typedef struct lens_mcmc lens_mcmc_t;           /* opaque */

/* Potential table in amplitude form; n entries; device arrays. */
typedef struct {
    int32_t n;
    const double *x0, *y0; /* centre [arcsec] */
    const double *b0;      /* amplitude at Dls/Ds = 1 [arcsec], >= 0 */
    const double *eps;     /* Kassiola-Kovner ellipticity (a-b)/(a+b), 0 <= eps < 1 */
    const double *phi;     /* position angle [rad] */
    const double *rcore;   /* core radius [arcsec], >= 0 */
    const double *rcut;    /* cut radius [arcsec], > rcore, may be +inf */
} lens_pot_table_t;

/* Potential table in physical form (Sec. 2.2: centre, velocity dispersion,
 * ellipticity, orientation, profile radii); n entries; device arrays. */
typedef struct {
    int32_t n;
    const double *x0, *y0; /* centre [arcsec] */
    const double *sigma;   /* velocity dispersion [km/s], >= 0 */
    const double *e;       /* ellipticity (a^2-b^2)/(a^2+b^2), 0 <= e < 1 */
    const double *phi;     /* position angle [rad] */
    const double *rcore, *rcut; /* [arcsec] */
} lens_phys_table_t;

/* Rectangular image-plane grid (Sec. 2.4: one point per image pixel). */
typedef struct {
    int32_t nx, ny;   /* >= 1 each */
    double x0, y0;    /* coordinates of point (0, 0) [arcsec] */
    double dx, dy;    /* spacing [arcsec], > 0 */
} lens_grid_t;

/* A batch of model samples for chi^2 (one MCMC proposal per sample).  Model
 * m is the fixed table followed by free entries free_offset[m] ..
 * free_offset[m+1]-1, summed in that order.  Samples may differ in size. */
typedef struct {
    int32_t n_samples;          /* >= 0 */
    const int32_t *free_offset; /* device [n_samples+1], non-decreasing, [0] = 0 */
    lens_pot_table_t free;      /* concatenated free potentials of all samples */
    lens_pot_table_t fixed;     /* shared by every sample (n may be 0) */
} lens_model_batch_t;

/* Constraint catalogue (Eq. (6)): n_sys multiple-image systems; images of
 * system i are img_offset[i] .. img_offset[i+1]-1. */
typedef struct {
    int32_t n_sys;             /* >= 1 */
    int32_t n_img;             /* total images = img_offset[n_sys], 1..4000 */
    const int32_t *img_offset; /* device [n_sys+1], non-decreasing, [0] = 0 */
    const double *x, *y;       /* observed positions c_ij [arcsec] */
    const double *sigma;       /* position error sigma_ij [arcsec], > 0 */
    const double *dlsds;       /* Dls/Ds of each system's source, (0, 1] */
} lens_catalog_t;

typedef struct {
    lens_chi2_mode_t mode;
    lens_precision_t prec;     /* evaluation precision of the deflections */
    lens_chi2_path_t path;
    lens_grid_t grid;          /* image mode: the triangulated grid */
    int32_t max_img_per_sys;   /* image mode: stored images per (sample, system), 1..64 */
    double missing_penalty;    /* image mode: added per constraint left without an image */
    int32_t refine_max_iter;   /* image mode: Newton iterations per found image, 0..64
                                  (0: positions stay the grid estimates) */
    double refine_tol;         /* image mode, refine_max_iter > 0: stop when a Newton step
                                  is shorter than this [arcsec], > 0 */
} lens_chi2_opts_t;

/* Launch configuration of the map kernel (chosen by the autotuner).
 * block_x * block_y threads per block (block_x a multiple of 64, product
 * <= 256), each thread evaluating pix_per_thread points along x;
 * stage = 1 stages the derived potential constants in LDS in chunks of
 * lds_chunk potentials, stage = 0 reads them with wave-uniform loads. */
typedef struct {
    int32_t block_x, block_y, pix_per_thread, stage, lds_chunk;
} lens_map_tuning_t;

/* ---- context ---------------------------------------------------------- */
lens_status_t lens_ctx_create(int32_t device, uint64_t scratch_bytes_max, uint32_t flags,
                              lens_ctx_t **out);
lens_status_t lens_ctx_destroy(lens_ctx_t *ctx);
/* Sticky device-side status of unchecked contexts; synchronises the device. */
lens_status_t lens_ctx_status(lens_ctx_t *ctx);
/* Set (tuning != NULL) or reset to the built-in default (NULL) the map
 * kernel's launch configuration for one precision. */
lens_status_t lens_set_map_tuning(lens_ctx_t *ctx, lens_precision_t prec,
                                  const lens_map_tuning_t *tuning);
lens_status_t lens_get_map_tuning(lens_ctx_t *ctx, lens_precision_t prec,
                                  lens_map_tuning_t *out);
/* Number of persistent one-wave blocks per compute unit that the batched
 * source-plane chi^2 launches (1..64, default 16; each wave evaluates whole
 * samples).  Does not change any result. */
lens_status_t lens_set_chi2_tuning(lens_ctx_t *ctx, int32_t waves_per_cu);
lens_status_t lens_get_chi2_tuning(lens_ctx_t *ctx, int32_t *waves_per_cu);

/* ---- parameter prologue ------------------------------------------------- */
/* Physical -> amplitude form on the device (Sec. 2.2 parameters):
 *   b0  = K pi (sigma/c)^2 rad in arcsec, K = 6 (convention 0, the Lenstool
 *         dPIE convention) or 4 (convention 1, singular isothermal sphere);
 *   eps = (1 - sqrt(1 - e^2))/e (eps = 0 at e = 0).
 * out_b0 and out_eps are device arrays of phys->n doubles; the other fields of
 * the amplitude table are the physical table's own arrays. */
lens_status_t lens_table_from_physical(lens_ctx_t *ctx, const lens_phys_table_t *phys,
                                       int32_t convention, double *out_b0, double *out_eps,
                                       void *stream);

/* ---- maps (Sec. 4.1 Eq. (10); Sec. 2.4 Eqs. (7)-(9)) ---------------------- */
/* Deflection map: ax, ay = dlsds * sum_k grad psi_k at every grid point.
 * Outputs: nx*ny doubles each for LENS_FP64, floats otherwise. */
lens_status_t lens_grad_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                            const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                            void *ax, void *ay, void *stream);

/* Second-derivative map: hxx, hxy, hyy = dlsds * sum_k d^2 psi_k, computed in
 * one pass with the deflection, which is stored too when ax and ay are both
 * non-NULL.  Element type as for lens_grad_map. */
lens_status_t lens_hessian_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                               const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                               void *hxx, void *hxy, void *hyy, void *ax, void *ay,
                               void *stream);

/* lens_hessian_map without device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Arguments, results and errors are those of
 * lens_hessian_map; the context's scratch is neither used nor grown.  The
 * potentials' derived constants go instead to a fixed array of device memory
 * that the library holds on each device from load to process exit
 * (LENS_NOALLOC_MAX_POT potentials, 356 bytes each: 2.8 MiB per device).
 *   - A table of more than LENS_NOALLOC_MAX_POT potentials is LENS_ENOMEM,
 *     detected before anything is launched.
 *   - Every call on one device uses that device's one array, whatever the
 *     context or stream: calls that overlap on a device race and must be
 *     ordered by the caller (one stream, or events between streams).  The
 *     array is fully rewritten by each call before it is read.
 *   - The call itself allocates nothing (checked contexts still synchronise
 *     `stream` once, as lens_hessian_map does). */
#define LENS_NOALLOC_MAX_POT 8192
lens_status_t lens_hessian_map_noalloc(lens_ctx_t *ctx, const lens_pot_table_t *table,
                                       const lens_grid_t *grid, double dlsds,
                                       lens_precision_t prec, void *hxx, void *hxy, void *hyy,
                                       void *ax, void *ay, void *stream);

/* Lensing potential psi = dlsds * sum_k psi_k (alpha = grad psi, Sec. 2.1;
 * one of the lensing maps of Sec. 2.4), FP64 only (psi must be nx*ny
 * doubles; other precisions return LENS_EUNSUPPORTED).  Each cored isothermal
 * ellipsoid contributes Keeton's (2001) softened-isothermal-ellipsoid
 * potential under the mapping of the deflection,
 *   P_w = x' a'x + y' a'y - b0 (1 - eps^2) w ln sqrt((psi_w + S_w)^2 + k^2 x'^2)
 * (circular: b0 [psi_w - w - w ln(psi_w + w)]), a dPIE F (P_a - P_s): the
 * potential is defined up to an additive constant, fixed by this form. */
lens_status_t lens_potential_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                                 const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                                 double *psi, void *stream);

/* Time-delay (Fermat) surface of a source at (beta_x, beta_y) [arcsec]:
 *   t = scale (|theta - beta|^2 / 2 - dlsds * sum_k psi_k)
 * at every grid point (nx*ny doubles); its stationary points are the images
 * and differences of t between images are their arrival-time differences.
 * scale converts arcsec^2 to time, e.g. lens_time_delay_scale's days. */
lens_status_t lens_time_delay_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                                  const lens_grid_t *grid, double dlsds, double beta_x,
                                  double beta_y, double scale, double *t, void *stream);

/* Derived maps (Sec. 2.4, Eqs. (7)-(9), with the inverse magnification matrix
 * of Sec. 2.1, A^-1 = [[1 - kappa - gamma1, -gamma2], [-gamma2, 1 - kappa +
 * gamma1]]), from H = dlsds * sum_k d^2 psi_k at every grid point:
 *   kappa  = (Hxx + Hyy)/2             convergence
 *   gamma1 = (Hxx - Hyy)/2, gamma2 = Hxy, gamma = sqrt(gamma1^2 + gamma2^2)
 *   det    = (1 - kappa)^2 - gamma^2   det A^-1 (zero on the critical lines)
 *   mu     = 1/det                     magnification (infinite where det = 0)
 * The paper prints gamma^2 with the off-diagonal term inside the quarter and
 * mu with (1 - kappa)^2 + gamma^2; the forms above are the ones its Sec. 2.1
 * matrix gives.  Computed in one pass with the second derivatives, which are
 * not stored.  Any output may be NULL (at least one is required); element
 * type as for lens_grad_map (the derived values are formed in FP64 from the
 * accumulated sums and rounded once). */
lens_status_t lens_derived_map(lens_ctx_t *ctx, const lens_pot_table_t *table,
                               const lens_grid_t *grid, double dlsds, lens_precision_t prec,
                               void *kappa, void *gamma1, void *gamma2, void *gamma, void *mu,
                               void *det, void *stream);

/* ---- chi^2 of a batch of samples (Sec. 2.2 Eq. (6); Sec. 2.3; Sec. 4.2) --- */
/* chi2[m] for every sample m (device, n_samples doubles).
 * Source mode: chi2 = sum_i sum_j |beta_ij - mean_j beta_ij|^2 / sigma_ij^2,
 *   beta_ij = theta_ij - dlsds_i alpha(theta_ij).
 * Image mode: per sample, sources = those barycentres; every grid cell (i, j)
 *   is split into T0 = (v[i,j], v[i+1,j], v[i,j+1]) and
 *   T1 = (v[i+1,j+1], v[i,j+1], v[i+1,j]) (ids 2(j(nx-1)+i) and +1); each
 *   vertex is unlensed as u = v - dlsds_i alpha(v); a source found inside a
 *   triangle (exact orientation tests, ties broken by the perturbation
 *   p + (d, d^2)) gives an image at the barycentric interpolation of the
 *   triangle's image-plane vertices.  Each image is assigned to its nearest
 *   constraint (ties: lower index); each constraint keeps its nearest assigned
 *   image (ties: lower triangle id) and adds |c - x|^2/sigma^2, or
 *   missing_penalty when it has none.
 *   nimg (device [n_samples*n_sys] int32, or NULL): exact number of images;
 *   nmissing (device [n_samples] int32, or NULL): constraints without image;
 *   img_xy (device [n_samples*n_sys*max_img_per_sys*2] doubles, or NULL):
 *   stored image positions in increasing triangle id, unused slots NaN.
 *   Returns LENS_EOVERFLOW (after completing the stream, counts exact) when a
 *   (sample, system) had more images than max_img_per_sys.
 *   Image mode synchronises `stream` once at the end to report overflow and
 *   the search's own checks (below).
 * Domain of the image search (image mode and lens_find_images): a source's
 * Dls/Ds must lie in (0, 1] (the tile cull assumes f > 0); the exact
 * orientation tests are exact for finite coordinates (unlensed vertices and
 * sources) whose nonzero magnitudes lie in [2^-400, 2^400].  Both are checked
 * on the device while the search runs; a violation returns LENS_EINVAL after
 * the stream completes (outputs written, not meaningful). */
lens_status_t lens_chi2_batch(lens_ctx_t *ctx, const lens_model_batch_t *batch,
                              const lens_catalog_t *cat, const lens_chi2_opts_t *opts,
                              double *chi2, int32_t *nimg, int32_t *nmissing, double *img_xy,
                              void *stream);

/* Image search alone (stage 3 of Sec. 4.2) for a given deflection grid:
 * ax, ay (device, nx*ny doubles, Dls/Ds = 1) are the total deflection at the
 * grid vertices; source s sits at (src_x[s], src_y[s]) with Dls/Ds f[s]
 * (device arrays of n_src).  Outputs per source, images in increasing
 * triangle id: nimg[s] (exact count), img_tri/img_x/img_y[s*kmax + k]
 * (k < min(nimg[s], kmax); unused slots -1 / NaN).  Returns LENS_EOVERFLOW
 * when a count exceeded kmax (synchronises `stream`), LENS_EINVAL for an f[s]
 * outside (0, 1] or coordinates outside the exact domain (see above; that
 * source gets no images, the others are searched). */
lens_status_t lens_find_images(lens_ctx_t *ctx, const double *ax, const double *ay,
                               const lens_grid_t *grid, int32_t n_src, const double *src_x,
                               const double *src_y, const double *f, int32_t kmax,
                               int32_t *nimg, int64_t *img_tri, double *img_x, double *img_y,
                               void *stream);

/* ---- captured batches (batching form) ------------------------------------ */
/* Record the whole of one lens_chi2_batch call (batched path), bound to these
 * exact buffers and shapes; replaying it re-evaluates the batch with whatever
 * the buffers then hold.  An image-mode plan replays a HIP graph of its
 * sequence; a source-mode plan, one or two kernels, replays their recorded
 * launch descriptions as plain launches (no argument checks, no scratch
 * carving, no graph launch).  lens_chi2_plan_create and
 * _create_ex record source-mode calls (other modes: LENS_EUNSUPPORTED);
 * lens_chi2_plan_create2 records either mode, with the image mode's optional
 * outputs.  The plan owns its scratch (device memory allocated here, freed
 * by lens_chi2_plan_destroy), so other calls on the context do not disturb
 * it; it uses the context's device and, in checked contexts, validates the
 * tables once at creation, so destroy plans before their context.  Creating
 * a plan synchronises `stream`. */
lens_status_t lens_chi2_plan_create(lens_ctx_t *ctx, const lens_model_batch_t *batch,
                                    const lens_catalog_t *cat, const lens_chi2_opts_t *opts,
                                    double *chi2, void *stream, lens_chi2_plan_t **out);

/* Plan flags.
 *   LENS_PLAN_FIXED_RESIDENT  the fixed potentials and the catalogue are read
 *     once, when the plan is created: their per-image constants (the fixed
 *     potentials' deflection at every constraint, each image's Dls/Ds) are
 *     computed then and kept in the plan, and a launch evaluates only the
 *     free potentials (the case of a sampler, where only the free parameters
 *     change between evaluations).  The fixed table and catalogue buffers must
 *     not change while the plan is used; results are bit-identical to the
 *     plain batched path on the same inputs. */
#define LENS_PLAN_FIXED_RESIDENT 1u
lens_status_t lens_chi2_plan_create_ex(lens_ctx_t *ctx, const lens_model_batch_t *batch,
                                       const lens_catalog_t *cat, const lens_chi2_opts_t *opts,
                                       double *chi2, uint32_t flags, void *stream,
                                       lens_chi2_plan_t **out);
/* Either mode (the Sec. 4.2 pipeline of the image mode: sources, deflection
 * grids, triangle search, assignment).  A launch of an image-mode plan does
 * not synchronise: what the eager call reports after its search (slot
 * overflow, Dls/Ds or coordinates outside the search's domain) is kept in
 * the plan's status word, which each launch clears first and
 * lens_chi2_plan_status reads.  With LENS_PLAN_FIXED_RESIDENT the image mode
 * also keeps the fixed potentials' derived table and their deflection at the
 * grid vertices from creation. */
lens_status_t lens_chi2_plan_create2(lens_ctx_t *ctx, const lens_model_batch_t *batch,
                                     const lens_catalog_t *cat, const lens_chi2_opts_t *opts,
                                     double *chi2, int32_t *nimg, int32_t *nmissing,
                                     double *img_xy, uint32_t flags, void *stream,
                                     lens_chi2_plan_t **out);
lens_status_t lens_chi2_plan_launch(lens_chi2_plan_t *plan, void *stream);
/* The outcome of the plan's last launch as lens_chi2_batch would report it
 * (LENS_OK, LENS_EOVERFLOW or LENS_EINVAL); synchronises `stream`, on which
 * the launch was made.  Source-mode plans: LENS_OK. */
lens_status_t lens_chi2_plan_status(lens_chi2_plan_t *plan, void *stream);
lens_status_t lens_chi2_plan_destroy(lens_chi2_plan_t *plan);

/* ---- sampler (the MCMC of Sec. 2.2; Sec. 4's third bottleneck) ----------- */
/* Metropolis sampling of the free potentials' physical parameters with many
 * independent walkers.  Walker w holds n_free potentials of 7 parameters
 * (x0, y0, sigma, e, phi, rcore, rcut) in params[w][k][0..6].  A step, for
 * every walker at once: propose theta'_i = theta_i + step_i (2 u_i - 1)
 * (symmetric); reject a proposal outside the uniform prior box [lo, hi];
 * otherwise evaluate its source-plane chi^2 (fixed potentials then the
 * walker's, FP64) and accept it when chi2' <= chi2 or -2 ln u_last >
 * chi2' - chi2 (probability min(1, exp(-(chi2' - chi2)/2)), likelihood
 * exp(-chi2/2)).  The uniforms u[w][0 .. 7 n_free] in (0, 1] are written by
 * the caller before each step (any generator; they are inputs so that a run
 * can be reproduced elsewhere). */
typedef struct {
    int32_t n_walkers, n_free;  /* >= 1 each */
    double *params;             /* device [n_walkers][n_free][7], updated in place */
    double *chi2;               /* device [n_walkers]: written by create, updated by step */
    int32_t *accepted;          /* device [n_walkers]: accepted moves, incremented */
    const double *lo, *hi;      /* device [n_free][7]: uniform prior box */
    const double *step;         /* device [n_free][7]: proposal half-widths, >= 0 */
    const double *u;            /* device [n_walkers][7 n_free + 1] uniforms, per step */
    int32_t convention;         /* sigma -> b0: 0 Lenstool dPIE (6 pi), 1 SIS (4 pi) */
} lens_mcmc_desc_t;

/* Create a sampler bound to these buffers.  The fixed potentials and the
 * catalogue are read once here (their per-image constants are kept; they
 * must not change while the sampler is used); chi2 receives the chi^2 of the
 * initial parameters.  The prior box must lie in the valid domain (sigma >=
 * 0, 0 <= e < 1, 0 <= rcore, rcore's upper bound below rcut's lower bound)
 * and every walker inside it (LENS_EINVAL otherwise).  The sampler owns its
 * scratch; destroy it before its context.  Synchronises `stream`. */
lens_status_t lens_mcmc_create(lens_ctx_t *ctx, const lens_pot_table_t *fixed,
                               const lens_catalog_t *cat, const lens_mcmc_desc_t *desc,
                               void *stream, lens_mcmc_t **out);
/* One step of every walker (one kernel launch, asynchronous on stream). */
lens_status_t lens_mcmc_step(lens_mcmc_t *sampler, void *stream);
lens_status_t lens_mcmc_destroy(lens_mcmc_t *sampler);

/* ---- host helpers (synchronous, no device) -------------------------------- */
/* Dls/Ds for a flat cosmology (om + ol = 1; the paper's Eq. (3) distances):
 * 1 - chi(zl)/chi(zs), chi the comoving distance.  0 <= zl < zs. */
lens_status_t lens_dlsds(double zl, double zs, double om, double ol, double *out);
/* Time-delay scale (1 + zl) Dl Ds / (c Dls) in days per arcsec^2 for a flat
 * cosmology (om + ol = 1) with H0 in km/s/Mpc: with angular-diameter
 * distances (c/H0) chi/(1+z) it is chi_l chi_s / ((chi_s - chi_l) H0).
 * 0 < zl < zs. */
lens_status_t lens_time_delay_scale(double zl, double zs, double h0, double om, double ol,
                                    double *out);
lens_status_t lens_b0_from_sigma(double sigma_kms, int32_t convention, double *out);
lens_status_t lens_eps_from_e(double e, double *out);
/* Context scratch (bytes) that one call of these sizes takes: for callers
 * that budget device memory or size scratch_bytes_max (the serving loop).
 * lens_map_scratch_bytes: any map call over a table of n_pot potentials (its
 * derived constants).  lens_chi2_scratch_bytes: lens_chi2_batch with these
 * table sizes, samples and catalogue sizes under opts (mode, path, grid,
 * max_img_per_sys are read); image mode is sized for the largest chunk of
 * samples the call uses when the context allows it (128, or 1 on the
 * per-sample path).  Pure arithmetic: the result is exact for the current
 * library, written to *out. */
lens_status_t lens_map_scratch_bytes(int32_t n_pot, uint64_t *out);
lens_status_t lens_chi2_scratch_bytes(int32_t n_fixed, int32_t n_free, int32_t n_samples,
                                      int32_t n_sys, int32_t n_img,
                                      const lens_chi2_opts_t *opts, uint64_t *out);

const char *lens_last_error(void); /* thread-local; valid until the next call */
int32_t lens_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LENSHPC_H */
