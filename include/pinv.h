/*
 * pinv.h -- C-ABI of libpinv, the Pinv-Recon hot path on AMD MI355X (gfx950).
 *
 * The library computes the regularised pseudoinverse of an MRI encoding matrix
 * E by the Cholesky route and applies it to k-space frames:
 *
 *     data  = E x                                      (paper Eq. 1)
 *     R     = (E^H E + lambda I)^-1 E^H                (Eq. 6, normal equations)
 *     E^H E + lambda I = L L^H,  R = L^-H L^-1 E^H     (Eq. 8, Cholesky route)
 *     image = R data                                   (Eq. 3)
 *     R     = E^H (E E^H + lambda I)^-1 when M < N     (Sec. 2.2, right pseudoinverse)
 *
 * `lambda` here is the diagonal shift itself (the paper writes it lambda^2).
 * R depends on the encoding only, so it is built once and applied to any
 * number of frames and acquisitions (Sec. 4.5; Sec. 5).
 *
 * The encoding element (Eq. 2 with the coil, chemical-shift and off-resonance
 * factors of Sec. 3.3 multiplied in; sign convention exp(-i 2 pi ...)):
 *
 *     E[m, n] = C_c(v) exp(-i 2 pi (k_i . r_v + (f_s + B0(v)) t_i))
 *     m = c*nk + i          (coil-major rows, i = sample within a coil)
 *     n = s*V + v,  v = iy*nx + ix,  V = nx*ny   (species-major columns)
 *     r_v = ((ix - nx/2)/nx, (iy - ny/2)/ny)     (field-of-view units)
 *     k in cycles per field of view, f_s and B0 in Hz, t in seconds.
 *
 * Conventions for every entry point:
 *   - Status codes only: no exceptions or aborts cross this ABI.  The detail
 *     of the last failure on the calling thread is in pinv_last_error().
 *   - "host" pointers are read during the call and may be freed on return.
 *   - "device" pointers are HIP device memory owned by the caller; they must
 *     stay valid until the work enqueued on `hip_stream` has completed.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously; nothing blocks unless stated.
 *   - Complex arrays are interleaved (re, im) pairs, row-major:
 *     complex64 (float2) for FP32 and BF16X3 plans, complex128 (double2)
 *     for FP64 plans.
 */
#ifndef PINV_H
#define PINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PINV_OK = 0,
  PINV_ERR_INVALID = 1,     /* bad argument or encoding */
  PINV_ERR_NOMEM = 2,       /* device memory or the context budget exhausted */
  PINV_ERR_NOT_PD = 3,      /* a Cholesky pivot was <= 0 or NaN (message names the column) */
  PINV_ERR_DEVICE = 4,      /* a HIP runtime error */
  PINV_ERR_BUSY = 5,        /* the plan is still building (non-blocking query) */
  PINV_ERR_UNSUPPORTED = 6  /* a valid request this library does not implement */
} pinv_status;

typedef enum {
  PINV_FP64 = 0,    /* everything in FP64 (complex128 data and images) */
  PINV_FP32 = 1,    /* W, R and apply on FP32 MFMA; the Gram (default form) and the
                       factorisation in FP64 */
  PINV_BF16X3 = 2   /* as FP32 but products as three BF16 MFMAs (hi*hi + hi*lo + lo*hi),
                       operands split into bf16 hi/lo once, where produced */
} pinv_precision;

typedef enum {
  PINV_LAMBDA_ABS = 0,           /* lambda is the absolute diagonal shift */
  PINV_LAMBDA_REL_MEAN_DIAG = 1  /* shift = lambda * trace(E^H E) / N (= lambda * mean diagonal) */
} pinv_lambda_mode;

/* Encoding description (all host pointers, FP64; copied during pinv_build).
 * Defines E as above (Eq. 2; Sec. 3.3 generalised encoding; Eq. 11 coil rows).
 *
 * Voxel mask (Sec. 3.1 and Sec. 4.4: voxels outside the object or a circular
 * field of view are left out of the unknowns, shrinking the Gram): with
 * `voxels` non-NULL only the nvox listed voxels v = iy*nx + ix are unknowns,
 * so V = nvox in the column index n = s*V + j (j = position in the list) and
 * N = S*nvox.  The list must be strictly ascending and inside [0, nx*ny).
 * coil and b0_hz still cover the whole grid ([C][nx*ny], [nx*ny]). */
typedef struct {
  int32_t nx, ny;             /* image grid, nx, ny >= 1 */
  int64_t nk;                 /* samples per coil, >= 1 */
  const double *k;            /* [nk][2] (kx, ky) in cycles/FOV; required */
  const double *t;            /* [nk] sample times in s; required if nspecies > 1,
                                 species_hz != NULL or b0_hz != NULL */
  int32_t ncoil;              /* C >= 1 */
  const double *coil;         /* [C][nx*ny][2] complex sensitivities; NULL => C == 1, all ones */
  const double *b0_hz;        /* [nx*ny] off-resonance in Hz, or NULL */
  int32_t nspecies;           /* S >= 1 */
  const double *species_hz;   /* [S] species frequencies in Hz, or NULL (=> S == 1 at 0 Hz) */
  const int32_t *voxels;      /* [nvox] ascending voxel indices of the mask, or NULL (all) */
  int32_t nvox;               /* entries in voxels (ignored when voxels is NULL) */
} pinv_encoding;

#define PINV_FLAG_KEEP_GRAM 1   /* accepted for compatibility: every plan keeps E^H E */
#define PINV_FLAG_UNCACHED 2    /* build a fresh plan outside the cache (freed on its last release) */
#define PINV_FLAG_GRAM_FULL 4   /* the same as gram = PINV_GRAM_FULL */
#define PINV_FLAG_NO_R 8        /* factor-only plan: Gram, shift and Cholesky with L^-1, but no W
                                   and no R.  Applies solve the normal equations directly,
                                   image = L^-H L^-1 (sum_c E_c^H data_c), with E regenerated per
                                   tile (Sec. 2.4, direct solution without explicit inversion; the
                                   coil-wise adjoint after Eq. 11).  Holds N*N instead of N*M + N*N
                                   complex values and skips 8MN^2 build flops; each frame costs the
                                   same 8NM as R*data plus 8N^2 for the two triangular products.
                                   SRF, noise matrix and the R buffer are unavailable.  Not with
                                   PINV_BF16X3 (the split products only form W and R). */
#define PINV_FLAG_R_FP64 16     /* PINV_FP32 plans only: form W = L^-1 E^H and R = L^-H W in FP64
                                   (E generated from the FP64 tables, L^-1 kept in FP64) and round
                                   R once to complex64.  Applies then run on FP32 MFMA with the
                                   error of that one rounding (~u32 times the cancellation in
                                   R*data, about 1e-6 relative) instead of kappa(G)*u32, so they
                                   need no refinement for a 1e-5 target (Sec. 5: lower precision
                                   for the bulk of the arithmetic, results stored at higher
                                   precision).  The build costs what an FP64 build costs. */

/* Complex-product form of the triangular products W, R and the apply (MFMA). */
typedef enum {
  PINV_CPROD_AUTO = 0,   /* 3M for FP32 plans, 4M for FP64 plans and FP64-formed R */
  PINV_CPROD_3M = 1,     /* three real products per complex product (Gauss):
                            re = ar br - ai bi, im = (ar + ai)(br + bi) - ar br - ai bi;
                            25% fewer matrix-core operations, the imaginary part carries
                            about twice the rounding of 4M */
  PINV_CPROD_4M = 2      /* four real products per complex product */
} pinv_cprod;

/* How the Gram E^H E is formed. */
typedef enum {
  PINV_GRAM_AUTO = 0,    /* PSF without an off-resonance map, otherwise SHARED */
  PINV_GRAM_PSF = 1,     /* Toeplitz / point-spread form (needs b0_hz == NULL): with every
                            coil on one trajectory, E^H E = (F^H F) o (coil cross-products)
                            (Eq. 11), and F^H F between voxels a, b of species s_a, s_b is the
                            PSF at the offset r_b - r_a,
                              sum_i exp(-i 2 pi (k_i . (r_b - r_a) + (f_sb - f_sa) t_i)),
                            formed once on the (2nx-1) x (2ny-1) offset grid for each species
                            pair (FP64) and then expanded: O(K nx ny S^2 + C N^2) work instead
                            of O(K N^2) */
  PINV_GRAM_SHARED = 2,  /* F^H F on MFMA in FP64 over one coil's nk rows (F generated per
                            tile), times the coil cross-products: 4 nk N^2 flops */
  PINV_GRAM_FULL = 3     /* E^H E over all M = C*nk rows in the plan's precision (Eq. 11 as
                            written): 4 M N^2 flops; the only form for an FP32 Gram */
} pinv_gram_form;

/* How R is formed from the Gram. */
typedef enum {
  PINV_ROUTE_CHOLESKY = 0,  /* G + lambda I = L L^H, R = L^-H L^-1 E^H (Eq. 8) */
  PINV_ROUTE_EIGEN = 1      /* E^H E = P Lambda P^H (Eq. 7), R = P_r diag(1/(mu_j + lambda))
                               P_r^H E^H over the eigenvalues mu_j the truncation keeps: with
                               lambda = 0 the truncated SVD of Eq. 4, with no truncation the
                               Tikhonov R of the Cholesky route, or both combined (Sec. 2.2).
                               The FP64 eigendecomposition is a parallel cyclic Jacobi method
                               on the GPU; pinv_build then blocks until it has converged, or
                               returns PINV_ERR_UNSUPPORTED after 60 sweeps without
                               converging (O(N^3) each; 52 sweeps, 48 s at N = 4096).
                               PINV_FP64 and PINV_FP32 plans with M >= N; no refinement, no
                               PINV_FLAG_NO_R. */
} pinv_route;

/* Truncation of the eigenvalue route (Sec. 2.1: singular values below a
 * threshold are dropped; the ratio of the largest to the smallest kept one is
 * the condition number kappa, and a threshold may instead keep a fraction of
 * the energy).  mu_j are the eigenvalues of E^H E (sigma_j^2), largest first. */
typedef enum {
  PINV_TRUNC_NONE = 0,     /* keep all */
  PINV_TRUNC_KAPPA = 1,    /* keep sigma_j with sigma_1 / sigma_j <= trunc_value (>= 1) */
  PINV_TRUNC_ENERGY = 2    /* keep the fewest largest mu_j whose sum reaches trunc_value
                              (in (0, 1]) of sum mu_j */
} pinv_trunc;

typedef struct {
  double lambda;              /* >= 0; meaning set by lambda_mode */
  int32_t lambda_mode;        /* pinv_lambda_mode */
  int32_t prec;               /* pinv_precision */
  int32_t flags;              /* PINV_FLAG_* */
  int32_t cprod;              /* pinv_cprod; PINV_BF16X3 plans take only AUTO */
  int32_t nb;                 /* factorisation block size (Sec. 2.3): 0 (default, 128), 64 or
                                 128.  The factorisation steps 64 columns at a time (the
                                 diagonal-block kernel holds one 64 x 64 complex128 block in
                                 registers, one column per lane of a wavefront); nb = 64
                                 updates the whole trailing matrix after every step (rank 64),
                                 nb = 128 after every second step (rank 128, the first step of
                                 a pair updating only the next block column).  The
                                 factorisation's products run 4M whatever cprod says */
  int32_t gram;               /* pinv_gram_form */
  int32_t route;              /* pinv_route */
  int32_t trunc;              /* pinv_trunc (PINV_ROUTE_EIGEN only) */
  double trunc_value;         /* kappa or energy fraction, as pinv_trunc says */
} pinv_build_opts;

typedef struct {
  int64_t N, M;               /* unknowns S*V and rows C*nk */
  double lambda_abs;          /* the diagonal shift actually used */
  int32_t prec;               /* pinv_precision */
  int32_t ready;              /* 1 once pinv_plan_wait has returned PINV_OK */
  uint64_t key;               /* cache key (hash of encoding, shift and precision) */
  size_t device_bytes;        /* device memory the plan holds */
  float stage_ms[4];          /* Gram, Cholesky+inverse, W = L^-1 E^H, R = L^-H W
                                 (HIP event times on the build stream; valid when ready;
                                 the last two are 0 for factor-only plans; with M < N the
                                 last holds both products of the right pseudoinverse and
                                 the third is 0; on the eigenvalue route the second is the
                                 eigendecomposition, truncation and Q^H) */
  int32_t has_r;              /* 0 for plans built with PINV_FLAG_NO_R */
  int64_t gram_order;         /* N, or M when M < N (the samples' Gram E E^H, right
                                 pseudoinverse R = E^H (E E^H + lambda I)^-1, Sec. 2.2) */
  int32_t ncoil;              /* C */
  int32_t cprod;              /* the product form used: PINV_CPROD_3M or PINV_CPROD_4M */
  int64_t nk;                 /* samples per coil */
  int32_t gram_form;          /* the Gram form used (PSF, SHARED or FULL; SHARED for M < N) */
  int32_t r_fp64;             /* 1 if R was formed in FP64 (PINV_FLAG_R_FP64) */
  int32_t route;              /* pinv_route */
  int32_t rank;               /* eigenvalues kept by the eigenvalue route (N otherwise; valid
                                 when ready) */
  int32_t sweeps;             /* Jacobi sweeps the eigenvalue route took (0 otherwise) */
  int32_t reserved;           /* 0 */
} pinv_plan_info;

typedef struct {
  const void *plan;           /* const pinv_plan* */
  const void *data;           /* device [F][M] */
  void *image;                /* device [F][N] */
  int64_t F;                  /* frames >= 0 */
} pinv_apply_item;

typedef struct pinv_context pinv_context;
typedef struct pinv_plan pinv_plan;

/* Create a context on HIP device `device`.  It owns the plan cache and an HBM
 * budget: `hbm_budget_bytes` (0 = 90% of the device memory free at creation).
 * Errors: INVALID (bad device), DEVICE. */
pinv_status pinv_context_create(int device, size_t hbm_budget_bytes, pinv_context **out);

/* Destroy a context: synchronises the device and frees every cached plan.
 * Plans the caller still holds become invalid. */
pinv_status pinv_context_destroy(pinv_context *ctx);

/* Build (or fetch from the cache) R for encoding `e` (Eq. 6, Eq. 8).
 * With at least as many samples as unknowns (M >= N), R = (E^H E + lambda I)^-1
 * E^H through the N x N Gram.  With fewer (M < N) the build takes the right
 * pseudoinverse R = E^H (E E^H + lambda I)^-1 through the M x M samples' Gram
 * (Sec. 2.2): the same R for lambda > 0, and the minimum-norm solution for
 * lambda = 0; such plans (gram_order = M) take no PINV_FLAG_NO_R or
 * PINV_FLAG_GRAM_FULL and no PINV_BF16X3, their L^-1 and Gram
 * buffers are M x M, and their stage times put W, Z = L'^-H W and R = Z^H
 * in the last stage.  Enqueues on `hip_stream` and returns at once with a new
 * reference to the plan in *out (release it with pinv_plan_release).  A plan
 * with the same key already in the cache is returned without new work.
 * Admission: if the plan's footprint exceeds the free budget,
 * least-recently-used cached plans that no caller holds are evicted; if that
 * is not enough, NOMEM.  Errors: INVALID (bad encoding, lambda < 0, flag
 * combinations above), UNSUPPORTED (BF16X3 with M < N), NOMEM, DEVICE.  A
 * non-positive-definite shifted Gram is reported by pinv_plan_wait as NOT_PD. */
/* With PINV_ROUTE_EIGEN the second stage time is the eigendecomposition, the
 * truncation and Q^H = diag(1/sqrt(mu_j + lambda)) P_r^H; the third and fourth
 * are W = Q^H E^H and R = Q W (dense factors, rank rows). */
pinv_status pinv_build(pinv_context *ctx, const pinv_encoding *e, const pinv_build_opts *o,
                       void *hip_stream, pinv_plan **out);

/* Block until the plan's build has finished; returns its outcome
 * (OK, NOT_PD with the failing column in pinv_last_error, DEVICE). */
pinv_status pinv_plan_wait(pinv_plan *p);

/* Non-blocking: PINV_OK if the plan's build has finished successfully,
 * PINV_ERR_BUSY while it is still running, otherwise its failure status. */
pinv_status pinv_plan_query(pinv_plan *p);

/* The cache key pinv_build would give this encoding and options (host only). */
pinv_status pinv_encoding_key(const pinv_encoding *e, const pinv_build_opts *o, uint64_t *key,
                              size_t *plan_bytes);

/* image[f] = R data[f] for F frames (Eq. 3), enqueued on `hip_stream` behind
 * the plan's build.  data: device [F][M], image: device [F][N], dtype of the
 * plan (see conventions).  A factor-only plan (PINV_FLAG_NO_R) gives
 * image = L^-H L^-1 E^H data instead, E^H data formed with E generated in the
 * plan's precision.  refine_steps (0..4) adds iterative refinement on
 * the normal equations (Eq. 6): r = E^H (d - E x) - lambda x in FP64 with E
 * regenerated in FP64, then x += L^-H L^-1 r.  Plans with M < N refine on the
 * sample side instead: y = G'^-1 d with G' = E E^H + lambda I refined against
 * the FP64 G', then x = E^H y with E in FP64.  Applies of a few frames read
 * R once, bound by HBM bandwidth: at most 8 frames of an FP64 plan and 2 of
 * an FP32 or BF16X3 plan stream R row by row on the vector units, 3 to 32
 * frames of an FP32 or BF16X3 plan stream it into the matrix cores; more
 * frames run as MFMA tiles.  The paths round
 * differently.  The path and the split of the sum over M follow from F, N and
 * M alone, and a frame's result does not depend on the values of the other
 * frames.  Errors: INVALID, NOMEM (scratch), DEVICE. */
pinv_status pinv_apply(pinv_context *ctx, const pinv_plan *p, const void *data, int64_t F,
                       void *image, int32_t refine_steps, void *hip_stream);

/* Several applies (possibly of different plans and sizes) in grouped launches
 * (Sec. 4.1: one R reconstructs every time point and metabolite in a few
 * matrix-matrix products; Sec. 5: R reused across acquisitions): one MFMA
 * launch per run of up to 32 items of the same precision and product form.
 * Each item's result equals what pinv_apply gives for it alone.  Errors as
 * pinv_apply. */
pinv_status pinv_apply_grouped(pinv_context *ctx, int32_t n, const pinv_apply_item *items,
                               int32_t refine_steps, void *hip_stream);

/* ------------------------------------------------------------------------
 * Apply without allocation.  For callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.
 * ------------------------------------------------------------------------ */
#define PINV_NOALLOC_SCRATCH_BYTES (512ull << 20)

/* pinv_apply (same arguments, same results bit for bit) with every scratch
 * buffer it uses (split-contraction partials, refinement vectors and
 * residuals, factor-only intermediates) taken from a fixed device region of
 * PINV_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call.  Every call on a GPU shares that GPU's region, which keeps
 * the last call's contents (nothing in it needs to start at zero): calls that
 * overlap on one GPU (on different streams or threads) race, and the caller
 * must serialise them.  Work enqueued here is not tracked by the plan: it must
 * have completed before the plan is released.  Errors: as pinv_apply, and
 * INVALID for an apply that needs more scratch than the region holds (the
 * message gives the bytes; pinv_apply, or fewer frames per call, serves it). */
pinv_status pinv_apply_noalloc(pinv_context *ctx, const pinv_plan *p, const void *data, int64_t F,
                               void *image, int32_t refine_steps, void *hip_stream);

/* Shapes of the image-quality metrics. */
typedef enum { PINV_METRIC_DIAG = 0, PINV_METRIC_FULL = 1 } pinv_metric_mode;

/* Spatial response function of the plan's reconstruction (Sec. 2.5, Eq. 9):
 * SRF = R E, with E regenerated from the plan's tables as in the build.
 * PINV_METRIC_DIAG writes the N diagonal entries (the SRF map; the caller
 * reshapes column order n = s*V + iy*nx + ix to the grid); PINV_METRIC_FULL
 * writes the N x N matrix, row-major.  Entries are complex: complex128 for FP64
 * plans, complex64 otherwise (for an exact R the matrix is Hermitian and the
 * diagonal real, so imaginary parts of the map are rounding-level).
 * out: device, caller-owned, N or N*N entries.  Ordered on hip_stream after
 * the plan's build.  Errors: INVALID (NULL, bad mode, plan of another
 * context), UNSUPPORTED (factor-only plan), DEVICE. */
pinv_status pinv_srf(pinv_context *ctx, const pinv_plan *p, int32_t mode, void *out,
                     void *hip_stream);

/* Noise matrix of the reconstruction (Sec. 2.5, Eq. 10): X = R Psi R^H for
 * data noise that is white over samples and correlated over coils,
 * Psi = Psi_c (kron) I_K.  coil_cov: host [C][C] complex128 interleaved,
 * row-major, Hermitian positive definite, copied before return; NULL means
 * Psi = I.  PINV_METRIC_DIAG writes diag(X), N real values (double for FP64
 * plans, float otherwise; the noise map is their square root).
 * PINV_METRIC_FULL writes X, N x N complex, row-major; with a coil covariance
 * it allocates an N x M work array on hip_stream's memory pool for the call.
 * With coil_cov the call synchronises hip_stream once (the covariance factor is
 * staged through pinned host memory).  Errors: INVALID (NULL, bad mode,
 * coil_cov not Hermitian positive definite), UNSUPPORTED (factor-only plan),
 * NOMEM, DEVICE. */
pinv_status pinv_noise(pinv_context *ctx, const pinv_plan *p, const double *coil_cov, int32_t mode,
                       void *out, void *hip_stream);

/* Forward model data[f] = E image[f] (Eq. 1) in the plan's precision, with E
 * generated on the fly.  image: device [F][N], data: device [F][M].  Enqueued
 * on `hip_stream` behind the upload of the plan's tables. */
pinv_status pinv_forward(pinv_context *ctx, const pinv_plan *p, const void *image, int64_t F,
                         void *data, void *hip_stream);

/* Eigenvalues of E^H E (the squared singular values of E, Sec. 2.1) of a
 * plan built with PINV_ROUTE_EIGEN, largest first: out is device [N] double,
 * caller-owned; ordered on hip_stream after the build.  Errors: INVALID (NULL,
 * a plan of another route). */
pinv_status pinv_spectrum(pinv_context *ctx, const pinv_plan *p, double *out, void *hip_stream);

/* Plan metadata; stage_ms are filled once the plan is ready. */
pinv_status pinv_plan_info_get(const pinv_plan *p, pinv_plan_info *out);

/* Device pointers held by a ready plan (any may be NULL on output):
 *   R     [N][M] complex, the reconstruction matrix.  A PINV_BF16X3 plan holds
 *         it split-packed instead: N rows of Mp = 32*ceil(M/32) columns (zero
 *         past M), each 8 consecutive columns of a row stored as 64 bytes,
 *         the bf16 planes re_hi[8], re_lo[8], im_hi[8], im_lo[8] (value =
 *         hi + lo); pinv_plan_copy_buffer returns it as complex64.
 *   Linv  [N][N] complex, L^-1 (lower; FP32 plans hold it as complex64)
 *   gram  [N][N] complex128, E^H E (full Hermitian; used by the refinement residual)
 * The memory stays owned by the plan.  Work the caller enqueues on these
 * pointers itself is not tracked by the plan: it must have completed, or be
 * ordered before a later library call on the plan, when the plan is released. */
pinv_status pinv_plan_buffers(const pinv_plan *p, void **R, void **Linv, void **gram);

/* Copy one of the plan's buffers (0 = R, 1 = L^-1, 2 = Gram) into caller
 * device memory `dst` of `bytes` bytes (must equal the buffer's size:
 * N*M or N*N complex of the plan's type; the Gram is complex128), enqueued on
 * `hip_stream` behind the build.  Errors: INVALID (size or missing buffer). */
pinv_status pinv_plan_copy_buffer(const pinv_plan *p, int32_t which, void *dst, size_t bytes,
                                  void *hip_stream);

/* Drop one reference.  The last reference held by neither a caller nor the
 * cache frees the plan without waiting on the host: its buffers return to the
 * context's plan pool once the build and every apply, forward, metric and copy
 * enqueued on the plan, on whatever stream, have completed. */
pinv_status pinv_plan_release(pinv_plan *p);

/* Hand device memory that the context's stream-ordered pools keep after
 * completed work (refinement scratch, build workspaces, buffers of released
 * plans) back to the device.  The library does this by itself for scratch and
 * workspaces when less than a quarter of the device is free, and for all of it
 * when a plan or workspace allocation fails. */
pinv_status pinv_context_trim(pinv_context *ctx);

/* Evict every cached plan no caller holds; returns the bytes freed in *freed. */
pinv_status pinv_cache_trim(pinv_context *ctx, size_t *freed);

/* Budget accounting: bytes in use by plans and the budget. */
pinv_status pinv_context_usage(const pinv_context *ctx, size_t *used, size_t *budget,
                               int32_t *cached_plans);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request loop on one device.
 *
 * R depends on the encoding only (Sec. 4.5; Sec. 5), so the server keeps
 * built plans in an LRU cache keyed by encoding (pinv_encoding_key), admits a
 * new build only while its device footprint fits `hbm_budget_bytes`
 * (evicting least-recently-used plans that no queued or running request
 * holds), and packs the applies of every request whose plan is ready into
 * grouped launches (pinv_apply_grouped).  Builds and applies run on two
 * HIP streams of the library's own, so requests arriving while others run
 * overlap on the device.  The library creates its streams (these two and the
 * factorisation's look-ahead stream) once per device and keeps them until the
 * process ends, so their mapping onto the process's few hardware queues does
 * not change as contexts and servers come and go.  Each request's result is the same as pinv_apply of its plan on its
 * data alone.  A worker thread runs the scheduler; all calls are thread-safe.
 * Times are seconds on a host monotonic clock from server creation.
 * ------------------------------------------------------------------------ */
typedef struct pinv_server pinv_server;

typedef struct {
  size_t hbm_budget_bytes;    /* device bytes for plans (resident and build workspace), > 0 */
  int32_t max_group;          /* requests per grouped apply, 1..32 */
  int32_t max_inflight;       /* grouped applies in flight, >= 1 */
  int32_t max_builds;         /* concurrent builds, >= 1 */
  int32_t reserved;           /* 0 */
} pinv_server_opts;

typedef struct {
  const pinv_encoding *enc;   /* host; copied at submit */
  pinv_build_opts opts;       /* build options of the request's plan */
  const void *data;           /* device [F][M], caller-owned until completion; written
                                 and complete before submit (the server's streams are not
                                 ordered after the caller's streams) */
  void *image;                /* device [F][N], caller-owned until completion; no work of
                                 the caller may still be pending on it at submit */
  int64_t F;                  /* frames >= 0 */
  int32_t refine_steps;       /* 0..4, as in pinv_apply */
  int32_t reserved;           /* 0 */
  uint64_t tag;               /* returned in the completion */
} pinv_request;

typedef struct {
  uint64_t ticket, tag;
  int32_t status;             /* pinv_status of the request */
  int32_t built;              /* 1 if this request triggered its plan's build */
  double t_arrival, t_dispatch, t_done;   /* submit, grouped-apply issue, completion seen */
} pinv_completion;

typedef struct {
  uint64_t builds, build_failures, evictions, hits, batches, items, completed;
  uint64_t invariant_violations;   /* budget exceeded or a held plan evicted: always 0 */
  size_t used, peak_used, budget;
  int32_t cached_plans, pending, running;
} pinv_server_stats;

/* Errors: INVALID, DEVICE. */
pinv_status pinv_server_create(pinv_context *ctx, int device, const pinv_server_opts *o,
                               pinv_server **out);
/* Queue one request; *ticket identifies it.  Errors: INVALID (as pinv_build). */
pinv_status pinv_server_submit(pinv_server *s, const pinv_request *r, uint64_t *ticket);
/* Take up to `max` completions (in completion order); *n = how many. */
pinv_status pinv_server_poll(pinv_server *s, pinv_completion *out, int32_t max, int32_t *n);
/* Wait until no request is queued or running (timeout_s <= 0: no limit);
 * BUSY on timeout. */
pinv_status pinv_server_drain(pinv_server *s, double timeout_s);
pinv_status pinv_server_stats_get(pinv_server *s, pinv_server_stats *out);
/* Stop the worker, wait for device work, release every plan the server holds. */
pinv_status pinv_server_destroy(pinv_server *s);

const char *pinv_status_string(pinv_status s);
const char *pinv_last_error(void);   /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* PINV_H */
