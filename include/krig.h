/*
 * krig.h -- C ABI of libkrig, a GPU (gfx950) implementation of the rapid Kriging
 * predictor of Li, Fasshauer & Nychka, "Rapid Approximation Prediction for Kriging".
 *
 * Problem statement (Section 2): observations y_i at sites s_i (i < n) of a
 * zero-mean field g with stationary Matern covariance k (eq. Matern1) plus a
 * nugget tau^2 (eq. ObservationalModel, with the linear part X beta already
 * removed: y = z - X beta_hat).  Kriging coefficients c = (K + tau^2 I)^{-1} y
 * (eq. findc); predictions on a regular m1 x m2 grid approximate
 * g_hat(s_j) = sum_i k(s_j, s_i) c_i (eq. predictionh) by the rapid method of
 * Section 2.2: each k(., s_i) is replaced by an interpolant on the M = (2L)^2
 * grid nodes around s_i (eq. weights), the coefficients are scattered onto the
 * L-padded grid (c* = A^T c, Steps 5-6) and convolved with the covariance lag
 * image through a circulant-embedded 2-D FFT (Step 7, eq. Convolution).
 *
 * Conventions used by every entry point
 *  - Grid node (a, b) is (x0 + a dx, y0 + b dy), a < m1, b < m2, row-major with b
 *    fastest.  The padded grid has P1 = m1 + 2L by P2 = m2 + 2L nodes; padded
 *    index = unpadded index + L.  Sites must satisfy 0 <= (x-x0)/dx <= m1-1 and
 *    0 <= (y-y0)/dy <= m2-1.
 *  - Covariance k(d) = sigma2 * phi(d / range), phi of eq. (Matern1) with
 *    nu in {0.5, 1, 1.5, 2.5} (nu = 1: phi(r) = r K_1(r), evaluated by quadrature to
 *    about 1e-15 relative error; the others in closed form).
 *  - Neighbour offsets (ox, oy) in {-L+1..L}^2 of the lower-left node of the cell
 *    holding a site, listed ox-major; W[i][m] is the weight of offset m.
 *  - d_* pointers are device memory owned by the caller (contiguous, row-major);
 *    h_* pointers are host memory.  The plan keeps its own copies of what it needs.
 *  - "dt" arrays (images, lag, predictions, gradients) have the plan's dtype
 *    (float for KRIG_F32, double for KRIG_F64).  Data y, coefficients alpha,
 *    gradients w.r.t. y and the weights are always FP64.
 *  - Batch counts (B fields, R realisations) must lie in 1..65535 (one launch grid
 *    dimension each), and C components in 1..8; anything else, an empty batch
 *    included, returns KRIG_EINVAL without enqueueing anything.  Point counts of
 *    krig_interp and krig_exact_at may be 0.
 *  - All calls after krig_plan_create are asynchronous on the plan's stream
 *    (krig_set_stream), return a krig_status, never throw, and validate their
 *    arguments on the host before enqueueing anything.  A plan must not be used
 *    from two host threads at once; calls on one plan are ordered by its stream.
 */
#ifndef KRIG_H
#define KRIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KRIG_OK = 0,
  KRIG_EINVAL = -1,       /* bad argument (shape, NULL, size) */
  KRIG_EDOMAIN = -2,      /* a site lies outside the grid's bounding box */
  KRIG_ENOTSPD = -3,      /* non-positive pivot in K + tau^2 I or in K_N */
  KRIG_ECE = -4,          /* circulant embedding not non-negative definite */
  KRIG_ENOMEM = -5,       /* device allocation failed */
  KRIG_EHIP = -6,         /* HIP runtime error */
  KRIG_EUNSUPPORTED = -7  /* unsupported smoothness or transform size */
} krig_status;

typedef enum { KRIG_F32 = 1, KRIG_F64 = 2 } krig_dtype;

typedef struct {
  int32_t m1, m2;       /* prediction grid nodes per axis (>= 2) */
  double x0, y0;        /* first node */
  double dx, dy;        /* spacings (> 0) */
  int32_t L;            /* neighbour order, M = (2L)^2, 1 <= L <= 8 */
} krig_grid;

typedef struct {
  double sigma2;        /* process variance (> 0) */
  double range;         /* divides the distance (> 0) */
  double nu;            /* smoothness: 0.5, 1, 1.5 or 2.5 */
  double tau2;          /* nugget variance (>= 0) */
} krig_matern;

typedef struct krig_plan_s *krig_plan;

/* Sizes and status readable through krig_plan_info. */
enum {
  KRIG_INFO_N = 1, KRIG_INFO_M, KRIG_INFO_P1, KRIG_INFO_P2, KRIG_INFO_F1, KRIG_INFO_F2, KRIG_INFO_H2,
  KRIG_INFO_LDH,        /* pitch (elements) between frequencies of the saved spectra */
  KRIG_INFO_SAVED_PER_FIELD, /* elements (complex FP64) per field of the saved forward spectrum */
  KRIG_INFO_KN_STATUS,  /* 0 clean, 1 jitter added to K_N */
  KRIG_INFO_PIVOT,      /* first failing pivot (1-based) of K + tau^2 I, 0 if none */
  KRIG_INFO_DTYPE,
  KRIG_INFO_CE_CLAMPED, /* number of clamped circulant-embedding eigenvalues (after krig_csim) */
  KRIG_INFO_DLAG_GROUP, /* fields per block in the lag-gradient column pass */
  KRIG_INFO_CE_F1,      /* circulant-embedding torus size (0 before the first krig_csim) */
  KRIG_INFO_CE_F2,
  KRIG_INFO_NL_ROWS64,  /* lines (row pairs) per block of the row passes */
  KRIG_INFO_NL_COLS64,  /* columns per block of the prediction and adjoint column passes */
  KRIG_INFO_FFT_R1,     /* factorisation F2 = R1 * R2 * R3 of the row transforms (R1 = 1: two stages) */
  KRIG_INFO_FFT_R2,
  KRIG_INFO_FFT_R3,
  KRIG_INFO_FFT_VARIANTS_ROWS, /* compiled forms of the row / column transform length */
  KRIG_INFO_FFT_VARIANTS_COLS,
  KRIG_INFO_FFT_VARIANT_ROWS,  /* form in use, 1-based (1: the default form) */
  KRIG_INFO_FFT_VARIANT_COLS,
  KRIG_INFO_SOLVE_NOALLOC_MAX_B, /* largest B krig_solve_noalloc accepts for this plan (0: none) */
  KRIG_INFO_FILTER_SETUP,        /* how the plan's filter spectrum was built (KRIG_FILTER_*) */
  KRIG_INFO_COLS_PAIR,           /* KRIG_TUNE_COLS_PAIR's current value (1: column form) */
  KRIG_INFO_SCATTER              /* KRIG_TUNE_SCATTER's current value */
};

/*
 * Create a plan for one site set, kernel, grid and dtype (Steps 1-4 of Section 2.2
 * and the Cholesky factorisation named after eq. predictionf):
 *  - the lag image lag[a][b] = k((a dx, b dy)), a < m1+L, b < m2+L (Step 2), and
 *    its circulant-embedded spectrum, computed in FP64, scaled by 1/(F1 F2) and
 *    stored in dt, with F1, F2 even 2^a 3^b lengths >= 2m + 2L - 1;
 *  - K_N and its Cholesky factor (Step 1; jitter 1e-14*sigma2*M is added once if
 *    a pivot fails), k_i for every site (Step 3) and A_i = K_N^{-1} k_i (Step 4,
 *    applied as two FP64 MFMA products with the inverse Cholesky factor);
 *  - the CSR layout of A^T over the padded grid (Step 5), built without float
 *    atomics so the scatter sums in a fixed order;
 *  - M = K + tau^2 I, its Cholesky factor and the inverse factor L^{-1} (FP64).
 * h_sites: host [n][2] FP64.  stream: a hipStream_t (NULL = default stream).
 * Synchronises the stream once to read the pivot status.  Returns KRIG_EDOMAIN,
 * KRIG_ENOTSPD (pivot via KRIG_INFO_PIVOT), KRIG_EUNSUPPORTED, KRIG_EINVAL,
 * KRIG_ENOMEM or KRIG_EHIP on failure, in which case *out is NULL.
 */
int krig_plan_create(krig_plan *out, const krig_grid *g, const krig_matern *k, int32_t n,
                     const double *h_sites, int32_t dtype, void *stream);

/* Free the plan and its device memory (synchronises its stream first). */
int krig_plan_destroy(krig_plan p);

/* Read a size or status value (KRIG_INFO_*) into *value. */
int krig_plan_info(krig_plan p, int32_t what, int64_t *value);

/* Change the stream later calls are enqueued on. */
int krig_set_stream(krig_plan p, void *stream);

/*
 * Export the neighbour structure of Steps 3-4: d_anchor [n][2] int32 (lower-left
 * cell node (i0, j0) of each site, unpadded indices) and d_W [n][M] FP64 weights
 * A_i (eq. weights).  Either pointer may be NULL.
 */
int krig_weights(krig_plan p, int32_t *d_anchor, double *d_W);

/*
 * Replace the weights by caller-supplied ones (same layout as krig_weights) and
 * rebuild the CSR layout.  Used to compare the scatter and convolution with a
 * reference on identical weights when K_N is badly conditioned.
 */
int krig_set_weights(krig_plan p, const int32_t *d_anchor, const double *d_W);

/*
 * Nonstationary covariance vectors (Section 6, discussion): Step 3's k_i taken from a
 * caller covariance C while K_N and the lag image stay the plan's stationary ones.
 * d_kvec [n][M] FP64: kvec[i][m] = C(g_m, s_i) for the neighbourhood nodes g_m of site i
 * (anchor from krig_weights, offsets (ox, oy) in {-L+1..L}^2, ox-major, node
 * (x0 + (i0 + ox) dx, y0 + (j0 + oy) dy)).  Replaces the weights by
 * W_i = K_N^{-1} k_i (Step 4, the products of plan creation) and rewrites the scatter
 * structure's weights (its layout depends only on the anchors, which stay the same);
 * later krig_scatter / krig_convolve / krig_predict_adjoint use them.  The
 * coefficients of the nonstationary model are the caller's (krig_convolve takes them);
 * krig_solve / krig_predict keep solving with the plan's stationary K + tau^2 I.
 * Asynchronous on the plan's stream; d_kvec is read before the call's work completes.
 */
int krig_set_kvec(krig_plan p, const double *d_kvec);

/*
 * The plan's filter spectrum (Step 2): its construction, and an optional export.
 *  KRIG_FILTER_REFLECTED (plan_create's): the lag quadrant reflected evenly into the
 *    F1 x F2 torus (zeros beyond the quadrant), transformed;
 *  KRIG_FILTER_CENTERED: the alternative the remark after Step 7 describes, which avoids the
 *    reflections at the price of one more transform: the covariance between the torus centre
 *    node (F1/2, F2/2) and every torus node from plain coordinate differences, transformed and
 *    divided by the transform of the centre's indicator.  It fills every lag up to half the
 *    torus, so the spectrum differs from the reflected one; the kept predictions agree to
 *    rounding (lags beyond the quadrant never reach them).
 * Switching rebuilds the spectrum (FP64, on the plan's stream) for later calls that use the
 * plan's own lag image (caller lag images are always reflected).  d_spec: NULL, or device
 * [H2][F1] FP64 receiving the spectrum scaled by 1/(F1 F2) (frequency k2 < H2 of the row
 * transforms major, then k1 < F1).  KRIG_EINVAL for another setup value or while a recorded
 * batch holds the plan.
 */
enum { KRIG_FILTER_REFLECTED = 0, KRIG_FILTER_CENTERED = 1 };
int krig_filter(krig_plan p, int32_t setup, double *d_spec);

/* Export the lag quadrant (m1+L) x (m2+L) in dt (Step 2's filter). */
int krig_lag(krig_plan p, void *d_lag);

/* Kriging coefficients alpha = (K + tau^2 I)^{-1} y for B fields (eq. findc), FP64:
 * d_y, d_alpha [B][n] (may alias).  Two launches, L^{-1} y into a workspace, then L^{-T}
 * of that, with the explicit inverse Cholesky factor formed at plan creation; bitwise
 * repeatable for a given (n, B).  The products' tile shape depends on n and B (8 x 8 tiles
 * for B <= 8 or when there are few 16 x 16 ones), so one field's alpha can differ in its last
 * bits between calls with different B. */
int krig_solve(krig_plan p, int32_t B, const double *d_y, double *d_alpha);

/*
 * krig_solve for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * results as krig_solve (the same kernels in the same order: bitwise the same alpha), but
 * the workspace comes from a fixed scratch array of KRIG_SOLVE_NOALLOC_SCRATCH_BYTES that
 * the library holds on each GPU from its first use until the process ends; nothing is
 * allocated or freed, and stage timing does not cover this call.  The scratch holds the
 * intermediate vector between the two triangular products, B * (n rounded up to 4) doubles
 * (KRIG_INFO_SOLVE_NOALLOC_MAX_B gives the largest B for a plan: 41943 fields at n = 200,
 * 6132 at n = 1368, 1048 at n = 8000, 419 at n = 20000).  KRIG_EINVAL for a larger
 * request, or when the current device is not the one the plan was created on.
 * Every call on one GPU shares that GPU's scratch, and a call's work reads it after the
 * call returns: calls that overlap on one GPU (other streams, other plans, other host
 * threads) race and give wrong results.  Asynchronous on the plan's stream; d_y and
 * d_alpha may alias.
 */
#define KRIG_SOLVE_NOALLOC_SCRATCH_BYTES (64u << 20)
int krig_solve_noalloc(krig_plan p, int32_t B, const double *d_y, double *d_alpha);

/*
 * Steps 5-6 on their own: the padded coefficient image c* = A^T alpha for B fields,
 * d_alpha [B][n] FP64, d_img [B][P1][P2] dt.  Segment sums in a fixed order,
 * accumulated in FP64 and rounded once (bitwise repeatable).
 */
int krig_scatter(krig_plan p, int32_t B, const double *d_alpha, void *d_img);

/*
 * Rapid prediction from coefficients (Steps 5-7): d_alpha [B][n] FP64 ->
 * d_yhat [B][m1][m2] dt.  d_lag: NULL to use the plan's lag image, else a
 * caller lag quadrant (m1+L) x (m2+L) in dt whose spectrum is recomputed (FP64).
 * d_saved: NULL, or a buffer of B * KRIG_INFO_SAVED_PER_FIELD complex FP64 values
 * that receives the row spectra of c* for krig_predict_adjoint.
 * Precision: every transform, the scatter and the filter product run in FP64
 * arithmetic in both dtypes (the prediction is a cancellation-heavy sum: one FP32
 * rounding of the row spectra of c* moves y_hat by up to ~3e-5 when
 * sum |c*| / max |y_hat| ~ 1e5, so those stay FP64).  A KRIG_F32 plan stores the column
 * pass's output spectra in FP32 (up to ~3e-6 relative on such problems, ~1e-7 on the
 * rest), reads d_lag and writes d_yhat in FP32; a KRIG_F64 plan keeps FP64 throughout.
 */
int krig_convolve(krig_plan p, int32_t B, const double *d_alpha, const void *d_lag, void *d_yhat,
                  void *d_saved);

/*
 * Full prediction y -> yhat: alpha = (K + tau^2 I)^{-1} y (FP64), then
 * krig_convolve.  d_alpha_out [B][n] FP64 may be NULL (else receives alpha).
 */
int krig_predict(krig_plan p, int32_t B, const double *d_y, const void *d_lag, void *d_yhat,
                 double *d_alpha_out, void *d_saved);

/*
 * Adjoint of krig_predict for an upstream gradient d_g = dLoss/dyhat [B][m1][m2] dt:
 *   dalpha_i = sum_m W[i][m] (Phi (*) g)[anchor_i + offset_m]   (correlation with the
 *              symmetric filter on the padded grid, gathered at the neighbours),
 *   d_dy [B][n] FP64    = (K + tau^2 I)^{-1} dalpha            (NULL to skip),
 *   d_dlag (m1+L)x(m2+L) dt = sum_b sum over sign images of (g_b corr c*_b)
 *                               (NULL to skip; summed over the batch; needs the
 *                               coefficients: d_saved from krig_predict, or
 *                               d_alpha [B][n] FP64 to recompute c*).
 * A and the coefficients are held fixed with respect to the lag.  The adjoint runs
 * in FP64 arithmetic with FP64 spectra and correlation image for both dtypes (dy is
 * (K + tau^2 I)^{-1} applied to the gathered correlation, which amplifies any FP32
 * rounding of it by the system's condition number).  d_g and d_dlag are in dt.
 * With both d_dy and d_dlag given (and stage timing off), the lag-gradient tail runs on a
 * second stream that the plan owns, forked from and joined back into the plan's stream
 * with events inside the call (also when that stream is being captured into a graph):
 * callers see the usual ordering on the plan's stream.
 */
int krig_predict_adjoint(krig_plan p, int32_t B, const void *d_g, const double *d_alpha,
                         const void *d_saved, const void *d_lag, double *d_dy, void *d_dlag);

/*
 * Exact kriging prediction from coefficients (eq. predictionh): the dense cross-covariance
 * product that the rapid method approximates, O(N n) covariance evaluations,
 *   d_yhat[b][a][c] = sum_{i < n} k(|node(a, c) - s_i|) alpha[b][i],
 * with the plan's sites and Matern covariance (no nugget: k is the covariance of the
 * field g).  d_alpha [B][n] FP64 (e.g. from krig_solve), d_yhat [B][m1][m2] dt.  Each
 * value is summed in FP64 over the sites in index order and rounded once (bitwise
 * repeatable).  A reference for the approximation error and its cost; B <= 65535.
 * Asynchronous on the plan's stream.
 */
int krig_predict_exact(krig_plan p, int32_t B, const double *d_alpha, void *d_yhat);

/*
 * The same exact prediction at arbitrary points: d_pts [npts][2] FP64 (x, y), anywhere
 * in the plane; d_out [B][npts] FP64.  npts = 0 is a no-op.  Asynchronous.
 */
int krig_exact_at(krig_plan p, int32_t B, const double *d_alpha, int32_t npts, const double *d_pts,
                  double *d_out);

/*
 * The rapid method's interpolated covariance of site i at arbitrary points (eq. weights;
 * the quantity whose error Section 3.2 and Table 2 study):
 *   d_out[j] = sum_{m < M} W[i][m] k(|p_j - g_m|),
 * g_m the site's neighbour nodes (its anchor and the offsets of krig_weights), W[i] its
 * current weights.  d_pts [npts][2] FP64 anywhere in the plane, d_out [npts] FP64.
 * Reads the site's anchor back from the device first (synchronises the plan's stream);
 * npts = 0 is a no-op; KRIG_EINVAL for i outside 0..n-1.
 */
int krig_kernel_at(krig_plan p, int32_t i, int32_t npts, const double *d_pts, double *d_out);

/*
 * Universal kriging (Section 3, eqs. findbeta, findc, predictionf): data with a linear
 * trend in np covariates, 1 <= np <= 16.  d_z [B][n] FP64 data; d_Xs [np][n] FP64 the
 * covariates at the sites (covariate k of site i at d_Xs[k*n + i]: the columns of the
 * paper's X, one per row); d_Xg [np][m1][m2] FP64 the covariates at the grid nodes.
 *   beta_b = (X^T M^{-1} X)^{-1} X^T M^{-1} z_b,  c_b = M^{-1}(z_b - X beta_b),
 *   d_yhat[b] = X_grid beta_b + the rapid prediction of c_b   ([B][m1][m2] dt).
 * d_beta [B][np] FP64 and d_coef [B][n] FP64 may be NULL (else receive beta and c).
 * M^{-1} is the plan's FP64 solve; the np x np system is factored on the GPU, and when
 * X^T M^{-1} X is not numerically positive definite (a Cholesky pivot below 1e-8 of its
 * diagonal entry: covariates dependent at the sites to about four digits) beta, and with
 * it the prediction, is NaN.  B <= 65519.  Asynchronous.
 */
int krig_predict_universal(krig_plan p, int32_t B, const double *d_z, int32_t np, const double *d_Xs,
                           const double *d_Xg, void *d_yhat, double *d_beta, double *d_coef);

/*
 * Off-grid predictions (the closing discussion of Section 6: predict on a fine mesh,
 * then interpolate locally with polynomials).  d_yhat [B][m1][m2] dt is a mesh
 * prediction (e.g. from krig_predict); d_pts [npts][2] FP64 holds (x, y) per point;
 * d_out [B][npts] dt receives, per field, the tensor-product Lagrange polynomial of
 * degree q-1 in x and in y through the q x q mesh nodes around each point: with
 * t = (x - x0)/dx in FP64, the x nodes are sx .. sx+q-1, sx = floor(t) + 1 - ceil(q/2)
 * clamped to [0, m1-q] (the same in y).  A point on a mesh node gets that node's value
 * exactly.  Requires 2 <= q <= 8, q <= m1, q <= m2 and B <= 65535 (else KRIG_EINVAL).
 * Points outside the grid's bounding box (t or u outside [0, m-1], or NaN) give NaN.
 * FP64 arithmetic; asynchronous on the plan's stream; d_out must not overlap d_yhat.
 */
int krig_interp(krig_plan p, int32_t B, const void *d_yhat, int32_t npts, const double *d_pts, int32_t q,
                void *d_out);

/*
 * Nonstationary mixture (Section 6, discussion: a covariance that combines several
 * stationary covariances with spatially varying weights is predicted by running the
 * rapid predictor per stationary component and combining the results):
 *   C(s, s') = sum_c lam_c(s) lam_c(s') k_c(s - s'),
 *   d_yhat[b](s) = sum_c lam_c(s) * rapid_c( lam_c(s_i) alpha[b][i] )(s)  on the m1 x m2 grid.
 * plans[c], c < C <= 8: one distinct plan per component (its kernel k_c, its weights and lag
 * image), all built on the same sites in the same order (not checked) and the same grid
 * nodes and dtype (checked: KRIG_EINVAL otherwise).  d_alpha [B][n] FP64: the mixture
 * model's coefficients (the caller's solve); d_lam_sites [C][n] FP64: lam_c at the sites;
 * d_lam_grid [C][m1][m2] FP64: lam_c at the grid nodes; d_yhat [B][m1][m2] in the plans'
 * dtype.  When all plans have the same neighbour order L (the same transform geometry), the
 * scaling lam_c(s_i) alpha_i rides in each component's scatter and one inverse-row pass
 * transforms every component's rows and adds lam_c times them in FP64 in component order,
 * rounded once to the dtype.  Otherwise each component's prediction goes to its plan's
 * workspace (grown at a new B, like the other workspaces, and rounded to the dtype) and a
 * combine pass sums them in component order in FP64, rounded once.  Runs on stream (NULL:
 * plans[0]'s stream); asynchronous.
 */
int krig_mixture(const krig_plan *plans, int32_t C, int32_t B, const double *d_alpha,
                 const double *d_lam_sites, const double *d_lam_grid, void *d_yhat, void *stream);

/*
 * Conditional simulation (Section 1 steps (1)-(2); circulant embedding as in the
 * discussion section): R realisations on the m1 x m2 grid, d_fields [R][m1][m2] dt.
 * Realisation r: unconditional field u on the padded grid by circulant embedding
 * (complex Philox-4x32-10 noise, counter (bin, r/2, 0, 0), key = seed; real part
 * for even r, imaginary for odd r), u at the sites by the same neighbour weights,
 * simulated data u(s_i) + tau * xi_i (counter (i, r, 1, 0)), residual kriged by
 * the rapid predictor and added to u.  Negative embedding eigenvalues above
 * -1e-6 * max are clamped (count via KRIG_INFO_CE_CLAMPED); otherwise the torus is
 * enlarged up to twice, then KRIG_ECE.  d_y [n] FP64.
 */
int krig_csim(krig_plan p, int32_t R, uint64_t seed, const double *d_y, void *d_fields);

/* Pipeline stages whose kernel launches can be timed (krig_timing_*). */
enum {
  KRIG_STAGE_ROWS_FWD = 0,   /* scatter of alpha_i w_im fused with the forward row transforms */
  KRIG_STAGE_COLS_CONV,      /* column pass: forward transform, x filter, inverse (prediction) */
  KRIG_STAGE_ROWS_INV,       /* inverse row transforms, crop to the m1 x m2 grid */
  KRIG_STAGE_ADJ_ROWS_FWD,   /* adjoint: forward row transforms of the upstream gradient */
  KRIG_STAGE_ADJ_COLS,       /* adjoint: column pass (correlation, and lag-gradient spectra) */
  KRIG_STAGE_ADJ_ROWS_INV,   /* adjoint: inverse row transforms to the padded grid */
  KRIG_STAGE_GATHER,         /* adjoint: gather at the neighbours (d alpha) */
  KRIG_STAGE_SOLVE,          /* FP64 applications of the inverse Cholesky factor */
  KRIG_STAGE_DLAG_TAIL,      /* lag gradient: inverse transforms of the summed spectra + fold */
  KRIG_STAGE_CSIM_CE,        /* conditional simulation: sampler noise and column transforms */
  KRIG_STAGE_CSIM_ROWS,      /* conditional simulation: sampler row transforms (two realisations) */
  KRIG_STAGE_COUNT
};

/*
 * Per-stage kernel timing: while enabled, every launch of a stage is bracketed by
 * two HIP events on the plan's stream.  krig_timing_read synchronises on them and
 * returns the summed elapsed milliseconds and the number of launches since the
 * last read (then resets that stage).  Events are created on first use.
 */
int krig_timing_enable(krig_plan p, int32_t on);
int krig_timing_read(krig_plan p, int32_t stage, double *total_ms, int64_t *launches);

/*
 * Launch shapes.  plan_create picks defaults; a caller or an autotuner may change
 * them between calls.
 *   KRIG_TUNE_NL_ROWS64 / _COLS64: lines or columns per block, >= 1, with
 *     at most 256 threads and 64 KB of LDS per block.  Every line's arithmetic is
 *     unchanged, so results are bitwise the same for any value.
 *   KRIG_TUNE_DLAG_GROUP: fields per block in the lag-gradient column pass (one
 *     field per line of one column), >= 1, with the same thread and LDS limits; more
 *     fields per block means fewer partial spectra to write and sum.  It sets how the
 *     sum over fields of the lag gradient is grouped, so d lag changes by rounding
 *     only; the other outputs are bitwise the same.
 *   KRIG_TUNE_FFT_ROWS / _COLS: which compiled factorisation of the row / column
 *     transform length to use, 1-based (1: the default; count via
 *     KRIG_INFO_FFT_VARIANTS_*).  Resets that side's lines per block (and the field
 *     grouping, for columns) to the form's defaults.  Outputs change by rounding.
 *   KRIG_TUNE_COLS_PAIR: 1 (default): the convolution column pass in the column form;
 *     k + 1 (k = 1..4): the paired form with k columns per block, where the column length
 *     F1 is twice a compiled length that runs on 64 threads (F1 = 768, 1024).  Each column
 *     is then one wave: two half-length transforms (even and odd samples) and a radix-2
 *     butterfly, with no block barrier.  KRIG_EINVAL where F1 has no paired form.  The
 *     prediction and the correlation of the adjoint change by rounding.
 *   KRIG_TUNE_SCATTER: where the scatter of Steps 5-6 runs: 1, fused into the first row
 *     pass (a line of threads takes a whole row's nodes); 2, in calls of fewer than 64 fields,
 *     its own kernel (one thread per padded node) into a workspace image of B * P1 * P2
 *     doubles, then the row pass over that image, for site sets with many entries per node
 *     (calls of 64 fields or more keep the fused form).  Plan creation takes 2 when the sites
 *     give one or more CSR entries per padded node on average (n M >= P1 P2), else 1.  Both
 *     add each node's entries in segment order in FP64: the results are bitwise the same.
 *     A change takes effect at the next call (the first call that takes the scatter apart
 *     allocates the image).
 * Returns KRIG_EINVAL for an unknown key, a value outside those limits, or while a
 * recorded batch (krig_batch) holds the plan.
 */
typedef enum {
  KRIG_TUNE_DLAG_GROUP = 1,
  KRIG_TUNE_NL_ROWS64,
  KRIG_TUNE_NL_COLS64,
  KRIG_TUNE_FFT_ROWS,
  KRIG_TUNE_FFT_COLS,
  KRIG_TUNE_COLS_PAIR,
  KRIG_TUNE_SCATTER
} krig_tune_key;
int krig_plan_tune(krig_plan p, int32_t key, int64_t value);

/*
 * Autotuner: with B fields of synthetic data in temporary buffers, times
 * krig_predict (and, if with_adjoint, krig_predict_adjoint with the saved spectra)
 * on the plan's stream for each candidate value of every KRIG_TUNE_* key in turn
 * (transform forms first, then lines per block and field grouping; candidates are
 * the powers of two up to each key's limit and the limit itself).  Each timing is
 * the median of three windows of ten calls; a candidate replaces the current value
 * only when it is more than 1% faster.  The choice is recorded in a process-wide
 * table keyed by grid, neighbour order, transform lengths and dtype; plans created
 * later with the same key start from it (the scatter form only when they also have the
 * same number of sites, since it follows the site density).  Synchronises the plan's
 * stream.  KRIG_EINVAL while stage timing is on or a recorded batch holds the plan.
 */
int krig_plan_autotune(krig_plan p, int32_t B, int32_t with_adjoint);

/*
 * Uneven batch: predictions for several plans at once (different grids, sites,
 * kernels or dtypes; Section 2.2's predictor applied to each problem).  Problem i is
 * krig_predict(plans[i], h_B[i], h_y[i], NULL, h_yhat[i], NULL, NULL) (h_B NULL: one
 * field each); h_B, h_y and h_yhat are host arrays of count entries, the last two
 * holding device pointers.  stream NULL runs each problem on its plan's own stream;
 * otherwise every problem is enqueued on `stream` and the plans keep their streams.
 * Every argument is checked before anything is enqueued.
 */
int krig_predict_many(const krig_plan *plans, int32_t count, const int32_t *h_B, const double *const *h_y,
                      void *const *h_yhat, void *stream);

/*
 * The same batch recorded once as a HIP graph and replayed by one launch.
 * krig_batch_create grows every plan's workspaces for its B, then captures the
 * batch's kernel launches on `stream` (NULL: a stream of the batch's own), in one of
 * two forms:
 *  lanes 1..16: every problem's own launches, spread over `lanes` parallel branches so
 *    that small problems run side by side (largest problem first, each to the
 *    least-loaded branch);
 *  lanes 0 (persistent): each pass of all problems in one launch per pass and kernel form
 *    (the solve's triangular products and their sums, the scatter + forward rows, the
 *    columns, the inverse rows; problems grouped by transform form): a grid of about one
 *    resident round of blocks that walks the pass's (problem, tile) list, block b taking
 *    items b, b + grid, ..., every tile computing what the problem's own launch computes
 *    (bitwise the same predictions).  Each problem needs its own plan (KRIG_EINVAL for a
 *    repeat).
 * The device pointers in h_y / h_yhat are recorded: a replay reads and writes those
 * buffers.
 * krig_batch_launch replays the graph on `stream` (NULL: the capture stream).
 * While a batch exists its plans refuse krig_plan_destroy and any call that would
 * regrow their workspaces (KRIG_EINVAL); a replay must not overlap other calls on the
 * same plans.  krig_batch_create fails with KRIG_EINVAL while stage timing is on for
 * any of the plans.
 */
typedef struct krig_batch_s *krig_batch;
int krig_batch_create(krig_batch *out, const krig_plan *plans, int32_t count, const int32_t *h_B,
                      const double *const *h_y, void *const *h_yhat, int32_t lanes, void *stream);
int krig_batch_launch(krig_batch b, void *stream);
int krig_batch_destroy(krig_batch b);

/* Human-readable text for a status code (static storage). */
const char *krig_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* KRIG_H */
