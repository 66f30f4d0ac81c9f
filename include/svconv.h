/*
 * svconv.h - C ABI of the MI355X (gfx950) spatially-varying-kernel
 * convolution and image-subtraction library (libsvconv.so).
 *
 * The method (Hartung, Shukla, Miller & Pennypacker, Sec. 2):
 *
 *   D = (R (x) K) - I                                           (Eq. 1)
 *   K(x,y) = sum_n c_n(x,y) B_n,  c_n(x,y) = sum_m a[n][m] P_m(x,y)
 *                                                         (Eq. 2, Eq. 3)
 *
 * R is the reference image, I the image it is matched to, B_n the basis
 * functions, P_m the spatial polynomial terms and a[n][m] the coefficients.
 * The kernel differs at every pixel and is used in full at every pixel
 * (Sec. 3).
 *
 * Conventions used by every entry point:
 *   - images: float32, row-major [height][width], contiguous, x = column,
 *     y = row; R is treated as 0 outside the supplied array;
 *   - (R (x) K)(x,y) = sum_{u,v} K(x,y)[u,v] R(x-u, y-v), u,v in [-h, h]
 *     (true convolution; the kernel is taken at the output pixel);
 *   - basis: for Gaussian g (width sigma_g, degree d_g), for t = 0..d_g and
 *     i = t..0, j = t-i: exp(-(u^2+v^2)/(2 sigma_g^2)) u^i v^j scaled to unit
 *     L1 norm; sigma_g = 0 is a Kronecker delta (d_g must be 0);
 *   - spatial terms: P_m = xh^i yh^j for t = 0..spatial_degree, i = t..0,
 *     with xh = 2 (x + x0) / (frame_width - 1) - 1 and yh likewise, over the
 *     frame set by svconv_plan_set_frame (default: the image itself);
 *   - coefficients: a is float32 [N][M], n-major (N bases, M spatial terms).
 *
 * Memory: every image, coefficient, gradient and matrix pointer is a DEVICE
 * pointer owned by the caller, unless a comment says "host".  The plan owns
 * its tables and scratch, which are allocated by svconv_plan_create; the
 * compute entry points allocate nothing.
 *
 * Asynchrony: compute entry points enqueue work on the plan's stream and
 * return.  Invalid arguments are rejected with SVCONV_EINVAL before any HIP
 * call.  Launch failures return SVCONV_EDEVICE; faults inside a kernel
 * surface at the caller's next synchronisation.  Entry points that return a
 * value computed on the device (svconv_cholesky_factor, svconv_gn_step)
 * synchronise the plan's stream and say so.
 *
 * Threads: a plan must not be used by two threads at once; distinct plans
 * are independent.  No entry point aborts or exits.
 */
#ifndef SVCONV_H
#define SVCONV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct svconv_plan svconv_plan;

enum svconv_status {
    SVCONV_OK = 0,
    SVCONV_EINVAL = -1,       /* invalid argument (checked before any HIP call) */
    SVCONV_ENOMEM = -2,       /* device or host allocation failed */
    SVCONV_EDEVICE = -3,      /* HIP runtime or launch error */
    SVCONV_EUNSUPPORTED = -4, /* valid but outside what the kernels support */
    SVCONV_ENOTSPD = -5       /* matrix not symmetric positive definite */
};

/* Arithmetic of the basis contraction (the dominant step); for the
 * SEPARABLE form see below. */
enum svconv_precision {
    SVCONV_FP32 = 0,    /* float32 matrix cores (v_mfma_f32_16x16x4_f32)      */
    SVCONV_BF16 = 1,    /* bf16 inputs, fp32 accumulation, 1 product          */
    SVCONV_FP16 = 2,    /* fp16 inputs, fp32 accumulation, 1 product          */
    SVCONV_BF16X3 = 3,  /* R and B split hi+lo in bf16: hh + lh + hl          */
    SVCONV_FP16X2 = 4,  /* R split hi+lo in fp16, B in fp16: hh + lh          */
    SVCONV_FP16X3 = 5   /* R and B split hi+lo in fp16: hh + lh + hl          */
};
/* Error of D against its float64 definition, max |dD| over the interior of
 * star fields on a 1000 ADU sky (sigma_sky = sqrt(1000) = 31.6 ADU; the
 * brightest stars near 1e5 ADU), with the pedestal at the sky level:
 *   SVCONV_FP32    below 1e-4 sigma_sky in every form;
 *   SVCONV_FP16X3  about 1e-4 sigma_sky;
 *   SVCONV_BF16X3  up to 1.5e-3 sigma_sky;
 *   SVCONV_FP16X2  up to 5e-2 sigma_sky (the taps keep 11 bits);
 *   SVCONV_FP16    up to 5e-2 sigma_sky, and
 *   SVCONV_BF16    up to 0.5 sigma_sky (one 16-bit part per operand).
 * Only FP32, FP16X3 and BF16X3 stay within 1e-2 sigma_sky; FP16X2, FP16
 * and BF16 are faster and miss that bound at bright stars.  A split value x
 * is hi + lo with hi = x rounded to 16 bits and lo = (x - hi) rounded to 16
 * bits (x - hi is exact in float32).  The basis and regrouped forms and every
 * filter tap round to nearest even: |x - hi - lo| <= 2^-22 |x| (fp16) or
 * 2^-16 |x| (bf16).  The separable forms take the fp16 hi part of image data
 * and row responses toward zero (one instruction for two values) and round
 * lo to nearest even: |x - hi - lo| < 2^-21 |x|; the adjoint in R truncates
 * the bf16 hi part: < 2^-15 |x|.  The measured errors above include these
 * roundings. */

/* How the per-pixel kernel is contracted (both give D of Eq. 1 exactly, up
 * to rounding).  BASIS: N basis responses T_n = B_n (x) R, then
 * D = sum_n c_n T_n - I.  REGROUPED: Kt_m = sum_n a[n][m] B_n (built on the
 * device per call), then D = sum_m P_m (Kt_m (x) R) - I, which needs M
 * instead of N filters because P_m depends only on the output pixel. */
enum svconv_form {
    SVCONV_FORM_BASIS = 0,
    SVCONV_FORM_REGROUPED = 1,
    SVCONV_FORM_SEPARABLE = 2,
    SVCONV_FORM_SEPARABLE_REGROUPED = 3
};
/* SEPARABLE (Gaussian bases, 1 <= half_width <= 15): each Gaussian basis is a
 * product f_i(u) f_j(v) of one-dimensional factors (the L1 norm of the
 * product is the product of the norms), so T_n = f_j (x)_y (f_i (x)_x R): a
 * row pass per factor f_i of a family, then a column pass per basis.  With
 * SVCONV_FP32, SVCONV_BF16 or SVCONV_FP16 the passes run in float64 on the
 * vector units (row responses held in float32); with SVCONV_FP16X3,
 * SVCONV_BF16X3 or SVCONV_FP16X2 the forward passes run on the matrix cores
 * as banded Toeplitz products of 16-bit hi/lo parts with float32
 * accumulation (the coefficient weighting and the sum over the bases in
 * float32 on the vector units, the pedestal restore in float64).  In this
 * form svconv_backward, svconv_normal_matrix, svconv_gn_step and
 * svconv_pcg_fit also go through the factors.  With SVCONV_FP16X3 or
 * SVCONV_BF16X3, svconv_backward runs both adjoints on the matrix cores:
 * the adjoint in R in bf16 hi/lo parts for both (they keep the float32 range
 * of c_n gD; the correlation as the convolution with the mirrored factors
 * f_e(-w) = (-1)^e f_e(w)), the adjoint in a as the forward's passes in the
 * plan's split precision with moment sums in place of the epilogue.  At the
 * other precisions, and in the fit entry points (whose steps go through the
 * ill-conditioned normal matrix), the adjoints run in float64, and the basis
 * responses of the normal matrix always do (the float64 adjoint in a falls
 * back to the dense matrix-core product when its per-round moments do not
 * fit in LDS).  The adjoints in a sum with atomics, so repeated calls agree to
 * float64 rounding rather than bit for bit.  EUNSUPPORTED for delta-basis
 * plans. */

/* SEPARABLE_REGROUPED (Gaussian bases, 1 <= half_width <= 12, spatial
 * degree <= 2, precision SVCONV_FP16X3, SVCONV_BF16X3 or SVCONV_FP16X2; other
 * precisions return EUNSUPPORTED): the coefficients are folded into per-call
 * column filters, sum_n c_n T_n = sum_m P_m Z_m with
 * Z_m = sum_r g_{r,m} (x)_y (f_r (x)_x R) and g_{r,m} = sum_j a[n(r,j)][m] f_j
 * over the column factors j of row factor r's family (exact, since P_m
 * depends only on the output pixel).  One row pass per row factor and one
 * column pass per row factor and spatial term, both as Toeplitz products of
 * hi/lo parts on the matrix cores with float32 accumulation; no per-basis
 * work outside the matrix cores.  svconv_backward and the fit entry points
 * take the same paths as in the SEPARABLE form. */

/*
 * Create a plan for images of height x width with a (2 half_width + 1)^2
 * kernel, n_gauss Gaussian families (host arrays sigmas[n_gauss] in pixels,
 * degrees[n_gauss]) and spatial polynomial degree spatial_degree (Sec. 2,
 * Eq. 2, Eq. 3).  Builds the basis in float64 on the host and uploads its
 * tables; allocates all scratch.  Uses the current HIP device.
 * Limits: 0 <= half_width <= 31, 0 <= spatial_degree <= 6, N*M <= 1024,
 * N <= 64 (BASIS form).  EINVAL for bad values, EUNSUPPORTED beyond limits.
 */
int svconv_plan_create(svconv_plan** out, int height, int width, int half_width, int n_gauss,
                       const double* sigmas, const int* degrees, int spatial_degree,
                       int precision);

/*
 * Create a plan with the Dirac delta basis (Sec. 2: one basis function per
 * kernel pixel, k^2 bases with k^2 spatial polynomials): basis
 * n = (v + h) k + (u + h) is 1 at kernel pixel (u, v) and 0 elsewhere, so
 * K(x,y)[u,v] = sum_m a[n(u,v)][m] P_m(x,y) and a is [k^2][M].  The plan
 * starts in SVCONV_FORM_REGROUPED; the basis form and the normal matrix need
 * k^2 <= 64.  Limits as svconv_plan_create (k^2 M <= 1024).
 */
int svconv_plan_create_dfb(svconv_plan** out, int height, int width, int half_width,
                           int spatial_degree, int precision);

/* Crop support: the image is the sub-array at (x0, y0) of a frame of
 * frame_width x frame_height pixels; spatial terms use frame coordinates.
 * EINVAL unless 0 <= x0, 0 <= y0, x0 + width <= frame_width, y0 + height
 * <= frame_height. */
int svconv_plan_set_frame(svconv_plan* plan, int x0, int y0, int frame_width, int frame_height);

/* Stream for all later work of the plan (a hipStream_t; NULL = default). */
int svconv_plan_set_stream(svconv_plan* plan, void* stream);

/* Select the arithmetic (enum svconv_precision) for later calls. */
int svconv_plan_set_precision(svconv_plan* plan, int precision);

/* Select the contraction form (enum svconv_form) for later calls. */
int svconv_plan_set_form(svconv_plan* plan, int form);

/* Pedestal s subtracted from R before the contraction and restored exactly
 * through s * sum_n c_n sum(B_n); it shrinks the magnitude of partial sums
 * (default 0).  EINVAL if not finite. */
int svconv_plan_set_pedestal(svconv_plan* plan, float pedestal);

/* Number of bases N and spatial terms M (host outputs; either may be NULL). */
int svconv_plan_sizes(const svconv_plan* plan, int* n_basis, int* n_spatial);

/* Copy the float64 basis table B[n][v+h][u+h] to host memory host_out
 * (N * k * k doubles). */
int svconv_plan_get_basis(const svconv_plan* plan, double* host_out);

/* Free the plan and everything it owns (synchronises its stream).  NULL is
 * accepted. */
int svconv_plan_destroy(svconv_plan* plan);

/* out = R (x) K(x,y)  (Eq. 1 without the subtraction, Eq. 2).
 * R, out: [height][width]; a: [N][M].  out must not alias R. */
int svconv_forward(svconv_plan* plan, const float* R, const float* a, float* out);

/* D = (R (x) K(x,y)) - I  (Eq. 1).  D may alias I but not R. */
int svconv_difference(svconv_plan* plan, const float* R, const float* I, const float* a,
                      float* D);

/* Adjoint of svconv_difference for a loss L(D), given gD = dL/dD:
 *   gR[q]    = sum_{u,v} gD(q+(u,v)) K(q+(u,v))[u,v]         (float32, [H][W])
 *   ga[n][m] = sum_p gD(p) P_m(p) (B_n (x) R)(p)              (float64, [N][M])
 * (dL/dI = -gD needs no kernel.)  Either output may be NULL to skip it.
 * gR must not alias R or gD. */
int svconv_backward(svconv_plan* plan, const float* R, const float* a, const float* gD,
                    float* gR, double* ga);

/* Loss of the least-squares fit (OIS, Sec. 2) and its gradient in D:
 * L = sum_{p in mask} D(p)^2, gD = 2 D 1_mask.  mask: uint8 [H][W] (nonzero =
 * in), or NULL for the interior (pixels at least h from every edge).
 * loss: device float64 scalar (may be NULL); gD may alias D. */
int svconv_loss_grad(svconv_plan* plan, const float* D, const unsigned char* mask, float* gD,
                     double* loss);

/* Normal matrix of the fit: JtJ[(n,m)][(n',m')] = sum_{p in mask}
 * P_m P_m' T_n T_n' with T_n = B_n (x) R, index (n,m) -> n*M + m; float64
 * [NM][NM] device.  mask as in svconv_loss_grad.  With a background the
 * matrix is [(N+1)M][(N+1)M] and T_N = 1.  Allocates its band scratch on
 * the first call (and grows it when a later call needs more). */
int svconv_normal_matrix(svconv_plan* plan, const float* R, const unsigned char* mask,
                         double* JtJ);

/* Normal equations of the fit (OIS least squares, Sec. 2; D is linear in a
 * by Eq. 2 - Eq. 3, D = J a - I with columns J_(n,m) = P_m T_n):
 *   JtJ as svconv_normal_matrix, and rhs[(n,m)] = sum_{p in mask} P_m T_n I,
 * both float64 device arrays ([NM][NM] and [NM], NM = (N + bg) M), from the
 * same float32 basis-response planes in one pass over the image.  I: float32
 * [H][W] device.  Needs N + bg + 1 <= 64 (SVCONV_EUNSUPPORTED otherwise).
 * Allocates its band scratch on the first call, as svconv_normal_matrix. */
int svconv_normal_equations(svconv_plan* plan, const float* R, const float* I,
                            const unsigned char* mask, double* JtJ, double* rhs);

/* In-place Cholesky factorisation A = L L^T of an n x n float64 device
 * matrix (lower triangle of A is overwritten with L; the strict upper
 * triangle is zeroed).  Synchronises the plan's stream; returns
 * SVCONV_ENOTSPD if a pivot is not positive. */
int svconv_cholesky_factor(svconv_plan* plan, double* A, int n);

/* x = (L L^T)^-1 rhs for a factor from svconv_cholesky_factor; float64
 * device vectors of length n.  x may alias rhs. */
int svconv_cholesky_solve(svconv_plan* plan, const double* L, const double* rhs, double* x,
                          int n);

/* One Gauss-Newton iteration of the fit of a to min sum_mask D^2:
 * D = R (x) K(a) - I; ga = dL/da; delta = (JtJ)^-1 ga / 2; a -= delta.
 * With a background (svconv_plan_set_background) a64, a32 and L cover
 * (N + 1) M coefficients and D includes bg.
 * a64: float64 [N][M] master copy (updated); a32: float32 copy written from
 * it before the forward; D: float32 [H][W] output of this iteration's
 * residual; L: Cholesky factor of JtJ.  host_stats (host, 2 doubles, may be
 * NULL) receives (L before the step, ||delta||_2); when given, the call
 * synchronises the plan's stream. */
int svconv_gn_step(svconv_plan* plan, const float* R, const float* I, const unsigned char* mask,
                   const double* L, double* a64, float* a32, float* D, double* host_stats);

/* One Newton step of the least-squares fit on the normal equations from
 * svconv_normal_equations: D and its loss at the current a (as
 * svconv_gn_step), then g = JtJ a - rhs (= J^T D, float64), delta = (L L^T)^-1 g,
 * a -= delta.  D is linear in a, so the first step reaches the solution of
 * the normal equations and later steps are iterative refinement in float64,
 * independent of the forward pass's precision.  A: JtJ (unfactored), L: its
 * Cholesky factor, rhs: J^T I, all float64 device.  Other arguments and
 * host_stats as in svconv_gn_step. */
int svconv_ls_step(svconv_plan* plan, const float* R, const float* I, const unsigned char* mask,
                   const double* A, const double* L, const double* rhs, double* a64, float* a32,
                   float* D, double* host_stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * difference image D = (R (x) K) - I in the SEPARABLE_REGROUPED form without
 * a plan.  The arguments are those of svconv_plan_create and
 * svconv_difference together: image size, half-width, Gaussian families (HOST
 * arrays sigmas[n_gauss], degrees[n_gauss]), spatial degree, precision
 * (SVCONV_FP16X3, SVCONV_BF16X3 or SVCONV_FP16X2), pedestal, the device images
 * R, I, D (float32 [height][width]), a (float32 [N][M]) and the stream
 * (a hipStream_t; NULL = default).  Spatial terms are taken over the image
 * itself (no crop frame).  The call allocates nothing: every table (the
 * one-dimensional factors, the basis sums, the row- and column-pass
 * fragments) is built on the device, on `stream`, in one static 512 KiB
 * scratch array per GPU, which holds its contents until the process ends.
 * Limits: 1 <= half_width <= 12, spatial_degree <= 2, n_gauss <= 8, every
 * sigma > 0, degree <= 9, N <= 64 and sum_g (degree_g + 1) <= 32; beyond
 * them EUNSUPPORTED, before any HIP call (as are the EINVAL checks).  Calls
 * on one GPU share that GPU's scratch array: calls that overlap in time
 * (from several threads, or on streams that run concurrently) race and must
 * be serialised by the caller.  D may alias I but not R.  Asynchronous like
 * svconv_difference.
 */
int svconv_difference_noalloc(int height, int width, int half_width, int n_gauss,
                              const double* sigmas, const int* degrees, int spatial_degree,
                              int precision, float pedestal, const float* R, const float* I,
                              const float* a, float* D, void* stream);

/*
 * Optimal Image Subtraction on isolated stars (Sec. 2: the least-squares
 * kernel fit takes isolated stars of the reference as its source).
 */

/* Stamp mask of isolated stars of R.  A pixel p is a stamp centre when R(p)
 * is strictly larger than each of its neighbours inside the image, R(p) -
 * sky > threshold, p is at least `margin` pixels from every edge, and no
 * other such local maximum q within |qx - px|, |qy - py| <= r_iso has
 * R(q) - sky >= frac (R(p) - sky); every comparison is made in float64 on
 * the float32 values.  mask (device uint8 [H][W], written) is 1 inside the
 * (2 stamp_half + 1)^2 box of any centre, 0 elsewhere.  n_centres (HOST, may
 * be NULL) receives the number of centres; when given, the call synchronises
 * the plan's stream.  Limits: frac > 0, 1 <= r_iso <= 64,
 * 0 <= stamp_half <= 64, margin >= 0.  Uses the plan's gradient scratch. */
int svconv_stamp_mask(svconv_plan* plan, const float* R, double sky, double threshold, double frac,
                      int r_iso, int margin, int stamp_half, unsigned char* mask, int* n_centres);

/* Fit model with a differential background polynomial (enable = 1):
 * D = (R (x) K) + bg - I, bg(x,y) = sum_m b[m] P_m(x,y) with the plan's
 * spatial terms.  The fit entry points (svconv_normal_matrix,
 * svconv_gn_step, svconv_pcg_fit) then work on (N + 1) M coefficients: a
 * [N][M] followed by b [M]; the normal matrix treats the background as one
 * more basis whose response is the constant 1.  svconv_forward,
 * svconv_difference and svconv_backward are unchanged.  EUNSUPPORTED unless
 * N + 1 <= 64 and (N + 1) M <= 1024. */
int svconv_plan_set_background(svconv_plan* plan, int enable);

/* D += sum_m b[m] P_m (b: float32 [M] device). */
int svconv_add_background(svconv_plan* plan, const float* b, float* D);

/* Whole-image least-squares fit by conjugate gradients on the normal
 * equations J^T mask J a = J^T mask I, preconditioned by (L L^T)^-1 for a
 * Cholesky factor L of any SPD matrix of the fit's size (typically the
 * normal matrix of the stamp mask, which takes far fewer Gram products than
 * the whole image's).  Each iteration costs one forward pass of the search
 * direction and one adjoint in a (plus the background terms).  a64 (float64,
 * updated) is the starting point and the result; a32 receives its float32
 * copy; D (float32 [H][W]) is scratch and receives the residual at the
 * result.  host_residuals (HOST, may be NULL) receives ||J^T mask (I - J a)||
 * after each of the `iters` iterations; when given, the call synchronises
 * the plan's stream.  D must not alias R or I.  Uses the plan's vector and
 * gradient scratch. */
int svconv_pcg_fit(svconv_plan* plan, const float* R, const float* I, const unsigned char* mask,
                   const double* L, int iters, double* a64, float* a32, float* D,
                   double* host_residuals);

/*
 * Streamed tiles (Sec. 4: asynchronous transfers between page-locked host
 * memory and the device on streams; Sec. 3: a mosaic camera of many equal
 * tiles).  A pipeline runs svconv_difference on many tiles of the plan's
 * size whose images live in HOST memory: tile t is copied in, differenced
 * and copied back while the neighbouring tiles are in transfer.  It uses the
 * plan's tables, precision, form, frame and pedestal, but its own three
 * streams (copies in, compute, copies out); the plan's stream is unchanged.
 * A plan must not be used elsewhere while one of its pipelines runs.
 */
typedef struct svconv_pipeline svconv_pipeline;

/* Page-locked host memory for tile buffers (the copies overlap compute only
 * from such memory; pageable buffers work but serialise).  *out is a HOST
 * pointer owned by the caller, released with svconv_host_free.  EINVAL for
 * bytes == 0, ENOMEM if the allocation fails. */
int svconv_host_alloc(size_t bytes, void** out);

/* Release memory from svconv_host_alloc (NULL is accepted). */
int svconv_host_free(void* host_ptr);

/* Create a pipeline over `plan` with `depth` (1..8) slots of device buffers:
 * depth * (2 H W + N M) floats, allocated here.  The plan must outlive the
 * pipeline. */
int svconv_pipeline_create(svconv_plan* plan, int depth, svconv_pipeline** out);

/* For t = 0 .. n_tiles-1: D_host[t] = R_host[t] (x) K(a_host[t]) - I_host[t]
 * (Eq. 1).  All four arrays hold n_tiles HOST pointers: images float32
 * [H][W], coefficients float32 [N][M].  D_host[t] may alias I_host[t].
 * Blocking: returns when every D is in host memory.  EINVAL (before any HIP
 * call) for a NULL array or tile pointer or n_tiles < 0; n_tiles == 0 does
 * nothing. */
int svconv_pipeline_run(svconv_pipeline* pipeline, int n_tiles, const float* const* R_host,
                        const float* const* I_host, const float* const* a_host,
                        float* const* D_host);

/* Free the pipeline's buffers, events and streams (NULL is accepted). */
int svconv_pipeline_destroy(svconv_pipeline* pipeline);

/* Static description of a status code. */
const char* svconv_strerror(int status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* svconv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SVCONV_H */
