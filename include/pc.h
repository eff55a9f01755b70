/*
 * pc.h - convolution-product expansions on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the convolution-product expansion of order m
 * (introduction, eq. 1.4)
 *
 *     H_m u = sum_{k=1..m} h_k * (w_k . u)
 *
 * and its adjoint  H_m^* v = sum_k w_k . (h~_k * v),  h~_k[l] = h_k[-l],
 * on periodic 1D signals of N samples and periodic 2D images of N1 x N2
 * pixels (the extension of section 6.2).  "*" is the circular convolution of
 * section 3.5, written 0-based:  (h * z)[i] = sum_j h[(i - j) mod N] z[j];
 * in 2D the index pairs are taken modulo (N1, N2).  "." is the pointwise
 * product.  Windows w_k and impulse responses h_k are real; h_k is given in
 * lag layout (index 0 = zero lag, negative lags wrap to the end).  Results
 * are computed in FP32 with the DFT identity of section 3.5; no
 * normalisation is applied to h_k, the 1/N of the inverse transform is the
 * only scale.
 *
 * Conventions for every call:
 *   - every function returns a pc_status; nothing aborts or throws;
 *   - PC_ERROR_* codes leave a thread-local message in pc_last_error();
 *   - "device" pointers are HIP device memory on the plan's device,
 *     "host" pointers are ordinary host memory;
 *   - streams are hipStream_t values passed as void* (NULL = null stream);
 *   - layouts are row-major and contiguous: a batch of 1D signals is
 *     batch x N floats, a batch of images batch x N1 x N2 floats (N2
 *     contiguous).
 */
#ifndef PC_H_
#define PC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pc_plan_s* pc_plan;

typedef enum {
  PC_SUCCESS = 0,
  PC_ERROR_INVALID_VALUE = 1, /* null pointer, bad count, aliasing, ... */
  PC_ERROR_UNSUPPORTED = 2,   /* valid request this build has no kernel for */
  PC_ERROR_OUT_OF_MEMORY = 3, /* device allocation failed */
  PC_ERROR_HIP = 4,           /* a HIP runtime call failed (message has the HIP error) */
  PC_ERROR_INVALID_PLAN = 5   /* null, destroyed or foreign plan handle */
} pc_status;

/* Window formats. */
enum {
  /* m dense windows: m x N floats (1D) or m x N1 x N2 floats (2D). */
  PC_W_DENSE = 0,
  /* 2D only: a tensor grid of separable windows
   *   w_{k1*m_cols + k2}[n1, n2] = a_{k1}[n1] * b_{k2}[n2],
   * with m = m_rows * m_cols.  The buffer holds the m_rows row-axis factors
   * a (m_rows x N1 floats) followed by the m_cols column-axis factors b
   * (m_cols x N2 floats). */
  PC_W_SEPARABLE = 1
};

/* Plan flags. */
enum {
  /* Allocate, at plan creation, the workspace pc_grad_spectra and
   * pc_backward need (one spectrum-sized buffer), and keep the windowed
   * spectra of pc_apply_save calls within the plan's budget (default 1 GiB,
   * pc_plan_set_budget); without it the spectra gradients return
   * PC_ERROR_INVALID_VALUE. */
  PC_PLAN_GRADIENTS = 1u,
  /* The plan represents the product-convolution expansion of the
   * introduction (eq. 1.3) instead of the convolution-product one:
   *     G_m u = sum_k w_k . (h_k * u),   G_m^* v = sum_k h~_k * (w_k . v),
   * with the same windows, impulse responses, layouts and sizes.  pc_apply
   * evaluates G_m, pc_apply_adjoint G_m^*; the spectra calls still read and
   * write F^* h_k, and pc_grad_spectra differentiates through G_m.  Since
   * G_m is the adjoint of the convolution-product operator built on the
   * flipped responses h~_k, such a plan runs the same kernels with the two
   * directions exchanged. */
  PC_PLAN_PRODUCT_CONVOLUTION = 2u,
  /* 2D: always evaluate on the full N1 x N2 grid.  Without this flag, a 2D
   * plan whose windows and impulse responses have small supports is
   * evaluated section by section (the compact-support complexity lemma of
   * section 3.5, Lemma 3.2): term k runs on an M1 x M2 section with
   * M >= p + q - 1 per axis (p, q: the circular supports of w_k and h_k),
   * and the sections are added into the result.  The plan takes this route
   * only when it is estimated to be at least twice as cheap (never for a
   * product-convolution plan with gradients); pc_plan_query reports it as
   * path 3 and pc_plan_sections lists the sections.  A sectioned plan's
   * parameters are its sections' spectra (see the spectra calls), and
   * pc_plan_set_responses returns PC_ERROR_UNSUPPORTED for it.  Every pass
   * skips images beyond the call's batch. */
  PC_PLAN_FULL_GRID = 4u
};

typedef struct {
  int32_t ndim;     /* 1 or 2 */
  int32_t m;        /* number of terms, >= 1 */
  int64_t n0;       /* 1D: N; 2D: N1 (rows) */
  int64_t n1;       /* 1D: must be 1; 2D: N2 (columns, contiguous) */
  int64_t batch;    /* largest number of signals / images per apply call, >= 1 */
  int32_t w_format; /* PC_W_DENSE or PC_W_SEPARABLE */
  int32_t m_rows;   /* separable only: number of row-axis factors */
  int32_t m_cols;   /* separable only: number of column-axis factors */
  uint32_t flags;   /* PC_PLAN_* bits; other bits must be 0 */
} pc_plan_desc;

/* Supported sizes.
 *   1D:  N in {2^a, 3*2^a : 64 <= N <= 8192} (one workgroup per transform)
 *        or N = R*L with L in {4096, 6144, 8192} and R in {2, 4, 8, 16}
 *        (12288 ... 131072; four-step split).  The plan takes the shortest
 *        L whose windows' circular supports all fit in 2 L samples (the
 *        short-support kernels), else the longest L; sizes that are also
 *        a single-transform length take the one-workgroup path.
 *   2D:  N1, N2 in {2^a, 3*2^a : 64 <= N <= 8192}.
 * Other sizes return PC_ERROR_UNSUPPORTED. */

/*
 * pc_plan_create - build the operator H_m of eq. 1.4 on one device.
 *
 *   out      (out) receives the plan handle; set to NULL on failure.
 *   desc     (host) sizes, term count, batch capacity and window format.
 *   windows  (host) the windows w_k in the layout given by desc->w_format.
 *   h        (host) the impulse responses h_k, lag layout: m x N floats
 *            (1D) or m x N1 x N2 floats (2D).
 *   stream   stream used for the plan-time work (the spectra F^* h_k of
 *            section 3.5, computed on the device).
 *
 * The call is synchronous: it returns once the plan is ready.  The plan
 * copies what it needs (windows compacted to their support, spectra,
 * twiddle tables, workspaces sized for desc->batch); the caller may free
 * `windows` and `h` afterwards.  The plan is bound to the device current
 * at creation and may be used from one stream at a time (its workspace is
 * shared by its calls).
 * With PC_PLAN_PRODUCT_CONVOLUTION the plan is G_m of eq. 1.3 instead
 * (see the flag).
 * Errors: INVALID_VALUE (null pointers, ndim not 1/2, m < 1, batch < 1,
 * n1 != 1 in 1D, m != m_rows*m_cols, unknown flag bits), UNSUPPORTED (sizes above),
 * OUT_OF_MEMORY, HIP.
 */
pc_status pc_plan_create(pc_plan* out, const pc_plan_desc* desc, const float* windows, const float* h,
                         void* stream);

/*
 * pc_apply - y = H_m u for `batch` signals (eq. 1.4); y = G_m u (eq. 1.3)
 * for a product-convolution plan.
 *
 *   u, y   (device) batch x N (1D) or batch x N1 x N2 (2D) floats; u is
 *          read only; y is written entirely; the two must not overlap.
 *   batch  0 <= batch <= desc->batch (0 is a no-op).
 *   stream the work is enqueued on this stream; the call returns without
 *          waiting for it.
 * Errors: INVALID_PLAN, INVALID_VALUE (null or overlapping buffers, batch
 * out of range), HIP (launch failure).
 */
pc_status pc_apply(pc_plan plan, const float* u, float* y, int64_t batch, void* stream);

/*
 * pc_apply_adjoint - x = H_m^* v = sum_k w_k . (h~_k * v) for `batch`
 * signals (x = G_m^* v = sum_k h~_k * (w_k . v) for a product-convolution
 * plan).  Same buffer rules, errors and asynchrony as pc_apply.
 */
pc_status pc_apply_adjoint(pc_plan plan, const float* v, float* x, int64_t batch, void* stream);

/*
 * pc_destroy - release the plan and its device memory.  Waits for the
 * device to finish work that may still use the plan.  Destroying a NULL or
 * already destroyed handle returns INVALID_PLAN (a handle that was
 * destroyed must not be used again: its memory is freed).  A plan held by a
 * live batch returns INVALID_VALUE and stays alive.
 */
pc_status pc_destroy(pc_plan plan);

/* Read-only facts about a plan (for tests, benchmarks and tooling). */
typedef struct {
  int32_t path;          /* 0: 1D one workgroup per transform, 1: 1D four-step, 2: 2D full grid,
                            3: 2D sectioned */
  int32_t fft_inner;     /* 1D: inner transform length L (N for path 0); 2D: N1 (largest M1 if sectioned) */
  int32_t fft_outer;     /* 1D four-step: R = N / L; otherwise 1 (2D: N2, largest M2 if sectioned) */
  int32_t n_items;       /* 1D four-step: adjoint work items (one per non-empty term when every support
                            fits in 2 L, else one per L-sample chunk of each support); sectioned: sections */
  int64_t spectra_bytes; /* device bytes of the stored spectra */
  int64_t window_bytes;  /* device bytes of the stored (compacted) windows */
  int64_t workspace_bytes;
  int64_t keep_bytes;    /* device bytes held for the windowed spectra of pc_apply_save (0: recomputed) */
  int64_t spectra_count; /* complex entries of the spectra layout of pc_plan_get_spectra */
} pc_plan_info;

/* pc_plan_query - fill *info.  Errors: INVALID_PLAN, INVALID_VALUE. */
pc_status pc_plan_query(pc_plan plan, pc_plan_info* info);

/*
 * Per-kernel timing.  While tracing is enabled, every kernel launched by
 * pc_apply / pc_apply_adjoint on this plan is bracketed by two HIP events
 * recorded on the launch stream (the events add a few microseconds per
 * launch).  pc_plan_trace_stats waits for the recorded events, folds them
 * into per-kernel statistics and copies up to `capacity` entries into
 * `stats` (host memory); *count receives the number of distinct kernels.
 * pc_plan_trace_reset drops the statistics.  Errors: INVALID_PLAN,
 * INVALID_VALUE (null count, or null stats with capacity > 0), HIP.
 */
typedef struct {
  char kernel[32];  /* kernel family, e.g. "fwd1d_large" */
  int64_t launches;
  double total_ms;
  double min_ms;
  double max_ms;
} pc_kernel_stat;

pc_status pc_plan_set_tracing(pc_plan plan, int32_t enable);
pc_status pc_plan_trace_stats(pc_plan plan, pc_kernel_stat* stats, int32_t capacity, int32_t* count);
pc_status pc_plan_trace_reset(pc_plan plan);

/*
 * Sections of a sectioned plan (path 3), in the plan's order: term k, the
 * section's size, the window box and the impulse response's lag box (origin
 * and extent per axis, origins modulo the image size), and the offset of the
 * section's spectrum in the spectra layout.  Section s evaluates
 * h_k * (w_k . u) restricted to the window box, on an M1 x M2 grid whose
 * origin is the window box origin, with the response shifted by its lag box
 * origin; its output box (p + q - 1 samples per axis) is added into the
 * result at window origin + lag origin.
 */
typedef struct {
  int32_t term;
  int32_t m1, m2;
  int32_t win_o1, win_p1, win_o2, win_p2;
  int32_t lag_o1, lag_q1, lag_o2, lag_q2;
  int64_t spec_offset;
} pc_section_info;
/* pc_plan_sections - *count receives the number of sections (0 unless
 * sectioned); up to `capacity` entries are copied into `info` (host).
 * Errors: INVALID_PLAN, INVALID_VALUE (null count, or null info with
 * capacity > 0). */
pc_status pc_plan_sections(pc_plan plan, pc_section_info* info, int32_t capacity, int32_t* count);

/*
 * Spectra as parameters.  The operator's spectra F^* h_k (section 3.5) can be
 * read and replaced, in the natural layout of a real FFT:
 *   1D: m x (N/2 + 1) complex64 (interleaved re, im), spec[k][f];
 *   2D: m x N1 x (N2/2 + 1) complex64, spec[k][f1][f2] (the layout of a 2D
 *       real FFT over the last axis, then a complex FFT over the first);
 *   sectioned 2D: the sections' spectra one after another, section s an
 *       M1 x (M2/2 + 1) array at spec_offset (pc_plan_sections): the real
 *       FFT of its shifted response on the section grid.  The operator a
 *       sectioned plan applies is the sum of its sections, so these spectra
 *       are its parameters (a section whose spectrum no longer comes from a
 *       response within its lag box is evaluated circularly on its grid).
 *       Product-convolution sectioned plans only export them.
 * The represented h_k are real: on import, the imaginary parts of the 1D DC
 * and Nyquist bins are ignored, as an inverse real transform ignores them;
 * in 2D the imaginary parts discarded after the column transforms (DC and
 * Nyquist columns) are ignored the same way.  Both calls are enqueued on
 * `stream` and return without waiting.  `spec` is device memory.
 * Errors: INVALID_PLAN, INVALID_VALUE (null pointer), HIP.
 */
pc_status pc_plan_set_spectra(pc_plan plan, const void* spec, void* stream);
pc_status pc_plan_get_spectra(pc_plan plan, void* spec, void* stream);

/*
 * pc_grad_spectra - gradient of a scalar loss L with respect to the spectra,
 * given the input u of y = H_m u and the upstream gradient gy = dL/dy:
 *   gspec[k][f] = (c_f / N) sum_b conj(F^*(w_k . u_b)[f]) (F^* gy_b)[f]
 * (for a product-convolution plan, y = G_m u:
 *   gspec[k][f] = (c_f / N) sum_b conj(F^* u_b[f]) (F^*(w_k . gy_b))[f]),
 * N the number of samples per signal, c_f = 1 on the bins of the last axis
 * that stand alone (DC, Nyquist), 2 on those that stand for a conjugate
 * pair; complex convention dL/dRe + i dL/dIm, summed over the batch.  Layout
 * of gspec as for pc_plan_set_spectra.  For a sectioned plan the same
 * formula holds per section on its M1 x M2 grid (N = M1 M2), with u_b the
 * section's window box of u and gy_b its output box of gy (zero elsewhere
 * on the section grid).  The windowed spectra F^*(w_k . u_b)
 * are recomputed from u rather than stored.  The plan must have been
 * created with PC_PLAN_GRADIENTS.  u, gy: device, batch x N floats; gspec:
 * device.  Enqueued on `stream`, returns without waiting; uses the plan's
 * workspace (not concurrently with other calls on the plan).
 * Errors: INVALID_PLAN, INVALID_VALUE (null pointers, batch out of range,
 * plan without PC_PLAN_GRADIENTS), HIP.
 */
pc_status pc_grad_spectra(pc_plan plan, const float* u, const float* gy, void* gspec, int64_t batch,
                          void* stream);

/*
 * The differentiable form of pc_apply (the torch.autograd binding uses it).
 *
 * pc_apply_save - pc_apply that also leaves, in the plan, what pc_backward
 *   needs about u: the row transforms of the windowed inputs (2D paths, as
 *   pc_apply does) and, for a plan with gradients whose windowed spectra
 *   U_k = F^*(w_k . u_b) fit in its budget, U_k themselves.  Same arguments
 *   and errors as pc_apply.
 *
 * pc_backward - for y = H_m u (G_m u) and gy = dL/dy, computes
 *   gu = dL/du = H_m^* gy (G_m^* gy) when gu is not NULL, and the spectra
 *   gradient of pc_grad_spectra into gspec when gspec is not NULL (at least
 *   one of them).  Both come from one transform of gy on the sectioned and
 *   2D paths.  With use_saved != 0 the caller states that u holds the values
 *   it held at the plan's last pc_apply / pc_apply_save call; the plan then
 *   reuses what that call left, if the call had the same u pointer and batch
 *   and no other call on the plan has reused its workspace since (otherwise,
 *   or with use_saved == 0, U_k are recomputed from u).
 *   u, gy: device, batch x N floats; gu: device, must not overlap u or gy;
 *   gspec: device, spectra layout.  Enqueued on `stream`, returns without
 *   waiting.  Errors: INVALID_PLAN, INVALID_VALUE (null u or gy, both
 *   outputs NULL, gspec without PC_PLAN_GRADIENTS, batch out of range,
 *   overlapping buffers), HIP.
 *
 * pc_plan_set_budget - the device bytes the plan may hold to keep U_k
 *   between pc_apply_save and pc_backward (they are recomputed when they do
 *   not fit; 0: always recomputed).  A plan with PC_PLAN_GRADIENTS starts with
 *   1 GiB; pc_plan_query reports the bytes held (keep_bytes).  Synchronous
 *   (allocates or frees; waits for the device before freeing).  Errors:
 *   INVALID_PLAN, INVALID_VALUE (bytes < 0), OUT_OF_MEMORY, HIP.
 */
pc_status pc_apply_save(pc_plan plan, const float* u, float* y, int64_t batch, void* stream);
pc_status pc_backward(pc_plan plan, const float* u, const float* gy, float* gu, void* gspec, int64_t batch,
                      int32_t use_saved, void* stream);
pc_status pc_plan_set_budget(pc_plan plan, int64_t bytes);

/*
 * pc_plan_set_responses - replace the impulse responses h_k of a plan by
 * device data (m x N or m x N1 x N2 floats, lag layout, as for
 * pc_plan_create) and recompute its spectra F^* h_k on the device; the
 * windows are unchanged.  Enqueued on `stream`, returns without waiting; h
 * may be freed once the stream has passed the call.  With the construction
 * calls below it keeps the whole construction of an operator on the device.
 * Errors: INVALID_PLAN, INVALID_VALUE (null h), UNSUPPORTED (sectioned plans,
 * whose sections follow the supports of the responses they were built
 * with), HIP.
 */
pc_status pc_plan_set_responses(pc_plan plan, const float* h, void* stream);

/*
 * Construction of the impulse responses from a time-varying impulse
 * response (TVIR) T(x, y) (section 4).  The windows w_k are given; for every
 * lag x, the coefficients c_k(x) are
 *   pc_construct_project:      the L2 projection of T(x, .) onto the span of
 *                              the windows (section 4.2; with B-spline
 *                              windows the approximation of Corollary 4.3):
 *                              (W W^T) c(x) = W T(x, .)^T on the grid;
 *   pc_construct_interpolate:  the interpolation at m nodes y_i
 *                              (section 4.4): sum_k c_k(x) w_k(y_i) = T(x, y_i);
 * and h_k[x] = c_k(x) / n, n the number of grid points (the quadrature
 * weight of the grid).  Grids are flat: 1D signals of n samples, or 2D
 * images with n = N1 N2 and row-major flat indices for lags, positions and
 * nodes.
 *
 *   n        grid points, a positive multiple of 16.
 *   m        number of windows, 1 <= m <= 128.
 *   rows     number of lags given (the TVIR rows that can be nonzero).
 *   lags     (host) rows distinct flat lag indices in [0, n), lag layout.
 *   tvir     (device, projection) rows x n floats: row r = T(lag r, y_j)
 *            over all positions j; 16-byte aligned.
 *   samples  (device, interpolation) rows x m floats: T(lag r, y_i) at the
 *            m nodes.
 *   nodes    (host, interpolation) m distinct flat positions y_i.
 *   windows  (device) m x n floats; 16-byte aligned for the projection.
 *   h        (device, out) m x n floats: c_k / n at the listed lags, 0 at
 *            every other lag.
 *
 * The contraction W T^T runs on the matrix cores in FP32 (partial sums over
 * chunks of 2048 positions added in float64); the m x m factorisations
 * (Cholesky of the Gram matrix, LU with partial pivoting of the node matrix)
 * and the per-lag solves are float64.  Both calls are synchronous: they
 * return once h is written.  Their workspace (and that of
 * pc_wavelet_transform and pc_plan_create_meyer) comes from a device scratch
 * buffer that the library keeps between calls, one per device, grown when a
 * call needs more (the projection of rows lags needs about
 * 4 rows m (n / 2048 + 4) bytes) and held until the process ends; calls on
 * one device that use it run one after another.
 * Errors: INVALID_VALUE (null pointers, sizes or indices out of range,
 * misaligned buffers, a singular Gram or node matrix), OUT_OF_MEMORY, HIP.
 */
pc_status pc_construct_project(int64_t n, int32_t m, int64_t rows, const float* tvir, const int64_t* lags,
                               const float* windows, float* h, void* stream);
pc_status pc_construct_interpolate(int64_t n, int32_t m, int64_t rows, const float* samples, const int64_t* lags,
                                   const int64_t* nodes, const float* windows, float* h, void* stream);

/*
 * Meyer's operator representation (section 4.5).  The TVIR is expanded in a
 * tensor basis of periodic orthonormal wavelets,
 *   T(x, y) = sum c_{lambda,mu} psi_lambda(x) psi_mu(y),
 * of which a few coefficients are kept; regrouped by mu (the paper's trick
 * equation) this is the convolution-product expansion with windows
 * w_mu = psi_mu and responses h_mu = c~_mu / n,
 * c~_mu = sum_lambda c_{lambda,mu} psi_lambda.
 *
 * Wavelets: the periodic discrete wavelet transform of `levels` levels
 * with the orthonormal lowpass filter `lowpass` (`taps` values, even,
 * <= 20; the highpass filter is g[k] = (-1)^k lowpass[taps-1-k]) on n = 2^J
 * samples; one level maps a (length len) to
 *   lo[i] = sum_k h[k] a[(2i + k) mod len], hi[i] = sum_k g[k] a[(2i + k) mod len],
 * and coefficients are in pyramid order [a_levels, d_levels, ..., d_1], so
 * that index lambda names one basis vector psi_lambda (a row of the
 * orthogonal transform matrix).
 *
 * pc_wavelet_transform - the transform (inverse = 0) or its inverse
 *   (inverse != 0) of `count` vectors; element i of vector b is at
 *   b * dist + i * stride in both `in` and `out` (device; distinct buffers).
 *   A 2D transform is one call over the rows (stride 1, dist n) and one
 *   over the columns (stride n, dist 1).  Synchronous (allocates scratch).
 *
 * pc_plan_create_meyer - a 1D plan (n samples, batch capacity `batch`,
 *   plan flags as for pc_plan_create) for the kept coefficients
 *   c[i] = c_{lam[i], mu[i]} (host arrays of `count` entries, indices in
 *   [0, n), repeated pairs add up).  The windows psi_mu and the responses
 *   c~_mu / n are synthesised on the device; the plan's terms are the
 *   distinct mu in increasing order.  Synchronous, like pc_plan_create.
 *
 * Errors: INVALID_VALUE (null pointers, n not a power of two, levels out of
 * range, bad taps, indices out of range, in == out), UNSUPPORTED (n not a
 * supported 1D size), OUT_OF_MEMORY, HIP.
 */
pc_status pc_wavelet_transform(int32_t inverse, int64_t n, int32_t levels, int32_t taps, const float* lowpass,
                               int64_t count, int64_t stride, int64_t dist, const float* in, float* out,
                               void* stream);
pc_status pc_plan_create_meyer(pc_plan* out, int64_t n, int32_t levels, int32_t taps, const float* lowpass,
                               int64_t count, const int64_t* lam, const int64_t* mu, const float* c, int64_t batch,
                               uint32_t flags, void* stream);

/*
 * pc_wavelet_transform_noalloc - pc_wavelet_transform for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments,
 * results and errors; it calls no allocation routine and does not wait:
 * the work is enqueued on `stream` and the call returns.  Its scratch is a
 * fixed device array of 16 MiB per device (4194304 floats), kept until the
 * process ends and shared by every call of this function on that device, so
 * such calls that overlap on one device (several streams, several host
 * threads) race; calls ordered on one stream do not.  Limit: count * n <=
 * 4194304; larger requests return PC_ERROR_INVALID_VALUE before anything is
 * launched.
 */
pc_status pc_wavelet_transform_noalloc(int32_t inverse, int64_t n, int32_t levels, int32_t taps,
                                       const float* lowpass, int64_t count, int64_t stride, int64_t dist,
                                       const float* in, float* out, void* stream);

/*
 * Uneven batches.  A batch runs many 2D operators of different sizes and
 * term counts together: every pass of the evaluation is one launch per
 * transform length (the work of all instances with that row or column
 * length shares the launch), and the sequence of launches of each direction
 * is captured once into a HIP graph, so that one pc_batch_apply call is one
 * graph launch.  The kernels read each instance's input and output pointers
 * from a device table, so every call may name new buffers.
 *
 *   plans   (host array of count handles) distinct 2D plans, full-grid or
 *           sectioned (a sectioned plan's sections join the launches of
 *           their lengths, followed by the plan's overlap-add into the
 *           call's output; a handle listed twice is rejected: its
 *           instances would share the plan's workspace).  While the batch lives, pc_destroy refuses its
 *           plans, and the plans must not be used by other calls while a
 *           batch call runs (the batch uses their workspaces).
 *           Convolution-product and product-convolution plans may share a
 *           batch.
 *   flags   PC_BATCH_NO_GRAPH: launch the passes directly instead of
 *           through the captured graphs; PC_BATCH_PERSISTENT: one persistent
 *           launch per pass (below).
 *   stream  unused (creation is synchronous).
 * Errors: INVALID_VALUE (count < 1, null array, a repeated plan, a plan that
 * is not 2D, plans on different devices, unknown flags),
 * INVALID_PLAN, OUT_OF_MEMORY, HIP.
 */
typedef struct pc_batch_s* pc_batch;
enum {
  PC_BATCH_NO_GRAPH = 1u,
  /* Persistent passes: one launch per pass (rows in, forward column passes
   * and column transforms, adjoint column passes, rows out) and length group
   * (points per thread 8: 64, 128; 12: 96, 192, 384; 16: 256, 512) instead
   * of one launch per pass and transform length: every block of the pass
   * over all instances of the group's lengths is a work item of a list
   * (longest transforms first) that the launch's workgroups walk with a grid
   * stride.  Other lengths keep their own launches.  Without the flag, a
   * tuning table entry for the batch (PC_TUNE_BATCH_PERSISTENT) decides. */
  PC_BATCH_PERSISTENT = 2u
};
pc_status pc_batch_create(pc_batch* out, int32_t count, const pc_plan* plans, uint32_t flags, void* stream);
/*
 * pc_batch_apply - outputs[i] = H_i inputs[i] for every instance i (G_i for a
 * product-convolution plan); pc_batch_apply_adjoint - outputs[i] =
 * H_i^* inputs[i] (G_i^*).
 *
 *   inputs, outputs  (host arrays of count device pointers) each instance's
 *                    plan batch x N1 x N2 floats (the plan's full batch).  No
 *                    output may overlap another output or any input.
 *   stream           the work is enqueued on this stream; the call returns
 *                    without waiting.
 * When the pointers differ from the previous call's in the same direction,
 * the call first uploads them (a copy of 16 bytes per instance enqueued on
 * `stream`; the host waits only if the previous upload of that direction
 * has not run yet).  Calls on one batch must be ordered (one stream, or
 * synchronised streams): they share the table and the plans' workspaces.
 * Errors: INVALID_VALUE (null or destroyed batch, null arrays or entries,
 * overlapping buffers), HIP.
 */
pc_status pc_batch_apply(pc_batch batch, const float* const* inputs, float* const* outputs, void* stream);
pc_status pc_batch_apply_adjoint(pc_batch batch, const float* const* inputs, float* const* outputs, void* stream);
/* Release the batch (waits for the device first); its plans may then be
 * destroyed.  Errors: INVALID_VALUE (null or destroyed batch), HIP. */
pc_status pc_batch_destroy(pc_batch batch);

/*
 * Tuning table.  Per transform length, the 2D passes come in variants
 * (spectrum loads before or after the transform, prefetching, pipelined
 * tiles, row tiles of 16 or 4 rows, term groups) and 1D four-step plans have
 * a choice of inner length.  Plans and batches take each choice from rules
 * (the runtime's occupancy and register figures for the built kernels),
 * unless the tuning table holds a measured choice for their workload.  The
 * package's tuner times the variants on the device and writes the table;
 * the Python binding loads it at start-up for the device's architecture.
 *
 *   key     the workload: pc_tune_key of a plan description, or
 *           pc_tune_batch_key of a batch's plans (the sections of a sectioned
 *           plan use the plan's key);
 *   knob    a PC_TUNE_* choice; length: the transform length it applies to
 *           (the 1D size for PC_TUNE_FOURSTEP_L);
 *   value   0 / 1 for the variant switches, the term group count for
 *           PC_TUNE_COL_GROUPS (clamped to [1, column factors]), the inner
 *           length for PC_TUNE_FOURSTEP_L (ignored unless it splits N).
 *
 * pc_tune_set replaces the process-wide table (count = 0 clears it); it
 * affects plans and batches created afterwards.  Errors: INVALID_VALUE (null
 * entries with count > 0, count < 0, unknown knob).
 */
enum {
  PC_TUNE_COLS_FWD_LATE = 1,      /* forward column pass: spectrum loaded after the transform */
  PC_TUNE_COLS_ADJ_PREFETCH = 2,  /* adjoint column pass: next spectrum column loaded during the transform */
  PC_TUNE_ROWS_INV_PIPE = 3,      /* row-inverse pass: next plane's tile loaded during the transform */
  PC_TUNE_ROWS_FWD_SMALL = 4,     /* row-forward passes: 4-row tiles instead of 16-row ones */
  PC_TUNE_ROWS_INV_SMALL = 5,     /* row-inverse passes: 4-row tiles instead of 16-row ones */
  PC_TUNE_COL_GROUPS = 6,         /* full-grid forward column pass: term groups */
  PC_TUNE_FOURSTEP_L = 7,         /* 1D four-step: inner transform length */
  PC_TUNE_BATCH_PERSISTENT = 8,   /* batches: persistent passes (length 0) */
  PC_TUNE_SEC_STREAMS = 9,        /* sectioned plans: two launch chains, on two streams (length 0) */
  PC_TUNE_KEEP = 10               /* plans with gradients: keep the windowed spectra within the budget (1, the
                                     rule) or recompute them in every backward (0) (length 0) */
};
typedef struct {
  uint64_t key;
  int32_t knob;
  int32_t length;
  int32_t value;
  int32_t reserved; /* 0 */
} pc_tune_entry;
pc_status pc_tune_set(const pc_tune_entry* entries, int32_t count);
/* The workload key of a plan description, and of a batch of plans (order
 * free).  Errors: INVALID_VALUE (null arguments), INVALID_PLAN. */
pc_status pc_tune_key(const pc_plan_desc* desc, uint64_t* key);
pc_status pc_tune_batch_key(int32_t count, const pc_plan* plans, uint64_t* key);

/* Static text for a status code (never NULL). */
const char* pc_status_string(pc_status status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* pc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PC_H_ */
