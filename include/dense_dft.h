/*
 * dense_dft.h -- C ABI of the MI355X (gfx950) alpha-dense DFT library.
 *
 * The transform (Xu, "Adaptive Frequency Bin Interval in FFT via Dense
 * Sampling Factor alpha", Section 2, eq. (7) first line on the grid of
 * eq. (6), forward factor T/N of eq. (2), W_N^{mn} = exp(-2 pi i mn / N) as
 * fixed in Section 3):
 *
 *     X_m = (T/N) * sum_{n=0}^{N-1} x_n * exp(-2 pi i m n / (alpha N)),
 *     m = 0 .. alpha*N - 1,
 *
 * i.e. a signal of N samples taken at interval T/N on [0, T] is mapped to
 * alpha*N spectral bins spaced 1/(alpha T) apart.  The library computes it
 * in the FFT-structured form of Section 3 (eq. (9)-(13)): for integer alpha,
 * with m = alpha*k + j, X_{alpha k + j} is the length-N FFT of the
 * pre-twiddled sequence x_n * W_{alpha N}^{j n}, so the work is alpha
 * interleaved length-N FFTs rather than one zero-padded alpha*N FFT.
 *
 * General conventions (all entry points):
 *   - Every function returns dd_status; DD_OK == 0.  On any other status the
 *     out-parameters are left as documented (plan handles are set to NULL).
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns them and the library never frees caller memory.
 *   - Layout: x is [batch][N] contiguous, X is [batch][alpha*N] contiguous.
 *     Complex values are interleaved (re, im).  Bins are in natural order
 *     m = 0 .. alpha*N-1 (no shift; the upper half holds the negative
 *     frequencies, Section 2).
 *   - Input dtypes: DD_F32 (real float), DD_C64 (complex float),
 *     DD_F64 (real double), DD_C128 (complex double).  The output is
 *     complex64 for DD_F32 / DD_C64 and complex128 for DD_F64 / DD_C128.
 *   - Execution calls only enqueue work on the given HIP stream (NULL = the
 *     default stream) and return at once; device faults surface at the
 *     caller's synchronisation or as DD_ERR_DEVICE from a later call.
 *   - Thread safety: a plan is immutable after creation; concurrent
 *     executions of one plan must use distinct workspaces.
 */
#ifndef DENSE_DFT_H
#define DENSE_DFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dd_dtype {
    DD_F32 = 0,
    DD_C64 = 1,
    DD_F64 = 2,
    DD_C128 = 3
} dd_dtype;

typedef enum dd_status {
    DD_OK = 0,
    DD_ERR_INVALID = 1,      /* bad argument: null/misaligned pointer, N<1, T<=0, overlap ... */
    DD_ERR_UNSUPPORTED = 2,  /* alpha not an integer >= 1, N with a prime factor > 5, size limits */
    DD_ERR_NOMEM = 3,        /* device or host allocation failed */
    DD_ERR_DEVICE = 4,       /* a HIP runtime call failed */
    DD_ERR_BUSY = 5,         /* serving: queue full / result not ready */
    DD_ERR_TOO_LARGE = 6,    /* serving: the request can never fit the memory budget */
    DD_ERR_TIMEOUT = 7,      /* serving: wait timed out */
    DD_ERR_CLOSED = 8        /* serving: server shut down */
} dd_status;

/* Plan flags.  Twiddle factors are always indexed by an exponent reduced
 * exactly in integers (q = j*n, k*n ... mod the transform length).
 *   DD_TWIDDLE_FP64: each factor is generated on the GPU in double precision
 *                    (sin/cos of 2 pi q / L) and rounded once to the working
 *                    precision (the default).
 *   DD_TWIDDLE_FP32: the angle and sin/cos are evaluated in single precision
 *                    from the same exact integer q (the low-precision variant
 *                    the precision study compares against).  Ignored for
 *                    double-precision dtypes. */
#define DD_TWIDDLE_FP64 0u
#define DD_TWIDDLE_FP32 1u

typedef struct dd_plan *dd_plan_t;

/* Create a plan for `batch` transforms of length N with integer dense factor
 * alpha and record duration T (seconds; only the T/N output factor depends
 * on it).  Validates the arguments, factors N (radices 2, 3, 4, 5, 8, 16),
 * chooses the kernel schedule (one fused pass when the alpha*N spectrum of a
 * signal fits on chip, otherwise two passes N = N1*N2), allocates and
 * generates the device twiddle tables on the current device, and
 * synchronises once.
 *   out    : receives the plan handle (NULL on failure).
 *   N      : samples per signal, 1 <= N, alpha*N <= 2^31.
 *   alpha  : dense sampling factor, integer >= 1 (alpha < 1 and non-integer
 *            alpha -> DD_ERR_UNSUPPORTED).
 *   T      : finite, > 0.
 *   batch  : number of signals, >= 1, batch*alpha*N must fit int64.
 *   dtype  : input dtype (see above).
 *   flags  : DD_TWIDDLE_FP64 or DD_TWIDDLE_FP32.
 * Errors: DD_ERR_INVALID, DD_ERR_UNSUPPORTED, DD_ERR_NOMEM, DD_ERR_DEVICE. */
dd_status dense_dft_plan(dd_plan_t *out, int64_t N, int32_t alpha, double T,
                         int64_t batch, dd_dtype dtype, uint32_t flags);

/* Bytes of device scratch one execution needs (0 for single-pass plans).
 * The plan owns a default workspace of this size. */
dd_status dense_dft_workspace_size(dd_plan_t plan, size_t *bytes);

/* Enqueue the transform of all `batch` signals of the plan on `stream`.
 *   x         : device, [batch][N] of the plan's input dtype, aligned to the
 *               element size (8 for C64/F64, 16 for C128, 4 for F32).
 *   X         : device, [batch][alpha*N] complex64/complex128 output, aligned
 *               to 8 / 16 bytes; must not overlap x.
 *   workspace : device scratch of dense_dft_workspace_size() bytes, or NULL
 *               to use the plan's own (then executions of this plan must not
 *               overlap in time).
 *   stream    : hipStream_t, NULL for the default stream.
 * Errors: DD_ERR_INVALID (null / misaligned / overlapping pointers),
 *         DD_ERR_DEVICE (kernel launch failed). */
dd_status dense_dft_exec(dd_plan_t plan, const void *x, void *X,
                         void *workspace, void *stream);

/* Free the plan's device tables and workspace (synchronises its device). */
dd_status dense_dft_destroy(dd_plan_t plan);

/* Query the schedule a plan chose: passes (1 or 2), N1, N2 (N = N1*N2; N2 = 1
 * for one pass).  Any pointer may be NULL. */
dd_status dense_dft_plan_info(dd_plan_t plan, int32_t *passes, int64_t *N1,
                              int64_t *N2);

/* Per-launch timing with HIP events, for benchmarks.  After
 * dense_dft_profile_begin(plan, max_launches), every kernel launch the plan
 * enqueues (up to max_launches) is bracketed by a pair of events recorded on
 * the launch stream; the work itself is unchanged.  dense_dft_profile_end
 * waits for the last recorded event, writes up to `cap` entries of kinds[]
 * (1 = single-pass kernel, 2 = pass 1, 3 = pass 2) and ms[] (duration of
 * each launch in milliseconds), sets *count, and turns profiling off.
 * Errors: DD_ERR_INVALID (null plan / arrays, max_launches < 1),
 *         DD_ERR_NOMEM, DD_ERR_DEVICE. */
dd_status dense_dft_profile_begin(dd_plan_t plan, int32_t max_launches);
dd_status dense_dft_profile_end(dd_plan_t plan, int32_t *kinds, float *ms,
                                int32_t cap, int32_t *count);

/* Static text for a status code. */
const char *dense_dft_status_string(dd_status status);

/* Library version as major*10000 + minor*100 + patch. */
int32_t dense_dft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DENSE_DFT_H */
