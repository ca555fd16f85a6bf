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
 *     Real input still yields all alpha*N bins; the kernels compute about
 *     half of them and write the rest as conjugates, X_{alpha N - m} =
 *     conj(X_m), which then hold exactly.
 *   - Execution calls only enqueue work on the given HIP stream (NULL = the
 *     default stream) and return at once; device faults surface at the
 *     caller's synchronisation or as DD_ERR_DEVICE from a later call.  With
 *     DD_DEBUG set in the environment, a kernel launch that HIP refuses is
 *     reported on stderr with its grid, block and LDS size.
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
    DD_ERR_UNSUPPORTED = 2,  /* alpha not an integer >= 1, N not of the built lengths, size limits */
    DD_ERR_NOMEM = 3,        /* device or host allocation failed */
    DD_ERR_DEVICE = 4,       /* a HIP runtime call failed */
    DD_ERR_BUSY = 5,         /* serving: queue full / result not ready */
    DD_ERR_TOO_LARGE = 6,    /* serving: the request can never fit the memory budget */
    DD_ERR_TIMEOUT = 7,      /* serving: wait timed out */
    DD_ERR_CLOSED = 8        /* serving: server shut down */
} dd_status;

/* Plan flags.  Twiddle factors are always indexed by an exponent reduced
 * exactly in integers (q = j*n, k*n ... mod the transform length).
 *   DD_TWIDDLE_FP64: each table entry is generated on the GPU in double
 *                    precision (sin/cos of 2 pi q / L) and rounded once to
 *                    the working precision (the default).  The inter-pass
 *                    factor of a two-pass schedule, W_{alpha N}^{m1 n2}, is
 *                    the working-precision product of two such entries
 *                    (W_N^{k1 n2} W_{alpha N}^{j n2}), so it carries up to
 *                    three roundings; every other factor is one entry.
 *   DD_TWIDDLE_FP32: the angle and sin/cos are evaluated in single precision
 *                    from the same exact integer q (the low-precision variant
 *                    the precision study compares against).  Ignored for
 *                    double-precision dtypes. */
#define DD_TWIDDLE_FP64 0u
#define DD_TWIDDLE_FP32 1u
/* Plan flag: allocate no default workspace; every execution of a two-pass
 * plan must then pass one (for callers that carve workspaces from a pool of
 * their own). */
#define DD_NO_WORKSPACE 2u

typedef struct dd_plan *dd_plan_t;

/* Create a plan for `batch` transforms of length N with integer dense factor
 * alpha and record duration T (seconds; only the T/N output factor depends
 * on it).  Validates the arguments, factors N (radices 2, 3, 4, 5, 8, 16),
 * chooses the kernel schedule (the tuning table's entry for the problem
 * class if it has one; else one fused pass when the alpha*N spectrum of a
 * signal takes at most 32 KiB and fits on chip, otherwise two passes
 * N = N1*N2), allocates and
 * generates the device twiddle tables on the current device, and
 * synchronises once.
 *   out    : receives the plan handle (NULL on failure).
 *   N      : samples per signal: 2^a (a <= 24), 3*2^a (a <= 22) or 5*2^a
 *            (a <= 21), the lengths the kernels are built for (N = N1*N2 with
 *            N1 a power of two, 3 or 5 times one, up to 4096, and N2 a power
 *            of two up to 4096); also alpha*N <= 2^31.  In double precision
 *            a pass-1 column of 4096 does not fit a workgroup's LDS, so N1
 *            stays below 4096 there and N = 2^24 is unsupported.
 *   alpha  : dense sampling factor, integer >= 1 (alpha < 1 and non-integer
 *            alpha -> DD_ERR_UNSUPPORTED; alpha = 1/p has its own plan,
 *            dense_dft_plan_decimated).
 *   T      : finite, > 0 (else DD_ERR_INVALID); T/N must be a normal number
 *            in the arithmetic's precision (float for DD_F32 / DD_C64,
 *            double otherwise), else DD_ERR_UNSUPPORTED: the kernels scale
 *            every bin by it.
 *   batch  : number of signals, >= 1, batch*alpha*N must fit int64.
 *   dtype  : input dtype (see above).
 *   flags  : DD_TWIDDLE_FP64 or DD_TWIDDLE_FP32, optionally | DD_NO_WORKSPACE.
 * Errors: DD_ERR_INVALID, DD_ERR_UNSUPPORTED, DD_ERR_NOMEM, DD_ERR_DEVICE. */
dd_status dense_dft_plan(dd_plan_t *out, int64_t N, int32_t alpha, double T,
                         int64_t batch, dd_dtype dtype, uint32_t flags);

/* Plan the transform with alpha = 1/p (Section 2, the case alpha < 1): N
 * samples to N/p bins spaced p/T apart,
 *     X_m = (T/N) * sum_{n<N} x_n * exp(-2 pi i m n / (N/p)),  m < N/p.
 * The kernel has period N/p in n, so an execution folds the signal,
 * x'_r = sum_{k<p} x_{r + k N/p} (into the workspace, summed in double
 * precision), then runs the plain transform of length N/p (a plan with
 * alpha = 1, chosen by the planner or the tuning table).  A one-way
 * transform: dense_dft_exec_inverse returns DD_ERR_UNSUPPORTED.
 *   p      : integer >= 1 dividing N; N/p must be a built length (as N of
 *            dense_dft_plan).  p = 1 gives the plain alpha = 1 plan.
 *   Other arguments and errors as dense_dft_plan; the plan executes with
 *   dense_dft_exec (x [batch][N], X [batch][N/p]); its workspace holds the
 *   folded signals as well. */
dd_status dense_dft_plan_decimated(dd_plan_t *out, int64_t N, int32_t p, double T,
                                   int64_t batch, dd_dtype dtype, uint32_t flags);

/* Bytes of device scratch one execution needs (0 for single-pass plans):
 * chunk signals of alpha*N1 rows each.  A row holds N2 elements, plus 512
 * bytes when a row takes at least 4 KiB and alpha rows at least 64 KiB (the
 * pad keeps a wavefront's stores off one memory channel), so one signal
 * needs at most 9/8 of its alpha*N output elements.  The plan owns a default
 * workspace of this size unless it was created with DD_NO_WORKSPACE. */
dd_status dense_dft_workspace_size(dd_plan_t plan, size_t *bytes);

/* Enqueue the transform of all `batch` signals of the plan on `stream`.
 *   x         : device, [batch][N] of the plan's input dtype, aligned to the
 *               element size (8 for C64/F64, 16 for C128, 4 for F32).
 *   X         : device, [batch][alpha*N] complex64/complex128 output, aligned
 *               to 8 / 16 bytes; must not overlap x.
 *   workspace : device scratch of dense_dft_workspace_size() bytes, or NULL
 *               to use the plan's own (then executions of this plan must not
 *               overlap in time; DD_ERR_INVALID for a two-pass plan made
 *               with DD_NO_WORKSPACE).
 *   stream    : hipStream_t, NULL for the default stream.
 * Errors: DD_ERR_INVALID (null / misaligned / overlapping pointers),
 *         DD_ERR_DEVICE (kernel launch failed). */
dd_status dense_dft_exec(dd_plan_t plan, const void *x, void *X,
                         void *workspace, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * forward transform of dense_dft_exec, with the two-pass scratch taken from
 * a fixed device array of DD_STATIC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends, instead of a workspace.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the first call on a device looks the array's address up once.
 * A batch runs in chunks of as many signals as the array holds (each
 * signal's arithmetic is that of dense_dft_exec: the results are identical).
 * Nothing in the array needs to start at zero (pass 1 writes every element
 * pass 2 reads); it keeps the last call's contents.
 * Every call on a device shares that device's array: calls whose executions
 * overlap in time on one device (other streams, other host threads) race
 * and corrupt each other's results; order them on one stream.  The plan
 * itself (made beforehand) owns its twiddle tables; create it with
 * DD_NO_WORKSPACE to allocate no workspace at all.
 *   plan, x, X, stream : as dense_dft_exec.
 * Errors: as dense_dft_exec; DD_ERR_TOO_LARGE when one signal's scratch
 *         (alpha*N output elements, and the row pad of
 *         dense_dft_workspace_size) exceeds DD_STATIC_SCRATCH_BYTES;
 *         DD_ERR_UNSUPPORTED for alpha = 1/p plans (dense_dft_plan_decimated). */
#define DD_STATIC_SCRATCH_BYTES (64u << 20)
dd_status dense_dft_exec_static(dd_plan_t plan, const void *x, void *X, void *stream);

/* Enqueue the inverse transform of all `batch` spectra of the plan on
 * `stream` (the reading of eq. (7), second line, with the factor 1/(alpha T)
 * that undoes the forward transform of eq. (2)):
 *     x_n = (1/(alpha T)) * sum_{m<alpha N} X_m * exp(+2 pi i m n / (alpha N)),
 *     n = 0 .. N-1,
 * computed as the adjoint of the plan's schedule: alpha length-N transforms
 * of the subsequences X_{alpha k + j}, each times W_{alpha N}^{-jn}, summed
 * over j (with the plan's own twiddle tables).
 *   X         : device, [batch][alpha*N] complex64 (plans of DD_F32 / DD_C64)
 *               or complex128 (DD_F64 / DD_C128), aligned to its element.
 *   x         : device, [batch][N] complex output of the same precision (also
 *               for plans of real input); must not overlap X.
 *   workspace : as dense_dft_exec (the same size serves both directions).
 *   stream    : hipStream_t, NULL for the default stream.
 * Profiled launches (dense_dft_profile_begin) report kinds 4 (one pass),
 * 5 (pass A) and 6 (pass B).
 * Errors: DD_ERR_INVALID (null / misaligned / overlapping pointers),
 *         DD_ERR_UNSUPPORTED (an alpha = 1/p plan, or 1/(alpha T) not a
 *         normal number in the plan's precision), DD_ERR_DEVICE (kernel
 *         launch failed). */
dd_status dense_dft_exec_inverse(dd_plan_t plan, const void *X, void *x,
                                 void *workspace, void *stream);

/* Free the plan's device tables and workspace (synchronises its device). */
dd_status dense_dft_destroy(dd_plan_t plan);

/* Query the schedule a plan chose: passes (1 or 2), N1, N2 (N = N1*N2; N2 = 1
 * for one pass).  Any pointer may be NULL. */
dd_status dense_dft_plan_info(dd_plan_t plan, int32_t *passes, int64_t *N1,
                              int64_t *N2);

/* ---- Schedules and the tuner ----
 *
 * How a plan runs the transform.  One pass: each block holds the whole
 * alpha*N spectrum of `lines` signals in LDS, and `jgroup` thread groups
 * share each signal, group g computing the pre-twiddled FFTs of j = g,
 * g + jgroup, ... at once with the others.  Two passes, N = N1*N2 (the
 * four-step split of the length-N FFTs of Section 3): pass 1 computes, for
 * every column n2, the alpha-dense DFT of length N1 (this library's
 * transform at size N1) times the inter-pass twiddles into a scratch of
 * alpha*N values; pass 2 computes the length-N2 FFTs of its rows and stores
 * the bins in natural order.  Zero fields take the planner's rule. */
typedef struct dd_sched {
    int32_t passes;   /* 1 or 2 */
    int32_t lines;    /* one pass: signals per block (0: rule) */
    int64_t N1, N2;   /* two passes: N = N1*N2 (one pass: N1 = N, N2 = 1) */
    int32_t jgroup;   /* two passes: values of j per pass-1 block, 1..alpha;
                         one pass: thread groups sharing a signal, each taking
                         its own values of j, 1..alpha (0: rule) */
    int32_t reserved; /* 0 */
    int64_t chunk;    /* two passes: signals per pass pair (0: 128 MiB of scratch) */
} dd_sched;

/* As dense_dft_plan, with the schedule given rather than chosen.
 * Errors: as dense_dft_plan; DD_ERR_UNSUPPORTED if the kernels cannot run N
 * with this schedule (N1*N2 != N, a length not compiled, LDS too small). */
dd_status dense_dft_plan_sched(dd_plan_t *out, int64_t N, int32_t alpha, double T,
                               int64_t batch, dd_dtype dtype, uint32_t flags,
                               const dd_sched *sched);

/* The schedule a plan runs, every field resolved. */
dd_status dense_dft_plan_get_sched(dd_plan_t plan, dd_sched *out);

/* The schedules dense_dft_tune measures for this problem class, the
 * planner's current choice first, every field resolved; up to cap are
 * written, *count receives their number.  Host only: no device memory or
 * launches (the planner's one-pass rule asks the runtime for the kernel's
 * occupancy on the current device, and without a device uses an LDS
 * model, so its first choice can differ between the two).
 * Errors: DD_ERR_INVALID, DD_ERR_UNSUPPORTED (no schedule for N). */
dd_status dense_dft_sched_candidates(int64_t N, int32_t alpha, int64_t batch, dd_dtype dtype,
                                     dd_sched *out, int32_t cap, int32_t *count);

typedef struct dd_tune_info {
    dd_sched best;       /* the fastest schedule measured */
    float ms_best;       /* its time per execution (per batch for the batch kernel) */
    float ms_default;    /* the time of the schedule used before the call */
    int32_t candidates;  /* schedules measured */
    int32_t reserved;
} dd_tune_info;

/* Measure, on the current device, every schedule the kernels can run this
 * problem class with (one pass at each block width; each two-pass split
 * N1*N2 with each j-group), on temporary buffers of the problem's size, and
 * record the fastest in the process's tuning table under (N, alpha,
 * dtype, batch size class floor(log2(batch))).  Later
 * dense_dft_plan calls of that class use it.  Synchronous.
 * Errors: as dense_dft_plan, DD_ERR_NOMEM, DD_ERR_DEVICE. */
dd_status dense_dft_tune(int64_t N, int32_t alpha, int64_t batch, dd_dtype dtype,
                         dd_tune_info *info);

/* The same for the persistent batch kernel and signals of class (N, alpha):
 * one pass or each two-pass split of its compiled lengths, timed on a batch
 * of that class alone (about 2^24 bins).  Later batch plans and servers use
 * the recorded schedule for the class (a server for classes it has not yet
 * met).  Errors: DD_ERR_INVALID, DD_ERR_UNSUPPORTED (no batch-kernel
 * schedule for N), DD_ERR_NOMEM, DD_ERR_DEVICE. */
dd_status dense_dft_tune_batch(int64_t N, int32_t alpha, dd_tune_info *info);

/* Write the tuning table to a text file / merge one into it (entries of the
 * file replace those of the same class; lines of the earlier format, keyed
 * by precision, serve both input dtypes of that precision).  A file named by
 * the environment
 * variable DD_TUNE_DB is merged at the first use of the table.  Entries are
 * re-validated when used: one the kernels cannot run falls back to the
 * planner's rule.  Errors: DD_ERR_INVALID (null path, file not writable /
 * readable). */
dd_status dense_dft_tune_save(const char *path);
dd_status dense_dft_tune_load(const char *path);

/* Empty the tuning table (and skip DD_TUNE_DB from then on). */
dd_status dense_dft_tune_clear(void);

/* Entries in the tuning table. */
dd_status dense_dft_tune_entries(int32_t *plans, int32_t *batch_classes);

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

/* ---- Many signals of uneven N and alpha in one persistent launch ----
 *
 * One descriptor per signal (the problem of Section 2 for each: N samples
 * over [0, T], dense factor alpha):
 *   N, alpha, T : as for dense_dft_plan (integer alpha >= 1, T > 0);
 *   dtype       : input dtype; output complex64 for DD_F32 / DD_C64,
 *                 complex128 for DD_F64 / DD_C128;
 *   x           : device, [N] input of `dtype`;
 *   X           : device, [alpha*N] output, must not overlap any x.
 */
typedef struct dd_desc {
    int64_t N;
    int32_t alpha;
    double T;
    dd_dtype dtype;
    const void *x;
    void *X;
} dd_desc;

typedef struct dd_batch *dd_batch_t;

/* Plan a batch: validate every descriptor, choose each signal's schedule
 * (one pass, or two passes N = N1*N2, as dense_dft_plan does), generate the
 * twiddle tables of every distinct (N, alpha) on the GPU in FP64 (rounded
 * once; DD_TWIDDLE_FP32 as for plans), allocate the scratch of the two-pass
 * signals, and build the device work list: one task per block-sized piece
 * (a single-pass signal, a pass-1 column tile, a pass-2 row block), with
 * the signals ordered largest spectrum first.  FP32/complex64
 * signals of the compiled lengths run in the persistent kernel; the others
 * (FP64 dtypes, other lengths) run as plain per-signal executions after it.
 * The descriptors are copied; the caller keeps ownership of x and X.
 * Errors: DD_ERR_INVALID (count < 1, bad descriptor, null or misaligned
 * pointer, T <= 0), DD_ERR_UNSUPPORTED (as dense_dft_plan), DD_ERR_NOMEM,
 * DD_ERR_DEVICE. */
dd_status dense_dft_batch_plan(dd_batch_t *out, const dd_desc *descs,
                               int32_t count, uint32_t flags);

/* As dense_dft_batch_plan, with every FP32 / complex64 signal run in the
 * batch kernel with the given schedule (passes, N1, N2; the other fields
 * are ignored), as the batch tuner does.  Errors: as dense_dft_batch_plan;
 * DD_ERR_INVALID (null schedule, passes not 1 or 2); DD_ERR_UNSUPPORTED if
 * the kernel cannot run some FP32 signal with it. */
dd_status dense_dft_batch_plan_sched(dd_batch_t *out, const dd_desc *descs, int32_t count,
                                     uint32_t flags, const dd_sched *sched);

/* The schedules the batch kernel can run (N, alpha) with (the candidates of
 * dense_dft_tune_batch); up to cap written, *count receives their number.
 * Host only.  Errors: DD_ERR_INVALID, DD_ERR_UNSUPPORTED. */
dd_status dense_dft_batch_sched_candidates(int64_t N, int32_t alpha, dd_sched *out, int32_t cap,
                                           int32_t *count);

/* Enqueue the whole batch on `stream`: a staging kernel that reads the
 * descriptor table from pinned host memory into device memory and clears the
 * two queue heads, then a persistent queue kernel (a fixed grid sized to the
 * device's occupancy; its blocks take tasks until the queue is empty) over
 * every single-pass and pass-1 task, then, if the batch has two-pass
 * signals, a second, lighter one over every pass-2 task, so no block waits
 * for another; then the
 * plain executions of the fallback signals.  Nothing synchronises, no memory
 * is allocated and no memset is enqueued, so the call can be captured in a
 * HIP graph; a replay re-reads the descriptor table at replay time.
 * Executions of one batch must not overlap in time. */
dd_status dense_dft_batch_exec(dd_batch_t b, void *stream);

/* Point the batch at new buffers of the same shapes: descs[i] must match the
 * planned descriptor i in N, alpha, T and dtype.  Takes effect at the next
 * execution or graph replay; the caller must ensure no execution of the
 * batch is in flight.  Errors: DD_ERR_INVALID (count or shape mismatch,
 * bad pointer). */
dd_status dense_dft_batch_set_buffers(dd_batch_t b, const dd_desc *descs,
                                      int32_t count);

/* Synchronise the batch's device; *flags is set to 0 (reserved).  Returns
 * DD_ERR_DEVICE if the device reports an error. */
dd_status dense_dft_batch_status(dd_batch_t b, uint32_t *flags);

/* Sizes of the planned batch: tasks in the persistent queue, blocks of its
 * launch, bytes of scratch, signals run as fallback executions. */
dd_status dense_dft_batch_info(dd_batch_t b, int32_t *tasks, int32_t *grid,
                               size_t *scratch_bytes, int32_t *fallback);

/* Free the batch (synchronises its device). */
dd_status dense_dft_batch_destroy(dd_batch_t b);

/* Convenience: plan, execute on `stream`, synchronise it, and free. */
dd_status dense_dft_exec_many(const dd_desc *descs, int32_t count,
                              void *stream);

/* ---- Serving: continuous batching of requests as they arrive ----
 *
 * A server keeps on one device: a scratch pool of hbm_budget_bytes, the
 * twiddle tables of every (N, alpha) class it has met (and plain plans for
 * requests outside the batch kernel), and max_inflight execution slots, each
 * with a stream, an event and HIP graphs of the persistent batch launch
 * captured once at creation, one per grid size (16, 64, 256 blocks and the
 * device's occupancy; a batch replays the smallest that covers its tasks;
 * the descriptor table is re-read from pinned host memory at every replay,
 * so one graph serves batches of any mix).
 * A scheduler thread fills a slot whenever one is free (when idle it polls
 * for new requests for spin_us before it sleeps).  While every queued
 * request can have a free slot of its own, the head takes a slot alone (at
 * light load requests run concurrently on separate slots, each at its solo
 * latency); once requests outnumber the free slots, batches form.  Requests above
 * batch_max_bins and the ones the batch kernel is not built for run as
 * plain executions of resident plans (with the schedules the tuner
 * recorded), each in a slot of its own when it reaches the head of the
 * queue, so that it overlaps the batches on the other slots.  Otherwise
 * the slot takes the queued kernel requests in arrival order, stepping over
 * the plain ones, as many as the batch size and the memory budget admit,
 * and launches them as one batch.  A request alone in its batch runs as a
 * plain execution too, unless DD_SERVE_DETERMINISTIC.  A request's footprint is its input and
 * output bytes plus its scratch (its output's bytes, plus 1/8 when they reach
 * 64 KiB: the most a plain execution's padded rows need, see
 * dense_dft_workspace_size); the footprints of admitted, unfinished requests never sum past
 * hbm_budget_bytes.  Each request is the transform of one dd_desc (the
 * problem of Section 2 for one signal); x and X are the caller's device
 * buffers and must stay allocated and untouched until the request is done.
 * The server's streams are not ordered after any of the caller's: x must
 * hold its samples (the stream that wrote it synchronised) when submitted,
 * and X is complete once its result reports done.
 * Times are host steady-clock nanoseconds (dense_dft_clock_ns). */

typedef struct dd_server *dd_server_t;

#define DD_SERVE_BATCHED 0
#define DD_SERVE_PLAIN 1
/* Server flag: every request the batch kernel can run goes through it, even
 * alone, and whatever is queued forms a batch, so that a result does not
 * depend on what else was queued (bit for bit).  Without it a batch of one
 * runs as a plain execution (lower latency when the server is idle; the same
 * result within the FP32 tolerance). */
#define DD_SERVE_DETERMINISTIC 0x100u

typedef struct dd_server_cfg {
    int32_t device;           /* HIP device ordinal */
    int32_t mode;             /* DD_SERVE_BATCHED, or DD_SERVE_PLAIN: every request runs
                                 alone as a plain execution (the per-request baseline) */
    size_t hbm_budget_bytes;  /* footprint bound and scratch pool size; 0 -> 8 GiB */
    int32_t max_inflight;     /* slots; 0 -> 8; at most 64 */
    int32_t max_batch;        /* requests per batch; 0 -> 256; at most 4096 (plain: 1) */
    int32_t max_queue;        /* queued, not yet admitted requests; 0 -> 65536 */
    uint32_t flags;           /* DD_TWIDDLE_FP64 or DD_TWIDDLE_FP32, | DD_SERVE_DETERMINISTIC */
    void *hip_stream;         /* NULL: a stream per slot; else every slot runs on this one */
    int64_t batch_max_bins;   /* larger requests (alpha*N bins) run as plain executions, which
                                 fill the device alone; 0 -> 2^20; -1 -> no limit */
    int32_t spin_us;          /* with nothing to do, the scheduler thread keeps polling for new
                                 requests this long before it sleeps (a sleeping thread takes
                                 time to wake: the first request after a pause pays it);
                                 0 -> 1000; -1 -> sleeps at once; at most 10^6 */
} dd_server_cfg;

typedef struct dd_result {
    dd_status status;         /* DD_OK, or the error its execution met */
    int32_t batch_requests;   /* requests in the batch it ran in */
    uint64_t t_arrival_ns;    /* submission time, or the caller's arrival stamp */
    uint64_t t_start_ns;      /* its batch was launched */
    uint64_t t_done_ns;       /* the scheduler saw its batch complete */
} dd_result;

typedef struct dd_server_stats {
    uint64_t submitted;
    uint64_t completed;
    uint64_t batches;             /* launches (batched: one per batch; plain: one per request) */
    uint64_t kernel_requests;     /* run in the persistent batch kernel */
    uint64_t fallback_requests;   /* run as plain executions */
    int32_t max_batch_seen;
    int32_t classes;              /* (N, alpha) classes with resident tables */
    size_t pool_bytes;
    size_t peak_footprint;
} dd_server_stats;

/* Create a server on cfg->device (allocates the pool, slots and graphs,
 * starts the scheduler thread).  Errors: DD_ERR_INVALID (null pointers,
 * fields out of range), DD_ERR_DEVICE (no such device, HIP failure),
 * DD_ERR_NOMEM. */
dd_status dense_dft_server_create(const dd_server_cfg *cfg, dd_server_t *out);

/* Make the resources of one request class resident now rather than at its
 * first admission: its batch-kernel tables and the plain plan that serves it
 * alone or above batch_max_bins.  Errors as dense_dft_plan, DD_ERR_CLOSED. */
dd_status dense_dft_server_warm(dd_server_t s, int64_t N, int32_t alpha, double T,
                                dd_dtype dtype);

/* Queue one request without blocking; *ticket identifies it.  The arrival
 * time is the call's time (dense_dft_submit) or t_arrival_ns, e.g. the time
 * an open-loop generator scheduled it (dense_dft_submit_at).
 * Errors: DD_ERR_INVALID (bad descriptor, as dense_dft_batch_plan),
 * DD_ERR_UNSUPPORTED, DD_ERR_TOO_LARGE (its footprint exceeds the budget),
 * DD_ERR_BUSY (max_queue requests already queued), DD_ERR_CLOSED. */
dd_status dense_dft_submit(dd_server_t s, const dd_desc *req, uint64_t *ticket);
dd_status dense_dft_submit_at(dd_server_t s, const dd_desc *req, uint64_t t_arrival_ns,
                              uint64_t *ticket);

/* Open-loop submission of a pre-drawn arrival schedule (load generation,
 * trace replay): request i is queued at host time t_arrival_ns[i] (the call
 * spins until then; the times must not decrease) and stamped with that time;
 * tickets[i] receives its ticket.  Returns once the last is queued, or at
 * the first refusal, whose status it returns (the statuses of
 * dense_dft_submit); *submitted is set to the number queued either way. */
dd_status dense_dft_submit_many_at(dd_server_t s, const dd_desc *reqs, const uint64_t *t_arrival_ns,
                                   int32_t count, uint64_t *tickets, int32_t *submitted);

/* Result of a request: DD_OK with *r filled once it is done (the ticket is
 * then retired), DD_ERR_BUSY while it is queued or running,
 * DD_ERR_INVALID for an unknown or retired ticket. */
dd_status dense_dft_poll(dd_server_t s, uint64_t ticket, dd_result *r);

/* As dense_dft_poll, but blocks until the request is done or timeout_us
 * microseconds pass (negative: no limit) -> DD_ERR_TIMEOUT. */
dd_status dense_dft_wait(dd_server_t s, uint64_t ticket, int64_t timeout_us, dd_result *r);

/* Hold (paused != 0) or release admission; queued requests wait while held. */
dd_status dense_dft_server_pause(dd_server_t s, int32_t paused);

/* Counters since creation. */
dd_status dense_dft_server_stats(dd_server_t s, dd_server_stats *st);

/* Stop accepting requests, run every queued request to completion, stop the
 * scheduler and free the server's device memory.  Unretired results are
 * discarded. */
dd_status dense_dft_server_destroy(dd_server_t s);

/* The host clock of the serving stamps, in nanoseconds. */
uint64_t dense_dft_clock_ns(void);

/* Static text for a status code. */
const char *dense_dft_status_string(dd_status status);

/* Library version as major*10000 + minor*100 + patch. */
int32_t dense_dft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DENSE_DFT_H */
