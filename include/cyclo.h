/*
 * cyclo.h - C ABI of the MI355X (gfx950) streaming cyclic-statistics library.
 *
 * A stream state accumulates, over every sample pushed into it, the cyclic
 * autocorrelation and its conjugate form (the streaming estimator of Sec. 4,
 * Eq. (11), applied to one signal x = y with non-negative lags; conjugate form
 * as in Sec. 2, Eq. (9); normalised cycle frequencies as in Sec. 2):
 *
 *   N_used     = max(0, L - T + 1)   after L samples (one count for all lags)
 *   R [t][a]   = (1/N_used) sum_{n<N_used} x[n+t] conj(x[n]) exp(-j2pi frac(alpha_a n))
 *   Rc[t][a]   = (1/N_used) sum_{n<N_used} x[n+t]      x[n]  exp(-j2pi frac(alpha_a n))
 *
 * for lags t = 0..T-1 and a caller-given list of cycle frequencies alpha_a
 * (cycles/sample, any real values; the tables are 1-periodic in alpha).  The
 * sample index n is absolute: n = 0 is the first sample pushed after
 * cyc_create() or cyc_reset(), so the phase carried across pushes plays the
 * role of the `state` attribute of the paper's block (Sec. 4).  Any
 * segmentation of the pushes gives bit-identical tables.
 *
 * Conventions for every call:
 *  - Every function returns a status code (CYC_OK = 0, negative on error) and
 *    never throws across the ABI.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All device work of a call is enqueued on it asynchronously; calls on one
 *    state must be ordered (same stream, or synchronised by the caller).
 *  - Device pointers (d_*) are caller-owned; the library never frees them and
 *    reads/writes them only from work enqueued on `stream`.
 *  - A state is not thread-safe; distinct states are independent.
 *  - After a device-side failure the state is poisoned: every call returns
 *    CYC_ESTATE until cyc_reset().
 *  - A push may run its FP64 accumulation on a stream of the state's own,
 *    ordered by events after the push's contraction on `stream`; the next
 *    read (and any later push that reuses the workspace) waits for it on its
 *    own stream, so results are as if everything ran on `stream`.
 *    cyc_destroy synchronises the device.  CYC_SERIAL_ACC=1 at creation keeps
 *    every step on `stream`.
 */
#ifndef CYCLO_H
#define CYCLO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define CYC_OK            0
#define CYC_EINVAL       -1  /* bad argument (NULL, negative size, non-finite alpha, ...) */
#define CYC_ENOMEM       -2  /* device or host allocation failed */
#define CYC_EDEVICE      -3  /* a HIP call or kernel launch failed; state poisoned */
#define CYC_ESTATE       -4  /* state is poisoned; call cyc_reset() */
#define CYC_EUNSUPPORTED -5  /* flag combination or size not supported */

/* ---- flags for cyc_create ------------------------------------------------ */
/* Operand precision of the matrix-core contraction (accumulation is always
 * FP32 within a chunk and FP64 across chunks; the alpha*n reduction is FP64).
 * A chunk is 4096 products with FP32 operands.  With BF16/FP16 a cumulative
 * single state coalesces pushes: a push commits nothing until 2^18 products
 * are pending (CYC_COALESCE, read at creation, sets the target; 0 commits at
 * every push), and a read commits what is left; results are the same either
 * way.  Its chunk is 8192 or 16384 when one such launch still spreads over at
 * least two workgroups per CU (16384 from 32 lag-by-alpha tiles on 256 CUs,
 * 8192 from 16; without coalescing, from 128 and 64 for a 2^16-sample push),
 * and batches take 16384.  The environment variable CYC_CHUNK, read at
 * creation, overrides it.  A single state's partial-sum workspace holds eight
 * chunks' FP32 partials, within 256 MiB .. 2 GiB (CYC_WORKSPACE_MB, read at
 * creation, overrides it). */
#define CYC_OP_FP32   0x0u   /* FP32 operands (default)                       */
#define CYC_OP_BF16   0x1u   /* BF16 operands                                 */
#define CYC_OP_FP16   0x2u   /* FP16 operands                                 */
#define CYC_OP_MASK   0x3u
/* Split the modulated operand conj(x[n])exp(-j2pi alpha n) (the one that holds
 * the twiddle) into hi + lo parts of the operand precision: two matrix-core
 * products per tile, about half the operand rounding error. BF16/FP16 only. */
#define CYC_TW_SPLIT  0x4u
/* cyc_read writes complex128 tables instead of complex64. */
#define CYC_OUT_C128  0x8u
/* Which tables a state keeps (the `conj` attribute of the paper's block,
 * Sec. 4, selects the conjugate form): CYC_TBL_R only the non-conjugate
 * table, CYC_TBL_RCONJ only the conjugate one, neither or both flags both.
 * A one-table state contracts only that table (half the matrix-core work;
 * its table is bitwise the one a two-table state gives), and cyc_read
 * returns CYC_EINVAL when asked for the other table.  cyc_create and
 * cyc_create2 only (window states and batches: CYC_EUNSUPPORTED). */
#define CYC_TBL_R     0x10u
#define CYC_TBL_RCONJ 0x20u

typedef struct cyc_state cyc_state;

/*
 * Create a stream state.
 *   out         : receives the new state (untouched on error).
 *   alphas_host : host array of n_alpha FP64 cycle frequencies (copied).
 *   n_alpha     : number of cycle frequencies, >= 1.
 *   n_lag       : T, the number of lags 0..T-1, 1 <= T <= 4096.
 *   flags       : CYC_OP_* | CYC_TW_SPLIT | CYC_OUT_C128 | CYC_TBL_R | CYC_TBL_RCONJ.
 *   stream      : stream for the set-up work; the call returns after it ends.
 * Errors: CYC_EINVAL (NULL pointer, n_alpha < 1, n_lag out of range,
 * non-finite alpha, unknown flag bits), CYC_EUNSUPPORTED (CYC_TW_SPLIT with
 * FP32), CYC_ENOMEM, CYC_EDEVICE.
 */
int cyc_create(cyc_state** out, const double* alphas_host, int32_t n_alpha,
               int32_t n_lag, uint32_t flags, void* stream);

/*
 * Push a block of n complex64 samples (interleaved re, im; 8-byte aligned,
 * contiguous) that live in device memory at d_x.  Asynchronous: the caller
 * must not overwrite d_x until `stream` has passed this call (a coalescing
 * push copies its samples into the state on `stream`).  n = 0 is a
 * no-op.  Errors: CYC_EINVAL (s NULL, n < 0, d_x NULL with n > 0),
 * CYC_ESTATE, CYC_EDEVICE (poisons the state).
 */
int cyc_push(cyc_state* s, const void* d_x, int64_t n, void* stream);

/*
 * Read the current tables without changing them: the state goes on as if the
 * read had not happened (it may commit chunks that coalescing pushes left
 * pending, which cyc_query then counts).
 *   d_R, d_Rc : caller-owned device buffers of T*n_alpha complex values,
 *               row-major [t][a], complex64 (or complex128 with CYC_OUT_C128);
 *               either may be NULL to skip that table.
 *   n_used    : host pointer (may be NULL) that receives N_used.
 * With N_used = 0 both tables are zero-filled and the call succeeds.
 * Errors: CYC_EINVAL (s NULL), CYC_ESTATE, CYC_EDEVICE.
 */
int cyc_read(cyc_state* s, void* d_R, void* d_Rc, int64_t* n_used, void* stream);

/*
 * Two inputs and a lag range of either sign (the block of Sec. 4, Eq. (11):
 * x[n+m] y*[n] with lags -M .. M in its Set mode).  Lags are
 * m = lag_min .. lag_min + n_lag - 1; lag m pairs x[k + m] with y[k], and the
 * phase is referenced to y's index k:
 *   R [t][a] = (1/N) sum_{n<N} x[n + dx + t] conj(y[n + dy]) exp(-j2pi frac(alpha_a (n + dy)))
 *   Rc[t][a] = (1/N) sum_{n<N} x[n + dx + t]      y[n + dy]  exp(-j2pi frac(alpha_a (n + dy)))
 * with dx = max(0, lag_min), dy = max(0, -lag_min), N = max(0, L - (n_lag - 1) - |lag_min|)
 * over L samples of each input (one count for all lags).  |lag_min| <= 2^20;
 * the other arguments as cyc_create.  cyc_push2 pushes n samples of each input
 * (separate device buffers, complex64); cyc_push on such a state uses x for
 * both inputs; read / reset / destroy / query are the single-input calls.
 * cyc_push2 on a state made by cyc_create returns CYC_EINVAL.  Results do not
 * depend on how the samples are split into pushes.
 */
int cyc_create2(cyc_state** out, const double* alphas_host, int32_t n_alpha, int64_t lag_min,
                int32_t n_lag, uint32_t flags, void* stream);
int cyc_push2(cyc_state* s, const void* d_x, const void* d_y, int64_t n, void* stream);

/*
 * Sliding-window form (the block of Sec. 4 emits the estimate over a window
 * of its latest samples, the phase re-referenced to the window's start by
 * its `state`).  Products are committed in hops of `hop` (aligned to the
 * first product); cyc_read returns the estimate over the last
 * W = min(n_hops, complete hops) hops, products n_w .. n_w + W hop - 1:
 *   R[t][a] = (1/(W hop)) sum_n x[n+t] conj(x[n]) exp(-j2pi frac(alpha_a (n - n_w)))
 * (and Rc alike), *n_used = W hop (zero tables before the first complete
 * hop; products of an incomplete hop are not part of any window yet).
 * hop: a multiple of 32 in [32, 2^20]; n_hops in [1, 4096]; the other
 * arguments as cyc_create.  push / read / reset / destroy are the
 * single-input calls; results do not depend on how samples are pushed.
 * Memory: 32 n_hops T A bytes for the window's FP64 hop sums.
 */
int cyc_create_window(cyc_state** out, const double* alphas_host, int32_t n_alpha, int32_t n_lag,
                      int32_t hop, int32_t n_hops, uint32_t flags, void* stream);

/*
 * Forget every pushed sample and clear the poison flag; alphas, T and flags
 * are kept.  Afterwards the state behaves exactly like a fresh one.  Host-only
 * (enqueues no device work).  Errors: CYC_EINVAL (s NULL).
 */
int cyc_reset(cyc_state* s);

/* Free the state and its device memory (synchronises the device). NULL is a no-op. */
void cyc_destroy(cyc_state* s);

/* Static, human-readable text for a status code. */
const char* cyc_status_str(int code);

/*
 * Introspection (host-only): samples pushed, products committed to the FP64
 * accumulator (a multiple of the chunk length), chunk length in samples, and
 * the index of the contraction kernel configuration in use.  Any output
 * pointer may be NULL.  Errors: CYC_EINVAL (s NULL).
 */
int cyc_query(const cyc_state* s, int64_t* n_pushed, int64_t* n_committed,
              int32_t* chunk, int32_t* kernel_cfg);

/*
 * Kernel timing (tracing aid).  cyc_profile(s, 1) clears the counters and
 * starts recording a pair of HIP events around every launch of the
 * contraction kernel, on the stream that launch runs on; cyc_profile(s, 0)
 * stops recording.  cyc_profile_read waits for the recorded events and
 * returns the summed kernel time in milliseconds, the number of launches and
 * the number of (alpha, tau, sample) triples those launches evaluated (each
 * triple is one complex multiply-add per table).  Outputs may be NULL.
 * Errors: CYC_EINVAL (s NULL), CYC_ENOMEM, CYC_EDEVICE.
 */
int cyc_profile(cyc_state* s, int32_t enable);
int cyc_profile_read(cyc_state* s, double* total_ms, int64_t* launches, double* work);

/*
 * Contraction-kernel configurations (tile shapes).  Index idx in
 * [0, cyc_kernel_cfg_count()).  cyc_kernel_cfg_info reports the operand
 * precision and split flags the configuration implements (CYC_OP_* |
 * CYC_TW_SPLIT), its lag and cycle-frequency tile, its workgroup size and a
 * static name; outputs may be NULL.  Errors: CYC_EINVAL (idx out of range).
 */
int cyc_kernel_cfg_count(void);
int cyc_kernel_cfg_info(int32_t idx, uint32_t* flags, int32_t* lag_tile, int32_t* alpha_tile,
                        int32_t* threads, const char** name);

/*
 * Use configuration idx for the state's contraction from now on.  Every
 * configuration of one precision evaluates each table entry with the same
 * operands in the same order, so switching does not change results.
 * Errors: CYC_EINVAL (s NULL, idx out of range), CYC_EUNSUPPORTED (idx
 * implements another precision or split mode).
 */
int cyc_set_kernel_cfg(cyc_state* s, int32_t idx);

/*
 * Autotuner.  Times every configuration that implements `flags` on pushes of
 * synthetic samples (16 chunks each) into a state of n_alpha cycle
 * frequencies and n_lag lags (HIP events on `stream`; after a warm-up the
 * candidates are timed round-robin, three rounds of two timed pushes each,
 * and each is ranked by its median), and records the fastest in the tuning
 * cache under
 * (device architecture, precision, split, n_lag, ceil(log2 n_alpha)).
 * cyc_create consults the cache.  If the environment variable CYC_TUNE_CACHE
 * names a file, the cache is loaded from it on first use and every new entry
 * is appended to it (one line per entry).  best_cfg / best_ms (may be NULL)
 * receive the winner and its time per push.  Allocates and frees device
 * memory.  Errors: as cyc_create, plus CYC_EDEVICE.
 */
int cyc_autotune(int32_t n_alpha, int32_t n_lag, uint32_t flags, int32_t* best_cfg, double* best_ms,
                 void* stream);

/*
 * Batches: many independent stream states with a common lag count, each with
 * its own cycle-frequency list, advanced together.  Per stream the semantics
 * are exactly those of cyc_push / cyc_read (tables bit-identical to a single
 * state fed the same samples with the same kernel configuration).  A push runs
 * one persistent contraction launch over every committed chunk of every
 * stream (work items taken from an atomic counter), bracketed by batched phase,
 * accumulation and pending-sample kernels; the sequence is captured once in a
 * HIP graph and replayed with new device-side descriptor tables (CYC_NO_GRAPH=1
 * in the environment at cyc_batch_create launches the kernels directly instead).
 *
 * cyc_batch_create
 *   n_streams     : number of streams, >= 1.
 *   alpha_offsets : host array of n_streams+1 offsets into `alphas`
 *                   (non-decreasing, alpha_offsets[0] = 0, each stream >= 1 alpha).
 *   alphas        : host FP64 cycle frequencies of all streams, concatenated.
 *   n_lag, flags  : as cyc_create (CYC_OP_*, CYC_TW_SPLIT, CYC_OUT_C128).
 * cyc_batch_push
 *   d_x : host array of n_streams device pointers (complex64 samples; a pointer
 *         may be NULL when its count is 0); n : host array of n_streams counts.
 *   The device buffers must stay unmodified until `stream` passes the call.
 * cyc_batch_read
 *   d_R, d_Rc : host arrays of n_streams device pointers to [T][A_s] tables
 *               (either array, or any entry, may be NULL to skip).
 *   n_used    : host array of n_streams (may be NULL).
 * Errors: as the single-stream calls.  The batch allocates its descriptor
 * tables and workspace at creation (CYC_WORKSPACE_MB, default 4096, bounds the
 * partial-sum workspace; larger pushes are processed in several rounds).  The
 * chunk length (CYC_CHUNK) defaults to 4096 products for FP32 operands and
 * 16384 for BF16/FP16.
 */
typedef struct cyc_batch cyc_batch;
int cyc_batch_create(cyc_batch** out, int32_t n_streams, const int64_t* alpha_offsets,
                     const double* alphas, int32_t n_lag, uint32_t flags, void* stream);
int cyc_batch_push(cyc_batch* b, const void* const* d_x, const int64_t* n, void* stream);
int cyc_batch_read(cyc_batch* b, void* const* d_R, void* const* d_Rc, int64_t* n_used,
                   void* stream);
int cyc_batch_reset(cyc_batch* b);
void cyc_batch_destroy(cyc_batch* b);
/* Kernel configuration in use, number of rounds of the last push and whether
 * the last push replayed a captured graph (outputs may be NULL). */
int cyc_batch_query(const cyc_batch* b, int32_t* kernel_cfg, int32_t* rounds, int32_t* graph);
/* Timing of the batch's persistent contraction launches, as cyc_profile /
 * cyc_profile_read for one state: while enabled, pushes launch directly
 * instead of through the graph, and HIP events bracket every contraction
 * launch (push rounds and the partial chunks of a read) on the call's stream;
 * work = products x lags x cycle frequencies contracted.  Enabling clears
 * the record. */
int cyc_batch_profile(cyc_batch* b, int32_t enable);
int cyc_batch_profile_read(cyc_batch* b, double* total_ms, int64_t* launches, double* work);

/*
 * Uniform-grid form: the same tables R, Rc (definition and conventions as
 * cyc_create .. cyc_read) on the whole grid alpha_k = alpha0 + k / n_alpha,
 * k = 0 .. n_alpha-1, evaluated by folding and an FFT (the paper's Full mode,
 * Sec. 4, covers a grid of cycle frequencies with an FFT).  Because
 * exp(-j2pi k n / A) depends only on n mod A, a push adds every product
 * x[n+t] conj(x[n]) exp(-j2pi frac(alpha0 n)) (and the conjugate one) into the
 * fold bin n mod A, and a read takes one A-point DFT per (table, lag).
 *   n_alpha : A, a power of two, 2 <= A <= 65536 (else CYC_EUNSUPPORTED).
 *   n_lag   : T, 1 <= T <= 4096.   alpha0 : any finite real.
 *   flags   : 0 or CYC_OUT_C128 (table element type; the arithmetic is FP64).
 * push / read / reset / destroy behave as cyc_push / cyc_read / cyc_reset /
 * cyc_destroy: asynchronous on `stream`, any segmentation gives the same bits,
 * read leaves the state unchanged, N_used = max(0, L - T + 1) (zero tables and
 * CYC_OK when it is 0).  Work per product is O(T); per read O(T A log A).
 * State memory: 32 T A bytes (64 T A when A > 8192) plus a 16 MiB phase
 * buffer.  Errors as the single-stream calls.
 */
typedef struct cyc_grid cyc_grid;
int cyc_grid_create(cyc_grid** out, double alpha0, int32_t n_alpha, int32_t n_lag, uint32_t flags,
                    void* stream);
int cyc_grid_push(cyc_grid* g, const void* d_x, int64_t n, void* stream);
/* Two inputs and lags lag_min .. lag_min + n_lag - 1 on the uniform grid, with
 * the conventions of cyc_create2 / cyc_push2 (|lag_min| <= 2^20; cyc_grid_push
 * on such a state uses x for both inputs; cyc_grid_push2 on a one-input state
 * returns CYC_EINVAL). */
int cyc_grid_create2(cyc_grid** out, double alpha0, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                     uint32_t flags, void* stream);
int cyc_grid_push2(cyc_grid* g, const void* d_x, const void* d_y, int64_t n, void* stream);
int cyc_grid_read(cyc_grid* g, void* d_R, void* d_Rc, int64_t* n_used, void* stream);
int cyc_grid_reset(cyc_grid* g);
void cyc_grid_destroy(cyc_grid* g);

/*
 * Cyclic spectrum from a lag table, by the cyclic Wiener-Khinchin relation
 * (the paper leaves spectral analysis of the cyclic statistics for future
 * work, Sec. 6):
 *   S[k][a] = sum_{t<n_lag} w(m_t) exp(-j pi alpha_a m_t) R[t][a] exp(-j2pi f_k m_t),
 *   m_t = lag_min + t,  f_k = -1/2 + k / n_freq,  k < n_freq.
 * exp(-j pi alpha m) R(m) is the symmetric form of the leading-lag tables this
 * library returns (either table, from cyc_read / cyc_grid_read, lags of
 * either sign from the two-input states).  window: 0 rectangular, 1 Hann,
 * w(m) = (1 + cos(pi m / (M + 1))) / 2 with M = max |m_t|.
 *   d_R      complex64 [n_lag][n_alpha] device table; d_alphas FP64 [n_alpha]
 *            device array of its cycle frequencies;
 *   d_S      complex64 [n_freq][n_alpha] device output.
 * FP64 phases, FP32 sums.  n_lag <= 8192, n_freq <= 65536, |lag_min| <= 2^20.
 * A workspace of 8 n_lag n_alpha bytes is allocated stream-ordered.  Errors:
 * CYC_EINVAL, CYC_ENOMEM, CYC_EDEVICE.
 */
int cyc_scf(const void* d_R, const double* d_alphas, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
            int32_t n_freq, int32_t window, void* d_S, void* stream);
/*
 * cyc_scf without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as cyc_scf (bit for
 * bit); the weighted lag table lives in a fixed 16 MiB device array that the
 * library holds on each GPU it runs on until the process ends, so
 * n_lag * n_alpha <= 2^21 (2097152; larger sizes return CYC_EUNSUPPORTED
 * before any work is enqueued).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (different streams, or host threads without
 * ordering) race and give undefined tables; calls ordered on one stream are
 * safe.  Nothing in the array needs to start at zero: each call overwrites
 * the part it reads.  Errors: CYC_EINVAL (as cyc_scf), CYC_EUNSUPPORTED,
 * CYC_EDEVICE (no current device, symbol lookup or launch failure).
 */
int cyc_scf_noalloc(const void* d_R, const double* d_alphas, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                    int32_t n_freq, int32_t window, void* d_S, void* stream);

/*
 * Cycle-frequency estimation (the paper leaves it for future work, Sec. 6;
 * Sec. 1 describes coarse-to-fine searches among related estimators), on one
 * table of the uniform grid alpha_k = alpha0 + k / n_alpha:
 *  1. noise scale sigma[t][c] per lag t and block c of 64 bins: the median of
 *     |R[t][.]| over blocks c-1, c, c+1 (circular) / sqrt(2 ln 2);
 *  2. q[k] = max_t |R[t][k]| / sigma[t][k / 64];
 *  3. candidates: q[k] > kappa, q[k] > q[k-1] and q[k] >= q[k+1] (circular);
 *  4. leakage masking in descending q (ties -> lower k): a candidate is kept
 *     if at some lag it exceeds kappa sigma and
 *     |R[t][k]| > (pi/2) n_alpha / (n_used (d - 1/2)) |R[t][p]| for every kept
 *     p at circular distance d: twice the most a feature within half a bin
 *     of p leaks there through the Dirichlet kernel of n_used products, which
 *     needs a grid at least as fine as 1/n_used (n_used <= n_alpha);
 *  5. (cyc_estimate_cycle_freqs) refinement on the zoom grid
 *     alpha_k + (j - zoom) / (zoom n_alpha), j = 0 .. 2 zoom: the first zoom
 *     point with the largest max_t |R| / sigma[t][k / 64].
 * |R| = sqrt(Re^2 + Im^2), scales and comparisons are FP64.
 *
 * cyc_cfe_detect: steps 1-4 on a device table d_R, complex64
 *   [n_lag][n_alpha] (n_alpha a multiple of 64, 1 <= n_lag <= 4096,
 *   1 <= n_used <= n_alpha, kappa >= 0 finite).  exclude_bin (-1 for none)
 *   takes part in the masking but is never reported (the alpha = 0 bin of the
 *   non-conjugate table).  Writes the kept bins in ascending order to d_bins
 *   (int32, the first min(count, max_out)), their number to *d_count (device
 *   int32) and the scales to d_sigma (FP64 [n_lag][n_alpha / 64], device).
 *   Synchronises the stream.  More than 4096 candidates: CYC_EUNSUPPORTED.
 * cyc_cfe_refine: step 5 on a device zoom table d_Rz, complex64
 *   [n_lag][n_peaks (2 zoom + 1)] (peak p's columns contiguous), with the
 *   detections d_bins and scales d_sigma of cyc_cfe_detect (n_alpha the
 *   coarse grid size): d_j[p] = best zoom index, d_q[p] = its statistic.
 * cyc_estimate_cycle_freqs: the whole estimator from n complex64 samples at
 *   d_x (device): the coarse table (table 0 = R, 1 = Rc) from the exact
 *   uniform-grid form when n_alpha is a power of two <= 65536, else the dense
 *   FP32 contraction; cyc_cfe_detect (exclude_zero: skip the alpha = 0 bin of
 *   R); the zoom table by the dense FP32 contraction; cyc_cfe_refine.  Host
 *   outputs: *count (all detections) and, for the first min(count, max_out)
 *   in ascending bin order, bins, alpha_hat (cycles/sample) and stat (the
 *   refined q).  Allocates its own work space; synchronises the stream.
 * Errors: CYC_EINVAL (NULL, sizes, n_used > n_alpha, non-finite arguments),
 * CYC_EUNSUPPORTED (too many candidates), CYC_ENOMEM, CYC_EDEVICE.
 */
int cyc_cfe_detect(const void* d_R, int32_t n_lag, int32_t n_alpha, int64_t n_used, double kappa,
                   int32_t exclude_bin, int32_t max_out, int32_t* d_bins, int32_t* d_count, double* d_sigma,
                   void* stream);
int cyc_cfe_refine(const void* d_Rz, int32_t n_lag, int32_t n_peaks, int32_t zoom, const int32_t* d_bins,
                   const double* d_sigma, int32_t n_alpha, int32_t* d_j, double* d_q, void* stream);
int cyc_estimate_cycle_freqs(const void* d_x, int64_t n, double alpha0, int32_t n_alpha, int32_t n_lag,
                             int32_t table, double kappa, int32_t zoom, int32_t exclude_zero, int32_t max_out,
                             double* alpha_hat, double* stat, int32_t* bins, int32_t* count, void* stream);

/*
 * Learned cycle-frequency proposal (coarse stage of a coarse-to-fine
 * estimator; the paper's related work in Sec. 1 describes the two-stage idea
 * and Sec. 6 names cycle-frequency estimation as future work).
 *
 * Features: for each window of 65536 complex64 samples, Welch spectra
 * (64 Hann-windowed segments of 1024, averaged |FFT|^2) of x, x^2 and |x|^2,
 * shifted to frequencies -1/2 + m/1024, log, standardised per channel.
 * Layout of a feature batch: float [3][n_windows][1024] (channel-major).
 * Network: 4 circular conv1d layers (64 channels, kernel 7, ReLU), then per
 * coarse bin k the sum of a dense 65536 -> 1024 layer, a bias and a local
 * layer (sum over channels c of Wl[c] * activation[c][position k], weights
 * shared by all bins), and a sigmoid: probability that coarse bin k (cycle
 * frequencies [-1/2 + k/1024, -1/2 + (k+1)/1024)) holds a feature.
 * Parameters: one FP32 vector of cyc_model_num_params() values, in the order
 * W0[64][3][7], b0[64], W1[64][64][7], b1, W2, b2, W3, b3, Wh[1024][65536],
 * bh[1024], Wl[64].  flags: CYC_OP_FP32 or CYC_OP_BF16 operands for every
 * matrix product (FP32 accumulation, FP32 master weights and AdamW moments;
 * the local layer is FP32 in both), optionally | CYC_NN_NO_LOCAL: the network
 * without the local layer (the four convolutions and the dense head alone; Wl
 * stays in the parameter vector, is ignored and gets a zero gradient).
 * max_batch bounds n_windows of every call (activations are allocated at
 * creation).  All d_* pointers are device memory.  Errors: CYC_EINVAL,
 * CYC_EUNSUPPORTED (other precisions), CYC_ENOMEM, CYC_EDEVICE.
 */
#define CYC_NN_NO_LOCAL 0x100u
typedef struct cyc_model cyc_model;
int64_t cyc_model_num_params(void);
int cyc_model_create(cyc_model** out, int32_t max_batch, uint32_t flags, void* stream);
void cyc_model_destroy(cyc_model* m);
/* Copy FP32 parameters from / to host memory (set also clears the AdamW state). */
int cyc_model_set_params(cyc_model* m, const float* host, void* stream);
int cyc_model_get_params(cyc_model* m, float* host, void* stream);
/* d_x: n_windows * 65536 complex64 samples -> d_feat [3][n_windows][1024]. */
int cyc_model_spectra(cyc_model* m, const void* d_x, int32_t n_windows, float* d_feat, void* stream);
/* d_prob: [n][1024] probabilities. */
int cyc_model_forward(cyc_model* m, const float* d_feat, int32_t n, float* d_prob, void* stream);
/* Gradients of the mean binary cross-entropy against d_labels [n][1024] (0/1)
 * into d_grad (num_params floats, may be NULL); *loss (host, may be NULL). */
int cyc_model_gradients(cyc_model* m, const float* d_feat, const float* d_labels, int32_t n,
                        float* d_grad, double* loss, void* stream);
/* One AdamW step (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay). */
int cyc_model_train_step(cyc_model* m, const float* d_feat, const float* d_labels, int32_t n,
                         float lr, float weight_decay, double* loss, void* stream);
/*
 * Selection: per window, the topk coarse bins of d_prob [n][1024] (ties ->
 * lower index), each widened by +-width bins circularly, plus zero_bin (-1 for
 * none) -> d_sel [n][1024] (1 = evaluate), and d_conf [n] = 1 - the largest
 * probability outside the selection (fall back to the full grid below a
 * threshold).  NaN probabilities are never selected, and a window with a NaN
 * or infinite probability gets d_conf = 0.
 */
int cyc_select(const float* d_prob, int32_t n, int32_t topk, int32_t width, int32_t zero_bin,
               uint8_t* d_sel, float* d_conf, void* stream);
/*
 * The whole coarse stage in one call, for n_windows (<= max_batch) windows of
 * 65536 complex64 samples at d_x (contiguous): spectra, network, selection as
 * cyc_select (topk, width, zero_bin), then per window
 *   d_bins     int32 [n_windows][1024]: the selected coarse bins in ascending
 *              order, -1 after the last; coarse bin k holds the fine cycle
 *              frequencies -1/2 + (64 k + f)/65536, f = 0..63;
 *   d_n_bins   int32 [n_windows]: the number of selected bins;
 *   d_conf     float [n_windows]: 1 - the largest probability left out (0 when
 *              a probability or a feature of the window is NaN or infinite,
 *              e.g. after a non-finite sample, so that the window falls back);
 *   d_fallback uint8 [n_windows]: 1 when conf < theta (evaluate the full grid).
 * The exact estimator then runs on those cycle frequencies (cyc_create or
 * cyc_batch_create).  Uses the model's own scratch buffers: calls on one model
 * are serialised by the caller.  Errors: CYC_EINVAL (NULL, sizes, NaN theta),
 * CYC_EDEVICE.
 */
int cyc_propose(cyc_model* m, const void* d_x, int32_t n_windows, int32_t topk, int32_t width,
                int32_t zero_bin, float theta, int32_t* d_bins, int32_t* d_n_bins, float* d_conf,
                uint8_t* d_fallback, void* stream);
/*
 * Labels from full-grid tables: d_R, d_Rc complex64 [n_lag][n_alpha] of one
 * window, n_alpha = n_coarse * (fine bins per coarse bin).  Coarse bin c is 1
 * if some fine bin of it has |R| > thresh * sigma_t at some lag t in either
 * table.  sigma is local: for fine bins of coarse bin c at lag t it is the
 * median of |R[t][.]| over the fine bins of coarse bins c-1, c, c+1 (circular)
 * divided by sqrt(2 ln 2), the Rayleigh scale of noise-only cells (an even
 * count takes the mean of the two middle magnitudes).  The non-conjugate
 * table is ignored in zero_bin (-1 for none).  Either table may be NULL (it
 * contributes no peaks), not both.  Magnitudes and the threshold are FP64.
 * Requires 3 * n_alpha / n_coarse <= 1024 and n_lag <= 65535.
 * A workspace of 16 * n_lag * n_coarse bytes is allocated stream-ordered.
 */
int cyc_peak_labels(const void* d_R, const void* d_Rc, int32_t n_lag, int32_t n_alpha,
                    int32_t n_coarse, int32_t zero_bin, float thresh, float* d_labels, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CYCLO_H */
