/*
 * perm.h -- exact matrix permanents on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpermgpu.so.  Every function is extern "C", takes plain pointers
 * and sizes, never throws, and returns a perm_status (0 = success).
 *
 * What is computed (Masschelein, Richer & Ayers, "Optimizing and benchmarking
 * the computation of the permanent of general matrices"):
 *
 *   per(A) = sum over injective maps s:[m]->[n] of prod_i a[i][s(i)], m <= n,
 *   per(A) = per(A^T) when m > n,
 *
 * (Sec. 1.1, Eq. permanent_definition and Eq. rectangular_permanent_definition),
 * and per(A) = 1 for m = 0 (empty product).  The three algorithms of Sec. 1.2
 * all return this same value; they differ only in cost and rounding.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - dA is a DEVICE pointer to a row-major m x n matrix with leading dimension
 *    lda >= n, counted in elements of the input dtype (a PERM_C128 element is
 *    16 bytes: real part then imaginary part).  m > n is served by reading the
 *    transpose in place (no copy).
 *  - dOut is a DEVICE pointer that receives one value of the requested output
 *    type (see perm_out).  The caller owns dA and dOut; the library never
 *    frees or retains them.
 *  - stream is a hipStream_t (NULL = the default stream).  All device work is
 *    enqueued on it and the call returns without waiting, with these
 *    exceptions: integer outputs (PERM_OUT_I64 / PERM_OUT_I128) run an overflow pre-check
 *    that reads per-row absolute sums back to the host and so synchronises the
 *    stream, unless PERM_FLAG_WRAP is set; square floating-point
 *    perm_ryser with n >= 30 (complex: n >= 29) or PERM_FLAG_SPARSE, and
 *    integer square perm_ryser at any n, read each row's nonzero pattern
 *    back to plan a column window, and wait again to upload it when one is
 *    used.
 *  - Temporary device memory (per-workgroup partial sums) is taken from the
 *    stream-ordered allocator and released on the same stream; calls on
 *    different streams do not share scratch memory and may run concurrently.
 *  - Results are bitwise reproducible: partial sums are combined in a fixed
 *    order that depends only on the shape and the device's compute-unit count.
 *  - On any error nothing is written to dOut.
 *
 * Status codes
 *   PERM_OK            success
 *   PERM_E_INVALID     null pointer, lda < n, negative size, unknown enum,
 *                      output type not valid for the input type
 *   PERM_E_TOO_LARGE   the shape exceeds the algorithm's limit (stated with
 *                      each function)
 *   PERM_E_OVERFLOW    an integer output could exceed its type (pre-check bound
 *                      prod_i sum_j |a_ij| >= 2^63 or 2^127) and PERM_FLAG_WRAP
 *                      was not given, or an exact integer product could not be
 *                      formed (an absolute row or column sum >= 2^52)
 *   PERM_E_HIP         a HIP runtime call failed
 *   PERM_E_UNSUPPORTED the combination of arguments is not implemented
 */
#ifndef PERM_H
#define PERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERM_VERSION 10000 /* 1.0.0 */

typedef enum perm_status {
  PERM_OK = 0,
  PERM_E_INVALID = -1,
  PERM_E_TOO_LARGE = -2,
  PERM_E_OVERFLOW = -3,
  PERM_E_HIP = -4,
  PERM_E_UNSUPPORTED = -5
} perm_status;

/* Input element type. */
typedef enum perm_dtype {
  PERM_F64 = 0,  /* double */
  PERM_C128 = 1, /* complex double, interleaved (re, im) */
  PERM_I64 = 2,  /* int64_t */
  PERM_B8 = 3    /* uint8_t, every entry 0 or 1 (other values are read as 1) */
} perm_dtype;

/* Output type.  Valid pairs:
 *   PERM_F64  input -> PERM_OUT_F64 or PERM_OUT_DD
 *   PERM_C128 input -> PERM_OUT_C128 or PERM_OUT_CDD
 *   PERM_I64 / PERM_B8 input -> PERM_OUT_I64, PERM_OUT_I128 (exact), or
 *                                PERM_OUT_F64 / PERM_OUT_DD (floating-point path)
 */
typedef enum perm_out {
  PERM_OUT_F64 = 0,  /* double */
  PERM_OUT_C128 = 1, /* double[2] = (re, im) */
  PERM_OUT_I64 = 2,  /* int64_t */
  PERM_OUT_I128 = 3, /* {uint64_t lo; int64_t hi;} two's complement */
  PERM_OUT_DD = 4,   /* double[2] = (hi, lo), value hi + lo, |lo| <= ulp(hi)/2 */
  PERM_OUT_CDD = 5   /* double[4] = (re.hi, re.lo, im.hi, im.lo) */
} perm_out;

typedef enum perm_algo {
  PERM_ALGO_COMBINATORIC = 0,
  PERM_ALGO_RYSER = 1,
  PERM_ALGO_GLYNN = 2,
  PERM_ALGO_GLYNN_ESYM = 3, /* perm_glynn_esym */
  PERM_ALGO_AUTO = 4,       /* batch plans: the sum chosen per matrix */
  PERM_ALGO_SWEEP = 5       /* perm_column_sweep */
} perm_algo;

/* Flags (bitwise or). */
#define PERM_FLAG_PAD_ONES 0x2u /* perm_glynn, floating point, m < n: pad with rows of
                                   ones exactly as Eq. glynn_filled_matrix (by default
                                   the padding value is a power of two scaled to the
                                   data, see perm_glynn) */
#define PERM_FLAG_WRAP 0x1u /* integer outputs: skip the overflow pre-check and
                               return the exact value modulo 2^64 / 2^128 (for
                               Glynn: modulo 2^(128-(n-1)-v), v the power of two
                               in (n-m)!), sign-extended */
#define PERM_BATCH_AUTOTUNE 0x4u /* perm_batch_plan_create: choose the matrices per
                                    wave of every small order by timing on the
                                    plan's first run (see perm_batch_plan_run) */
#define PERM_FLAG_SPARSE 0x8u /* square perm_ryser, floating point: read the
                                 nonzero pattern back and plan a column window at
                                 any order (see perm_ryser; one more wait for the
                                 stream) */

/* Library version, PERM_VERSION. */
int perm_version(void);

/* Releases the device memory the library keeps on the current device: the
 * cached tables of the rectangular Ryser walk (revolving-door transitions,
 * binomials; rebuilt on next use) and the unused memory of the device's
 * stream-ordered pool that per-call scratch came from.  Waits for the device
 * first, so no call may be in flight on it.  Batch plans keep their own memory
 * until perm_batch_plan_destroy. */
int perm_workspace_release(void);

/* Static description of a status code (never NULL). */
const char *perm_status_string(int status);

/* Measurement support.  perm_profile_enable(1) starts a session on the calling
 * thread: every later single-matrix call from that thread records a pair of
 * HIP events on its stream around its main kernel (the Gray-walk engine, the
 * e_m walk, the rectangular Ryser walk or the combinatoric kernel), without
 * waiting.  perm_profile_last waits for the session's most recent pair and
 * returns the kernel's duration in milliseconds (PERM_E_INVALID if none was
 * recorded); perm_profile_durations waits for the first min(capacity, count)
 * pairs and writes their durations to the HOST array ms, in call order, with
 * *count = the number of pairs recorded in the session.  perm_profile_enable(0)
 * stops recording (the session's pairs stay readable).  Off by default; costs
 * two event records per call when on. */
int perm_profile_enable(int on);
int perm_profile_last(double *ms);
int perm_profile_durations(double *ms, int capacity, int *count);

/* perm_glynn -- Glynn's formula, Sec. 1.2 Eq. glynn:
 *   per(A) = 2^-(n-1) sum_{delta in {+-1}^n, delta_1=+1} (prod delta) prod_j sum_i delta_i a_ij
 * summed in reflected Gray-code order; for m < n the matrix is padded with
 * n - m rows of ones and the sum divided by (n-m)! (Eq. glynn_filled_matrix,
 * Eq. glynn_rectangle).  With floating-point outputs the padding rows hold
 * c = 2^e instead, and the sum is divided by (n-m)! c^(n-m) (exact
 * rescaling: per([A; cJ]) = c^(n-m) per([A; J])).  e is chosen on the device
 * from the data's mean square s2 = sum |a_ij|^2 / n: among 21 powers of two
 * around sqrt(s2 / (n-m)) it minimises a model of the padded sum's relative
 * rounding error, F(c) = ln sum_t C(n-m, t) (s2 + c^2 (n-m-2t)^2)^(n/2)
 * - (n-m) ln c (the terms' typical magnitude against the value's factor
 * c^(n-m)); e is clamped to [-200, 200].  With rows of ones the padding
 * dominates the column sums and the sum loses most of its digits.
 * PERM_FLAG_PAD_ONES keeps the value 1.  Integer outputs always pad with
 * ones.  Cost 2^(n-1) terms of O(n), n = max(m, n).
 * Limit: n <= 48 for floating-point outputs, n <= 40 for integer outputs. */
int perm_glynn(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
               void *dOut, uint32_t flags, void *stream);

/* perm_glynn_noalloc -- perm_glynn for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and launch plan, hence bitwise the same
 * result, with the walk's scratch (update table, start vector, per-workgroup
 * partials, padding exponent) in a fixed device array of
 * PERM_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends (its address is looked up once per device, on
 * the first call there).  No hipMalloc, hipFree or other allocation happens
 * in the call.  Floating-point outputs only: integer outputs return
 * PERM_E_UNSUPPORTED (their overflow pre-check reads the matrix back through
 * allocated memory).  A shape whose scratch exceeds the array returns
 * PERM_E_TOO_LARGE (no admissible shape does on a device of up to 256 compute
 * units).  Every call on one device shares that array and leaves its last
 * contents in it, so calls that overlap on one device -- on different streams,
 * or from different threads -- race: the caller serialises them (one stream,
 * or events).  Other arguments, flags and limits as for perm_glynn. */
#define PERM_NOALLOC_SCRATCH_BYTES (256u * 1024u)
int perm_glynn_noalloc(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                       void *dOut, uint32_t flags, void *stream);

/* perm_glynn_esym -- the rectangular Glynn sum with its padding rows summed
 * out.  The n - m rows of ones that Eq. glynn_filled_matrix appends are
 * identical, and summing their signs leaves
 *   per(A) = 2^-(m-1) sum_{delta in {+-1}^m, delta_1=+1} (prod delta) e_m(c(delta)),
 *   c_j = sum_i delta_i a_ij,
 * with e_m the m-th elementary symmetric polynomial of c_1..c_n (expanding
 * e_m into row choices, the sign sum keeps the products that use every row
 * once).  Cost 2^(m-1) terms instead of Glynn's 2^(n-1) for m < n; a term
 * runs the recurrence e_k += c_j e_(k-1) over the columns, for floating-point
 * outputs at 14 <= m <= 32 only over the degrees that can still reach e_m
 * (max(1, j+1-(n-m)) <= k <= min(j+1, m) at column j: about m (n-m+1)
 * multiply-adds), otherwise over every degree up to min(n, 32).  Integer
 * outputs are exact (the degrees are kept modulo
 * 2^128, with the overflow pre-check of the integer paths: every column
 * absolute sum below 2^53 and |per| 2^(m-1) below 2^127, unless
 * PERM_FLAG_WRAP).  Limits: min(m, n) <= 32, max(m, n) <= 48. */
int perm_glynn_esym(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                    void *dOut, uint32_t flags, void *stream);

/* perm_ryser -- Ryser's inclusion-exclusion formula, Sec. 1.2
 * Eq. ryser_square (m = n) and Eq. ryser_rectangle (m < n, read over column
 * subsets of size m-k with weight (-1)^k C(n-m+k, k)).  Square: Gray-code
 * order over the 2^n column subsets; rectangular: the subsets of each size
 * s <= m in revolving-door order.  Limits: square n <= 48 (floating point)
 * or n <= 40 (integer); rectangular min(m, n) <= 40 and max(m, n) <= 64.
 * Square: a row whose nonzeros all lie in a column set U has an empty sum,
 * so a zero term, for every subset that misses them; when sparse rows make
 * this worthwhile (perm_ryser_window_plan), the columns of U go on the top
 * Gray bits and only their states that meet every such row are walked.
 * Integer outputs always consider it (the same integer results);
 * floating-point outputs when the whole walk is long, n >= 30 (complex:
 * n >= 29), or at any n with PERM_FLAG_SPARSE (the skipped terms are exact
 * zeros, so only the order of the additions changes; the extra wait for the
 * nonzero pattern, about 0.1 ms per call of lost overlap, is under 6% of a
 * dense walk from those orders on).  The environment variable
 * PERM_RYSER_WINDOW=0 keeps the whole walk; =2 takes a window whenever one
 * prunes any state, at any n. */
int perm_ryser(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
               void *dOut, uint32_t flags, void *stream);

/* perm_ryser_window_plan -- the column window perm_ryser uses for a square
 * n x n matrix (host only, no device call).  row_masks: HOST
 * uint64[n], bit j of row i set iff a_ij != 0.  lanes_max: the walk's lane
 * count (a power of two >= 256; the device's is resident workgroups x 256).
 * The window U is grown from the rows with the fewest nonzeros while it
 * holds at most min(16, n - 10) columns, and kept only if the model time
 * of the pruned walk (blocks per lane x block cost) is below 0.8 of the
 * whole walk's (force != 0: whenever it prunes a state).  Returns 1 and
 * fills *fw = |U|, *b = log2 of the block length, *wlow = block-index bits under the window state, *nstates = the
 * number of states of U that meet every row inside U, col_order (may be
 * NULL; HOST int32[n]: Gray bit q toggles column col_order[q], the window
 * on bits n - fw .. n - 1 in ascending column order) and states (may be
 * NULL; HOST uint32[states_cap]: bit p set = column col_order[n - fw + p]
 * in the subset; PERM_E_TOO_LARGE if more than states_cap); returns 0 (and
 * zeros) when the whole walk is kept; PERM_E_INVALID for n outside 0..64
 * or a null pointer. */
int perm_ryser_window_plan(int n, const uint64_t *row_masks, uint64_t lanes_max, int force,
                           int *fw, int *b, int *wlow, uint64_t *nstates, int32_t *col_order,
                           uint32_t *states, uint64_t states_cap);

/* perm_gray_chunk -- one chunk of the Gray-code sum of perm_glynn (algo
 * PERM_ALGO_GLYNN, square or rectangular) or of square perm_ryser (algo
 * PERM_ALGO_RYSER): the terms with Gray index k in [c 2^B, (c+1) 2^B),
 * B = chunk_log2, c = chunk, each scaled as the whole sum is (Sec. 1.2
 * Eq. glynn, Eq. glynn_rectangle, Eq. ryser_square), so that the values of the
 * 2^(nbits-B) chunks add up to the permanent (nbits = n-1 for Glynn, n for
 * Ryser; B = nbits is the whole sum, equal to perm_glynn / perm_ryser
 * bitwise).  Because g(c 2^B + k) = g(c 2^B) xor g(k) for k < 2^B, a chunk is
 * the same walk over B bits from another closed-form seed: chunks can be
 * computed on different GPUs or processes, or one after another with their
 * values kept (resuming a long evaluation), and added in double-double.
 * Floating-point outputs only (PERM_E_UNSUPPORTED for integer outputs, whose
 * partial sums are not divisible by the normalisation, and for rectangular
 * Ryser).  PERM_E_INVALID unless 1 <= B <= nbits (B = 0 when nbits = 0) and
 * c < 2^(nbits-B); m = 0 takes B = 0, c = 0 (value 1).  Flags, limits and
 * stream semantics as for perm_glynn / perm_ryser. */
int perm_gray_chunk(perm_algo algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                    perm_out ot, void *dOut, uint32_t flags, int chunk_log2, uint64_t chunk,
                    void *stream);

/* perm_column_sweep -- the definition (Sec. 1.1 Eq.
 * rectangular_permanent_definition) regrouped column by column: with g_j[R]
 * the sum over injective maps of the row set R into columns 0..j,
 *   g_j[R] = g_{j-1}[R] + sum_{i in R} a_ij g_{j-1}[R \ {i}],
 * and per(A) = g_{n-1}[all rows], over the 2^m row subsets (m = min(m, n)),
 * only the subset sizes that can still reach m at each column.  Cost about
 * n m 2^(m-1) multiply-adds and 2 2^m states of device memory (8 bytes each,
 * 16 for complex and integer outputs).  No computed value is ever subtracted,
 * so a floating-point result is within about (m + n) u per(|A|) of the true
 * value whatever the signs (the inclusion-exclusion forms can lose all digits
 * where their terms cancel).  Integer outputs are exact modulo 2^128, with
 * the overflow pre-check of perm_ryser.  Limit: min(m, n) <= 28. */
int perm_column_sweep(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                      void *dOut, uint32_t flags, void *stream);

/* perm_combinatoric -- the definition itself, one product per injective map
 * (Sec. 1.2, cost m n!/(n-m)!).  Limit: n!/(n-m)! <= 2^40 maps. */
int perm_combinatoric(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                      void *dOut, uint32_t flags, void *stream);

/* perm_auto -- ranks the algorithms whose size limits admit the shape
 * (combinatoric, Ryser, Glynn, the e_m form for m <= n, the column sweep) by
 * (m, n, density, dtype) with the learned selector if one is loaded
 * (perm_selector_load: the network predicts each one's run time), else with
 * the threshold table modelled on the paper's Alg. 5 (App. B) -- its choice
 * among the paper's three algorithms first, or the e_m form when its
 * operation count, 2^(m-1) n (min(m, 32) + 1), is below half of that choice's
 * (terms times 2n for Glynn, 2m for Ryser, m for the definition), the column
 * sweep last -- and runs the first one; if that one refuses the input with
 * PERM_E_TOO_LARGE or PERM_E_OVERFLOW (e.g. Glynn's integer sum carries an
 * extra factor 2^(n-1) (n-m)!) the next one is tried.  The value does not
 * depend on the choice beyond rounding; integer outputs are identical.
 * *chosen (may be NULL) receives the algorithm that ran.  density < 0 means
 * "unknown" (treated as 1).  Returns the last refusal if every algorithm
 * refuses. */
int perm_auto(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
              void *dOut, uint32_t flags, void *stream, double density, perm_algo *chosen);

/* ---------------------------------------------------------------------- */
/* Batched permanents                                                      */
/* ---------------------------------------------------------------------- */
/* A batch is `count` matrices inside one device buffer dData: matrix b is
 * hM[b] x hN[b] with hM[b] <= hN[b] <= 32, row-major with leading dimension
 * hLd[b] >= hN[b] (elements), starting at element offset hOffset[b].  The
 * shape arrays are HOST pointers, read during the call only.  dOut receives
 * `count` values of the output type, contiguous.  All input types and output
 * pairs of the single-matrix calls are accepted.  A matrix with hM[b] = 0 has
 * permanent 1.
 *
 * Which sum serves each matrix (the plan's algo):
 *   PERM_ALGO_GLYNN  square: Glynn's formula (Sec. 1.2 Eq. glynn);
 *                    rectangular: the rectangular Glynn sum with its n - m
 *                    padding rows summed out (the e_m form of
 *                    perm_glynn_esym: the value of Eq. glynn_rectangle without
 *                    the rounding loss of its padding), or, with
 *                    PERM_FLAG_PAD_ONES, padded with rows of ones exactly as
 *                    Eq. glynn_filled_matrix prints it;
 *   PERM_ALGO_RYSER  square only: Ryser's formula (Eq. ryser_square);
 *                    rectangular matrices give PERM_E_UNSUPPORTED;
 *   PERM_ALGO_AUTO   per matrix: rectangular -> the e_m form; square ->
 *                    Glynn for floating-point outputs (half of Ryser's terms),
 *                    Ryser for integer outputs (no extra factor 2^(n-1) in its
 *                    integer sum).
 * Integer outputs are exact under the rules of the single-matrix calls
 * (sums modulo 2^128, an overflow pre-check unless PERM_FLAG_WRAP).  For
 * 0/1 input whose shapes alone prove every result fits (|per| <= n!/(n-m)!)
 * the pre-check costs nothing; otherwise (PERM_I64 input, or 0/1 shapes near
 * the limits) every run first checks each matrix's bounds on the device and
 * waits for the flags (PERM_E_OVERFLOW if one may not fit; nothing is then
 * written).
 *
 * Square floating-point Glynn: the Gray-code terms of each matrix are cut
 * into chunks (work items); one persistent kernel per matrix order serves all
 * items of that order, every item writes its own partial slot, and one
 * finishing kernel adds each matrix's slots in a fixed order -- results are
 * bitwise reproducible for a given plan.  Orders n <= 14 run P matrices per
 * wave instead (P a power of two, 64 / P lanes per matrix, the wave's rows
 * staged in LDS): P follows a rule set by measurement (the largest P leaving
 * every lane a term within 8 KiB of LDS), or, with PERM_BATCH_AUTOTUNE, the
 * fastest P measured on the plan's own batch.  P changes how a matrix's terms
 * are split over lanes, so results of plans with different P agree to
 * rounding, not bitwise.  Every other matrix (exact integers, Ryser, the e_m
 * form) is staged: a kernel writes its update table to plan memory, and one
 * kernel per (order, term kind) walks chunks of 128 blocks per wave with the
 * single-matrix engine's update and products; its slots are added in chunk
 * order as well. */
typedef struct perm_batch_plan perm_batch_plan;

/* Build a plan (descriptors, work list, scratch) for a batch of shapes.
 * algo: PERM_ALGO_GLYNN, PERM_ALGO_RYSER or PERM_ALGO_AUTO (PERM_E_UNSUPPORTED
 * otherwise, for hM[b] > hN[b], and for a rectangular matrix under
 * PERM_ALGO_RYSER); hN[b] > 32 gives PERM_E_TOO_LARGE.  flags:
 * PERM_BATCH_AUTOTUNE, PERM_FLAG_PAD_ONES and/or PERM_FLAG_WRAP (other bits
 * PERM_E_INVALID).  The plan is bound to the current device and owns its
 * device memory.  Synchronous. */
int perm_batch_plan_create(int count, const int32_t *hM, const int32_t *hN,
                           const int64_t *hOffset, const int64_t *hLd, perm_dtype dt,
                           perm_out ot, perm_algo algo, uint32_t flags, perm_batch_plan **plan);

/* Run a plan on (dData, dOut), asynchronously on `stream`.  The first run for
 * a (dData, dOut) pair captures the launch sequence (the padding exponents of
 * rectangular matrices, the per-order kernels, the finishing kernel) into a
 * hipGraph owned by the plan; later runs with the
 * same pointers replay it with one graph launch.  Runs of one plan must not
 * overlap (they share the plan's scratch).  With PERM_BATCH_AUTOTUNE the
 * first run first times, for each small order, every admissible P (powers of
 * two up to 64 that leave each lane a term and stage at most 32 KiB in LDS)
 * on the plan's own stream after the work already queued on `stream`, three
 * launches each, keeps the fastest and waits for the timings (this run is
 * synchronous); the choice holds for the life of the plan. */
int perm_batch_plan_run(perm_batch_plan *plan, const void *dData, void *dOut, void *stream);

/* Matrices per wave the plan uses for order n: P >= 1 for a small order
 * present in the batch, 0 for an order served by the chunked kernel or absent
 * (and for n out of range).  After an autotuning plan's first run, the P it
 * chose. */
int perm_batch_plan_packing(const perm_batch_plan *plan, int n);

/* Release the plan, its graph and its device memory (NULL is ignored).  The
 * caller must make sure no run of the plan is still executing. */
int perm_batch_plan_destroy(perm_batch_plan *plan);

/* One-shot convenience: create a plan, launch it without graph capture, wait
 * for the stream, destroy the plan.  flags as for perm_batch_plan_create;
 * PERM_BATCH_AUTOTUNE has no effect here (nothing is timed).
 * perm_glynn_batched: algo PERM_ALGO_GLYNN (Sec. 1.2 Eq. glynn,
 * Eq. glynn_rectangle); perm_ryser_batched: PERM_ALGO_RYSER (Eq. ryser_square,
 * square matrices); perm_auto_batched: PERM_ALGO_AUTO. */
int perm_glynn_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                       const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                       void *dOut, uint32_t flags, void *stream);
int perm_ryser_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                       const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                       void *dOut, uint32_t flags, void *stream);
int perm_auto_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                      const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                      void *dOut, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------- */
/* Algorithm selection                                                     */
/* ---------------------------------------------------------------------- */
/* The three algorithms return the same value (Sec. 1.2); only their cost
 * differs, and which is fastest depends on the shape (Sec. 3.2 and App. B,
 * where the paper picks with a threshold table, Alg. 5).  perm_auto ranks the
 * algorithms whose size limits admit the shape either by a small network's
 * predicted run time or, when no network is loaded, by a table of Alg. 5's
 * form, and runs the first one that accepts the input. */

/* Load selector weights (the text format written by perm_selector_save);
 * path NULL unloads them (perm_auto then uses the threshold table).  Weights
 * trained on MI355X timings ship as selector_weights.txt beside the library
 * (the Python binding loads them at import); without them the built-in table
 * holds values fitted to the same timings.
 * PERM_E_INVALID if the file cannot be read or is malformed (the previous
 * weights stay loaded). */
int perm_selector_load(const char *path);

/* The selector's first choice (the algorithm perm_auto would try first),
 * without running anything, for the default output type of dt (PERM_I64 /
 * PERM_B8: exact integers).
 * *source (may be NULL) receives 1 if the network decided, 0 for the table.
 * PERM_E_TOO_LARGE if no algorithm admits the shape. */
int perm_select(int m, int n, perm_dtype dt, double density, perm_algo *chosen, int *source);

/* The selector's input features of a problem: x[0] = log min(m,n),
 * x[1] = log max(m,n), x[2] = density (fraction of nonzero entries; a
 * negative value means unknown and gives 1), x[3] = 0 for PERM_F64, 1 for
 * PERM_C128, 2 for PERM_I64 and PERM_B8.  x is a HOST array of 4 floats. */
int perm_selector_features(int m, int n, perm_dtype dt, double density, float *x);

/* perm_time -- timing of one algorithm, the selector's training data.  Runs
 * `algo` on the device matrix dA (arguments as for perm_glynn) 1 + reps times
 * on `stream`, waiting for the stream after each run, and returns in *ms the
 * median host wall time (call to completion) of the last reps runs.  With
 * fraction < 1 the algorithm's main kernel does only about that fraction of
 * the work of each lane or wave, so that a caller can extrapolate the time of
 * a long run from short ones (the time is about a + b x for the fraction x
 * run): Glynn, square Ryser and the e_m form run fewer Gray-code blocks per
 * lane (never fewer than two), in rectangular Ryser every wave stops after
 * that fraction of its share of the work (its last item's walks cut short),
 * the combinatoric sum runs whole rounds of its map prefixes (at least one),
 * so its x can differ from `fraction` by a round, and the column sweep always
 * runs whole (x = 1: its cost is bounded, at most about 0.2 s, while its
 * first columns, the cheapest, would leave only its fixed costs).  algo is
 * any perm_algo but PERM_ALGO_AUTO.  *fraction_run (may be NULL)
 * receives the fraction x actually run.  The value computed
 * is discarded.  Errors: those of the algorithm's entry point, and
 * PERM_E_INVALID for fraction outside (0, 1], reps < 1 or ms NULL.
 * Synchronous. */
int perm_time(perm_algo algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
              perm_out ot, uint32_t flags, double fraction, int reps, void *stream, double *ms,
              double *fraction_run);

/* ---- the selector network on the GPU (FP32) ----
 * Network 4 -> 64 -> 64 -> 5 with ReLU hidden layers on normalised features
 * z = (x - mean) / std, outputs y[k] = predicted log run time (ms) of
 * algorithm k in the order combinatoric, Ryser, Glynn, the e_m form
 * (perm_glynn_esym), the column sweep (perm_column_sweep).
 * Parameters: one DEVICE array of PERM_MLP_PARAMS floats,
 *   W1[64][4] | b1[64] | W2[64][64] | b2[64] | W3[5][64] | b3[5]
 * (weights row-major [output][input]); norm: DEVICE float[8] = mean[4] | std[4].
 * X: DEVICE float[batch][4]; T, Y: DEVICE float[batch][5].  A NaN target
 * (algorithm not available for that shape) takes no part in the loss
 *   L = scale * sum over finite T[b][k] of (Y[b][k] - T[b][k])^2.
 * All three are asynchronous on `stream` and deterministic (fixed-order sums). */
#define PERM_MLP_PARAMS 4805

/* Y = network(X). */
int perm_mlp_forward(const float *dParams, const float *dNorm, const float *dX, int batch,
                     float *dY, void *stream);

/* dGrad (DEVICE float[PERM_MLP_PARAMS]) = dL/dParams, *dLoss (DEVICE float,
 * may be NULL) = L.  Uses stream-ordered scratch for per-workgroup partials. */
int perm_mlp_grad(const float *dParams, const float *dNorm, const float *dX, const float *dT,
                  int batch, float scale, float *dGrad, float *dLoss, void *stream);

/* One Adam step (Kingma & Ba, 2015, with bias correction) on dParams.
 * dState: DEVICE array of 3 * PERM_MLP_PARAMS 32-bit words, zero before the
 * first step: first moments (float), second moments (float), and each
 * parameter's step count (int32).  total_steps > 0 decays the rate as
 * lr * (1 + cos(pi * min(t, total_steps) / total_steps)) / 2 at step t;
 * 0 keeps it constant. */
int perm_mlp_adam(float *dParams, const float *dGrad, float *dState, float lr, float beta1,
                  float beta2, float eps, int total_steps, void *stream);

/* Full-batch training on the GPU with the kernels above: feature statistics
 * of hX go to hNorm (HOST float[8]); with init != 0 hParams (HOST
 * float[PERM_MLP_PARAMS]) is first set from `seed` (He-uniform weights,
 * zero hidden biases, output biases at the mean finite target), otherwise
 * training starts from the values it holds.  One epoch (gradient with
 * scale = 1 / number of finite targets, Adam with beta1 0.9, beta2 0.999,
 * eps 1e-8 and cosine decay over `epochs`) is captured once in a hipGraph and
 * replayed `epochs` times.  On return hParams holds the trained parameters and
 * hLoss (HOST float[epochs], may be NULL) the loss before each step.  hX:
 * HOST float[count][4] features (perm_selector_features), hT: HOST
 * float[count][5] log run times.  Synchronous. */
int perm_selector_train(int count, const float *hX, const float *hT, int epochs, float lr,
                        uint64_t seed, int init, float *hParams, float *hNorm, float *hLoss,
                        void *stream);

/* Write a weights file for perm_selector_load: hParams (HOST, as above),
 * hNorm (HOST float[8]) and, if hTable is not NULL, threshold-table values
 * p1..p8 (HOST double[8]) in Alg. 5's form: with r = m/n,
 *   n <= p8: square and n <= p4 -> combinatoric; p1 r + p2 n + p3 > 0 ->
 *            combinatoric; otherwise Glynn;
 *   n >  p8: p5 r + p6 n + p7 > 0 -> Glynn, otherwise Ryser. */
int perm_selector_save(const char *path, const float *hParams, const float *hNorm,
                       const double *hTable);

#ifdef __cplusplus
}
#endif

#endif /* PERM_H */
