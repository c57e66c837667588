// Internal declarations shared by the host runtime (capi.cpp) and the HIP
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/perm.h"

namespace permgpu {

constexpr int kMaxN = 64;        // largest side accepted by any path

// Largest Gray-walk vector length per engine kind (the instantiated range).
#define ENGINE_MAX_NV_REAL 48
#define ENGINE_MAX_NV_CPLX 48
#define ENGINE_MAX_NV_INT 40
// Vector lengths of the paired real walk (two blocks per lane at a time).
#define GRAY_PAIR_MIN_NV 16
#define GRAY_PAIR_MAX_NV 40
#ifndef RECT_MAX_M
#define RECT_MAX_M 40
#endif
#define BATCH_MAX_N 32
constexpr int kReduceThreads = 256;

// Element kind of the Gray-code engine.
enum EngineKind : int {
  ENGINE_REAL = 0,  // binary64 sums, double-double accumulation
  ENGINE_CPLX = 1,  // complex binary64 sums, complex double-double accumulation
  ENGINE_INT = 2    // integer-valued binary64 sums (exact), products and sums mod 2^128
};

// How the engine's raw signed sum E = sum_k (-1)^k prod_j v_j(k) becomes the
// permanent.
enum FinishMode : int {
  FINISH_GLYNN = 0,     // per = E / (2^(n-1) (n-m)!)
  FINISH_RYSER_SQ = 1,  // per = (-1)^n E
  FINISH_PLAIN = 2      // per = E (weights already applied)
};

// A Gray-code walk: vector v of NV entries indexed by k in [0, 2^nbits).
//   v(0) = base,   bit q of g(k) = k ^ (k>>1) set  <=>  U[q] added.
// The update table holds, for each bit q, +U[q] (d = 0) and -U[q] (d = 1),
// at tbl[(2q + d) * NV * C + j * C + c] with C = 1 (real) or 2 (complex).
struct GrayWalk {
  const double *tbl;   // device, (2 * nbits) * NV * C doubles
  const double *base;  // device, NV * C doubles
  int nv;              // vector length
  int nbits;           // number of Gray bits (terms = 2^nbits)
  int b;               // log2 of the per-lane block length
  int prod_levels;     // ENGINE_INT only: the exact product's chunk selector
  int nonneg;          // ENGINE_INT only: every factor >= 0 (no sign to track)
  uint64_t blocks_per_lane;
  int m;               // e_m walk only: the degree (number of rows)
  // Square Ryser over a column window (engine only; null = the whole walk):
  // the top n - wshift Gray bits take only the wcount states in wlist (the
  // others leave some row sum empty), block blk walks state wlist[blk >>
  // wlow] with low block bits blk mod 2^wlow; wblocks = wcount << wlow.
  const uint32_t *wlist = nullptr;
  uint64_t wblocks = 0;
  int wlow = 0, wshift = 0;
};

// Small square walks in one workgroup (small_walk.hip): Glynn with n - 1
// and square Ryser with n Gray bits, at most SMALL_WALK_MAX_BITS bits and
// SMALL_WALK_MAX_NV entries; staging, walk, reduction and normalisation in
// one launch with no scratch memory.
#define SMALL_WALK_MAX_BITS 15
#define SMALL_WALK_MAX_NV 16
struct SmallWalk {
  int algo;  // 0 Glynn, 1 square Ryser
  int n;
  perm_dtype dt;
  const void *dA;
  int64_t lda;
  int tr;
  perm_out ot;
  int nonneg;  // ENGINE_INT: every factor >= 0 (0/1 Ryser)
};
hipError_t launch_small_walk(int kind, const SmallWalk &a, void *dOut, hipStream_t s);

// Rectangular Ryser by subset size (see ryser_rect.hip for the layout).
struct RectWalk {
  const double *colT;      // n columns of m (x C) doubles: colT[(j*m + i)*C + c]
  const double *D;         // l*l difference columns D[out*l + in] = col[in] - col[out]
  const uint32_t *trans;   // revolving-door transitions (out*l + in), all k-walks
  const uint32_t *meta32;  // k_lo[65], k_hi[65], trans offsets[66], start masks[65]
  const uint64_t *meta64;  // class cost0/item cost/items/lanes [65 each], w(s) int64/double
  const uint64_t *binom;   // C(x, t) for x, t <= 64, at [x*65 + t]
  int m, n, l, h;
  int a_lo, a_hi;
  int prod_levels;  // ENGINE_INT: the exact product's chunk selector
  int nonneg;       // ENGINE_INT: every row sum >= 0 (0/1 input)
  uint64_t total_cost;
  // Cut-down runs (timing only): each wave stops after about
  // range * cut_q / 2^32 cost units of its range, running the walks of its
  // last item only in part.  2^32 = everything.
  uint64_t cut_q;
};

// Batched Glynn: one descriptor per matrix (m <= n, row-major, ld elements),
// b = log2 of the lane block, nchunks chunks of 128 blocks, partial slots
// first_slot .. first_slot + nchunks - 1.
struct BatchMatrix {
  int64_t offset;
  int64_t ld;
  int32_t m, n;
  int32_t b;
  uint32_t nchunks;
  uint32_t first_slot;
  int32_t pad_e;  // padding rows hold 2^pad_e (set on the device for m < n; 0: ones)
};

// Padding exponents of the rectangular Glynn sum are clamped to this range
// (any nonzero padding value gives the same permanent; the range only bounds
// the conditioning it buys).
#define PAD_EXP_MAX 200

// The work items of all matrices of one order n: items [item_begin, item_end)
// of the item list, served round-robin by a persistent kernel of `grid`
// workgroups.
struct BatchBucket {
  int n;
  uint32_t item_begin, item_end;
  int grid;
  int pack = 0;  // > 0: small order, `pack` matrices per wave (batched_small.inc),
                 // one item and one slot per matrix; 0: chunked per-order kernel
};

struct BatchLaunch {
  int kind;  // ENGINE_REAL or ENGINE_CPLX
  BatchMatrix *mats;  // device descriptors (pad_e is written on the device)
  int count;
  const uint32_t *item_matrix;  // work items grouped by order n
  const uint32_t *item_chunk;
  const void *data;
  // constant padding rows, one per exponent e in [-PAD_EXP_MAX, PAD_EXP_MAX]:
  // row e holds BATCH_MAX_N entries 2^e (complex: (2^e, 0) pairs)
  const double *pad_rows;
  int scale_pad;  // 1: set each rectangular matrix's pad_e from its data first
  double *slots;
  const BatchBucket *buckets;  // host array
  int nbuckets;
  perm_out ot;
  void *out;
  const struct WalkLaunch *walk = nullptr;  // the batch's staged walks, if any
};

// Staged batch walks (batched_walk.hip / batched_walk.inc): matrices whose
// walk the per-order Glynn kernels above do not serve -- exact-integer
// batches, square Ryser, and the e_m form of rectangular matrices -- have
// their update table and start vector written to a plan-owned arena by a
// staging kernel (the single-matrix layout: row (q, d) at
// tbl[(2q + d) nv C + j C], d = 0 for +U[q], 1 for -U[q]; then base[nv C]),
// and one wave walks 128 blocks of 2^b terms (one chunk) per work item.
enum WalkType : int {
  WALK_GLYNN = 0,  // padded with rows of ones (Eq. glynn_filled_matrix), nbits = n-1
  WALK_RYSER = 1,  // square Ryser over column subsets (Eq. ryser_square), nbits = n
  WALK_ESYM = 2    // e_m form over the signs of the m rows, nbits = m-1
};
struct WalkDesc {
  int64_t offset, ld;  // the input matrix in the caller's buffer (elements)
  uint64_t arena;      // first double of its table in the arena
  int32_t m, n;        // m <= n
  int32_t walk;        // WalkType
  int32_t nv, nbits, b;
  int32_t pl;          // exact-integer kind: the product's chunk selector
  int32_t nonneg;      // exact-integer kind: every factor >= 0 (0/1 Ryser)
  uint32_t nchunks, first_slot;
};
// The walk items of one (order, term kind): items [item_begin, item_end).
struct WalkBucket {
  int nv;
  int esym;  // 0: product terms (Glynn, Ryser), 1: e_m terms
  uint32_t item_begin, item_end;
  int grid;
};
struct WalkLaunch {
  int kind;                     // ENGINE_REAL, ENGINE_CPLX or ENGINE_INT
  perm_dtype dt;                // input element type
  WalkDesc *descs;              // device
  const uint32_t *index;        // device: output index of each staged matrix
  int count;                    // staged matrices
  const uint32_t *item_desc;    // device
  const uint32_t *item_chunk;   // device
  const void *data;
  double *arena;                // device
  void *slots;                  // device, 4 doubles per slot
  const WalkBucket *buckets;    // host
  int nbuckets;
  perm_out ot;
  void *out;
};
// staging, the walk kernels of every bucket, and the per-matrix finish
hipError_t launch_walk_batch(const WalkLaunch &L, hipStream_t s);
// exact-integer batches whose bounds need the data: per-matrix product chunk
// selector into descs[i].pl and an overflow flag (1: the result may not fit ot, or an exact
// product cannot be formed) into flags[i]
hipError_t launch_walk_bounds(const WalkLaunch &L, int *flags, int wrap, hipStream_t s);
hipError_t launch_walk_bucket(int kind, const WalkBucket &bk, const WalkLaunch &L, hipStream_t s);
int walk_blocks_per_cu(int kind, int esym, int nv);

struct Finish {
  int mode;       // FinishMode
  int m, n;       // logical shape after orientation (m <= n)
  perm_out ot;
  const int *pad_exp = nullptr;  // FINISH_GLYNN, floating point: padding rows held 2^(*pad_exp)
};

// ---- launchers (each returns a hipError_t) ----
// Stage A into the update table of a Glynn walk (algo 0: padded rows of ones
// for m<n), a square Ryser walk (algo 1) or a walk over the signs of the m
// rows only (algo 2, for the e_m form); converts the input dtype; `tr` reads
// A^T.
// col_order (square Ryser only, may be null): Gray bit q toggles column
// col_order[q] of A.
hipError_t launch_stage_gray(int algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                             int tr, double *tbl, double *base, int cplx, hipStream_t s,
                             const int *pad_exp = nullptr, uint64_t g_start = 0,
                             const int32_t *col_order = nullptr);
// The exponent of the floating-point Glynn padding value (device int *e).
hipError_t launch_pad_scale(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                            int *e, hipStream_t s);

// Engine: one partial per workgroup into `partials` (real: 2 doubles,
// complex: 4 doubles, int: 2 uint64).  The walk's vector length w.nv must be
// at most ENGINE_MAX_NV_{REAL,CPLX,INT}.
hipError_t launch_gray_engine_real(const GrayWalk &w, int grid, int block, void *partials,
                                   hipStream_t s);
hipError_t launch_gray_engine_cplx(const GrayWalk &w, int grid, int block, void *partials,
                                   hipStream_t s);
hipError_t launch_gray_engine_int(const GrayWalk &w, int grid, int block, void *partials,
                                  hipStream_t s);
// Resident 256-thread workgroups per CU for an engine instantiation (0 = none).
// Walks of fewer than 8 terms (w.nbits <= 2; the engine needs blocks of at
// least 8 steps): one wave, one partial (count 1 for launch_finish).
hipError_t launch_gray_tiny(int kind, const GrayWalk &w, void *partials, hipStream_t s);
int gray_engine_blocks_per_cu_real(int nv);
int gray_engine_blocks_per_cu_cplx(int nv);
int gray_engine_blocks_per_cu_int(int nv);
// The paired real walk: GRAY_PAIR_MIN_NV <= w.nv <= GRAY_PAIR_MAX_NV, no
// column window, w.b >= 3 and w.blocks_per_lane a multiple of 4 (the caller
// guarantees them); partials as launch_gray_engine_real.
hipError_t launch_gray_engine_real_pair(const GrayWalk &w, int grid, int block, void *partials,
                                        hipStream_t s);
int gray_engine_blocks_per_cu_real_pair(int nv);

// The e_m form of the rectangular Glynn sum (esym.inc): the walk over the
// signs of rows 1..m-1 with the n column sums as its vector (w.nv = n,
// w.nbits = m-1, w.m = m <= ESYM_MAX_M); each term is +-e_m(v).  Partials as
// the real / complex / integer engine (the integer kind needs every column
// sum below 2^53 and keeps e_m modulo 2^128).
#define ESYM_MAX_M 32
hipError_t launch_esym_real(const GrayWalk &w, int grid, int block, void *partials,
                            hipStream_t s);
hipError_t launch_esym_cplx(const GrayWalk &w, int grid, int block, void *partials,
                            hipStream_t s);
hipError_t launch_esym_int(const GrayWalk &w, int grid, int block, void *partials,
                           hipStream_t s);
int esym_blocks_per_cu_real(int nv);
// Banded e_m kernels (exact degree w.m, kind ENGINE_REAL or ENGINE_CPLX):
// resident workgroups per CU, 0 if no banded kernel exists for (nv, m).
int esym_band_blocks_per_cu(int kind, int nv, int m);
hipError_t launch_esym_band(int kind, const GrayWalk &w, int grid, int block, void *partials,
                            hipStream_t s);
int esym_blocks_per_cu_cplx(int nv);
int esym_blocks_per_cu_int(int nv);

// Single-workgroup deterministic reduction of `count` partials, scaling, and
// the typed write of the result.
hipError_t launch_finish(int kind, const void *partials, int count, const Finish &f, void *dOut,
                         hipStream_t s);

// Magnitudes of the logical rows and columns of an integer matrix, in one
// pass: out[0 .. m+n) absolute sums (rows, then columns; exact, saturating
// at 2^64 - 1), out[m+n .. 2(m+n)) sums of squares (bit patterns of
// doubles), out[2(m+n) .. 2(m+n)+m) each row's nonzero mask (columns < 64).
hipError_t launch_int_stats(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                            uint64_t *out, hipStream_t s);
// out[i] = the nonzero mask of logical row i (columns < 64), any input type.
hipError_t launch_row_masks(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                            uint64_t *out, hipStream_t s);

// Rectangular Ryser staging (column table and difference columns) and engine.
hipError_t launch_stage_rect(int m, int n, int l, perm_dtype dt, const void *dA, int64_t lda,
                             int tr, double *colT, double *D, int cplx, hipStream_t s);
hipError_t launch_ryser_rect(int kind, const RectWalk &w, int grid, void *partials,
                             hipStream_t s);
hipError_t launch_ryser_rect_real(const RectWalk &w, int grid, void *partials, hipStream_t s);
hipError_t launch_ryser_rect_cplx(const RectWalk &w, int grid, void *partials, hipStream_t s);
hipError_t launch_ryser_rect_int(const RectWalk &w, int grid, void *partials, hipStream_t s);

// The definition: the n!/(n-m)! maps are `prefixes` prefixes (rows 0..q-1)
// times `suffixes` suffixes; T = grid x 256 lanes take the prefixes t, t + T,
// ... for `rounds` rounds (prefixes <= rounds T) and walk all suffixes of
// each.  One partial per workgroup.
struct CombPlan {
  int q = 0;
  uint64_t prefixes = 1, suffixes = 1;
  uint32_t rounds = 1;
  int grid = 1;
};
hipError_t launch_combinatoric(int kind, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                               int tr, const CombPlan &c, void *partials, hipStream_t s);
int combinatoric_blocks_per_cu(int kind, int m, int n);  // resident 256-thread workgroups per CU

// Batched Glynn: the per-order persistent kernels and the per-matrix finish.
hipError_t launch_batched(const BatchLaunch &L, hipStream_t s);
// the kernel of bucket i alone (no finishing kernel)
hipError_t launch_batched_bucket(const BatchLaunch &L, int i, hipStream_t s);
// Orders up to BATCH_PACK_MAX_N can run several matrices per wave.
#define BATCH_PACK_MAX_N 14
hipError_t launch_batched_small_real(int n, const BatchBucket &bk, const BatchLaunch &L,
                                     hipStream_t s);
hipError_t launch_batched_small_cplx(int n, const BatchBucket &bk, const BatchLaunch &L,
                                     hipStream_t s);
int batched_blocks_per_cu(int kind, int n);  // resident 256-thread workgroups per CU

// The column sweep (sweep.hip) on the logical m x n matrix (m <= n): two
// zeroed state buffers of state_bytes << m bytes each, the first ncols
// columns (n for the whole sum; fewer only to time part of it), the value at
// the full row set written to dOut.
#define SWEEP_MAX_M 28
hipError_t launch_sweep(int kind, int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                        void *buf0, void *buf1, size_t state_bytes, perm_out ot, void *dOut,
                        hipStream_t s, int ncols);

// Writes the value 1 in the output type (the permanent of an empty matrix).
hipError_t launch_write_one(perm_out ot, void *dOut, hipStream_t s);

}  // namespace permgpu
