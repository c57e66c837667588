// Host-side runtime declarations of libpermgpu (planning, pre-checks, the
// per-algorithm runners).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "internal.h"

namespace permgpu {

typedef unsigned __int128 u128_host;

struct GrayPlan {
  int b;                     // log2 of the per-lane block length (re-seed period)
  uint64_t lanes;            // lanes launched (a power of two)
  uint64_t blocks_per_lane;  // blocks walked by each lane (even, or 1 when lanes = 1)
  int block, grid;           // workgroup size and count
};

int device_cus();
// engine-kernel timing around one launch (no-ops unless perm_profile_enable(1))
void profile_begin(hipStream_t s);
void profile_end(hipStream_t s);
// Work truncation used only by perm_time (calling thread): the fraction of
// the main kernel's work to run (1 = all), and the fraction the last call
// actually ran (work is cut at block / item / map granularity).
double tune_fraction();
void tune_record(double ran);
void tune_set(double f);
double tune_ran();
int plan_gray(int kind, int nv, int nbits, GrayPlan &p);
int plan_gray_bpc(int bpc, int nbits, GrayPlan &p, int min_b = 1);
double esym_term_ops(int kind, int n, int m, bool band);
int plan_esym(int bpc, int nbits, double term_ops, double seed_ops, GrayPlan &p);
int engine_kind_for(perm_dtype dt, perm_out ot, int &kind);
int validate(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot, void *dOut,
             int &kind);
int int_prod_selector(const std::vector<uint64_t> &bounds);
int int_precheck(int algo, int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
                 perm_out ot, uint32_t flags, hipStream_t s, int &pl,
                 std::vector<uint64_t> *row_masks = nullptr);

// Runners on the logical M x N matrix (M <= N; tr = read A^T).
// chunk_log2 < 0: the whole walk; else the chunk of 2^chunk_log2 Gray indices
// starting at chunk * 2^chunk_log2 (floating-point outputs).  ext_scratch:
// device memory of ext_bytes bytes for the walk's tables and partials instead
// of a stream-ordered allocation (PERM_E_TOO_LARGE if it does not fit).
int run_gray(int algo, int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
             perm_out ot, void *dOut, uint32_t flags, hipStream_t s, int kind,
             int chunk_log2 = -1, uint64_t chunk = 0, void *ext_scratch = nullptr,
             size_t ext_bytes = 0);
int run_combinatoric(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
                     perm_out ot, void *dOut, uint32_t flags, hipStream_t s, int kind);
int run_sweep(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr, perm_out ot,
              void *dOut, uint32_t flags, hipStream_t s, int kind);
int run_esym(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr, perm_out ot,
             void *dOut, uint32_t flags, hipStream_t s, int kind);
int release_rect_tables(int dev);
int run_ryser_rect(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr, perm_out ot,
                   void *dOut, uint32_t flags, hipStream_t s, int kind);

}  // namespace permgpu
