// C ABI of libpermgpu: argument validation, orientation, the integer
// overflow pre-check, launch planning and scratch management.  Every step of
// the computation runs in the HIP kernels; this file only plans and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "internal.h"
#include "runtime.h"

using namespace permgpu;

namespace permgpu {

// ------------------------------------------------------------------ //
// device properties (cached per device)                               //
// ------------------------------------------------------------------ //
int device_cus() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev] = cus;
  }
  return cache[dev];
}

static int env_int(const char *name, int dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

static uint64_t pow2_floor(uint64_t x) {
  uint64_t p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}
static int ilog2(uint64_t x) {
  int r = 0;
  while (x > 1) { x >>= 1; ++r; }
  return r;
}

// ------------------------------------------------------------------ //
// optional engine-kernel timing (perm_profile_enable / perm_profile_last)  //
// ------------------------------------------------------------------ //
static std::atomic<int> g_profile{0};
// The calling thread's event pairs: every call since the last
// perm_profile_enable(1) records one pair; the events are reused by later
// sessions.
struct ProfileLog {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;     // pairs recorded in this session
  bool open = false;   // a begin without its end
};
static thread_local ProfileLog t_prof;

void profile_begin(hipStream_t s) {
  t_prof.open = false;
  if (!g_profile.load()) return;
  if (t_prof.used == t_prof.ev.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    t_prof.ev.emplace_back(a, b);
  }
  t_prof.open = hipEventRecord(t_prof.ev[t_prof.used].first, s) == hipSuccess;
}
void profile_end(hipStream_t s) {
  if (!g_profile.load() || !t_prof.open) return;
  t_prof.open = false;
  if (hipEventRecord(t_prof.ev[t_prof.used].second, s) == hipSuccess) ++t_prof.used;
}

static int profile_ms(size_t i, double *ms) {
  const auto &p = t_prof.ev[i];
  if (hipEventSynchronize(p.second) != hipSuccess) return PERM_E_HIP;
  float f = 0.f;
  if (hipEventElapsedTime(&f, p.first, p.second) != hipSuccess) return PERM_E_HIP;
  *ms = (double)f;
  return PERM_OK;
}

// ------------------------------------------------------------------ //
// work truncation for perm_time (thread-local, 1 outside perm_time)   //
// ------------------------------------------------------------------ //
static thread_local double t_tune_fraction = 1.0;
static thread_local double t_tune_ran = 1.0;
double tune_fraction() { return t_tune_fraction; }
void tune_record(double ran) { t_tune_ran = ran; }
void tune_set(double f) { t_tune_fraction = f; }
double tune_ran() { return t_tune_ran; }

// ------------------------------------------------------------------ //
// launch planning for the Gray-code engine                           //
// ------------------------------------------------------------------ //
int plan_gray(int kind, int nv, int nbits, GrayPlan &p) {
  int bpc = 0;
  switch (kind) {
    case ENGINE_REAL: bpc = gray_engine_blocks_per_cu_real(nv); break;
    case ENGINE_CPLX: bpc = gray_engine_blocks_per_cu_cplx(nv); break;
    default: bpc = gray_engine_blocks_per_cu_int(nv); break;
  }
  // the engine walks groups of 8 steps
  return plan_gray_bpc(bpc, nbits, p, 3);
}

// The plan for a walk whose kernel keeps `bpc` 256-thread workgroups resident
// per compute unit: blocks of 2^b steps, b >= min_b (unless the walk is
// shorter), as long as possible up to 2^12 while every lane gets two blocks.
int plan_gray_bpc(int bpc, int nbits, GrayPlan &p, int min_b) {
  const int cus = device_cus();
  if (bpc <= 0 || cus <= 0) return PERM_E_HIP;
  const uint64_t lanes_max = pow2_floor((uint64_t)cus * (uint64_t)bpc * 256u);
  const int lg = ilog2(lanes_max);
  int b;
  if (nbits == 0) {
    b = 0;
  } else {
    // as long as possible (up to 2^12 steps between closed-form re-seeds)
    // while every lane still gets at least two blocks
    b = nbits - lg - 1;
    b = std::max(min_b, std::min(b, 12));
    const int bo = env_int("PERM_BLOCK_LOG2", -1);
    if (bo >= min_b) b = bo;
    b = std::min(b, nbits);
  }
  const uint64_t L = 1ull << (nbits - b);
  uint64_t lanes, bpl;
  if (L == 1) {
    lanes = 1;
    bpl = 1;
  } else {
    lanes = std::min<uint64_t>(lanes_max, L / 2);
    bpl = L / lanes;  // even
  }
  p.b = b;
  p.lanes = lanes;
  p.blocks_per_lane = bpl;
  p.block = (int)std::min<uint64_t>(256, lanes);
  p.grid = (int)(lanes / (uint64_t)p.block);
  return PERM_OK;
}

// The paired real walk's plan (two blocks per lane at a time): blocks of 2^b
// steps, 3 <= b <= 12, and four or more blocks per lane on every lane the
// paired kernel keeps resident; false when the walk is too short to fill them.
static bool plan_gray_pair(int nv, int nbits, GrayPlan &p) {
  const int bpc = gray_engine_blocks_per_cu_real_pair(nv);
  const int cus = device_cus();
  if (bpc <= 0 || cus <= 0) return false;
  const uint64_t lanes = pow2_floor((uint64_t)cus * (uint64_t)bpc * 256u);
  const int lg = ilog2(lanes);
  int b = std::min(nbits - lg - 2, 12);
  const int bo = env_int("PERM_BLOCK_LOG2", -1);
  if (bo >= 0) b = bo;
  if (b < 3 || nbits - b < lg + 2) return false;
  p.b = b;
  p.lanes = lanes;
  p.blocks_per_lane = 1ull << (nbits - b - lg);
  p.block = 256;
  p.grid = (int)(lanes / 256u);
  return true;
}

// VALU operations of one e_m term on an n-vector (degree m): the n updates
// and the recurrence -- its band for the exact-degree kernels, every degree
// up to min(n, 32) plus the run-time pick of e_m for the generic ones; a
// complex operation counts 4 (a complex multiply-add), the integer kind's
// 128-bit multiply-add about 8.
double esym_term_ops(int kind, int n, int m, bool band) {
  double rec = 0.0;
  const int mv = std::min(n, ESYM_MAX_M);
  for (int j = 0; j < n; ++j) {
    if (band) {
      const int lo = std::max(1, j + 1 - (n - m)), hi = std::min(j + 1, m);
      if (hi >= lo) rec += hi - lo + 1;
    } else {
      rec += std::min(j + 1, mv);
    }
  }
  if (!band) rec += 2.0 * mv;
  switch (kind) {
    case ENGINE_CPLX: return 2.0 * n + 4.0 * rec;
    case ENGINE_INT: return n + 8.0 * rec;
    default: return n + rec;
  }
}

// The e_m walk's plan: the block length 2^b that minimises the estimated
// time, (waves per SIMD) x (blocks per lane) x (seed + 2^b terms), with the
// seed costing seed_ops per Gray bit at or above b-1.  Short walks thus keep
// every SIMD busy with short blocks; long ones amortise the seeds.  b = 0
// (one term per block, each lane its own seed; the kernel signs a block's
// first term by the parity of its index) may take one block per lane;
// longer blocks pair blocks of opposite parity, two or more per lane.
static uint64_t esym_lanes(uint64_t lanes_max, uint64_t L, int b) {
  if (L == 1) return 1;
  return std::min<uint64_t>(lanes_max, b == 0 ? L : L / 2);
}
int plan_esym(int bpc, int nbits, double term_ops, double seed_ops, GrayPlan &p) {
  const int cus = device_cus();
  if (bpc <= 0 || cus <= 0) return PERM_E_HIP;
  const uint64_t lanes_max = pow2_floor((uint64_t)cus * (uint64_t)bpc * 256u);
  const double simds = 4.0 * cus;
  int best_b = 0;
  double best = 0.0;
  for (int b = 0; b <= std::min(nbits, 12); ++b) {
    const uint64_t L = 1ull << (nbits - b);
    const uint64_t lanes = esym_lanes(lanes_max, L, b);
    const double bpl = (double)(L / lanes);
    const double waves = std::ceil((double)lanes / 64.0);
    const double wps = std::ceil(waves / simds);
    const double cost =
        wps * bpl * ((double)(nbits - std::max(b - 1, 0)) * seed_ops + (double)(1ull << b) * term_ops);
    if (b == 0 || cost <= best) {
      best = cost;
      best_b = b;
    }
  }
  const int bo = env_int("PERM_ESYM_BLOCK_LOG2", -1);
  if (bo >= 0 && bo <= nbits) best_b = bo;
  const uint64_t L = 1ull << (nbits - best_b);
  p.b = best_b;
  p.lanes = esym_lanes(lanes_max, L, best_b);
  p.blocks_per_lane = L / p.lanes;
  p.block = (int)std::min<uint64_t>(256, p.lanes);
  p.grid = (int)(p.lanes / (uint64_t)p.block);
  return PERM_OK;
}

// ------------------------------------------------------------------ //
// integer pre-check: bounds on |v_j| and on |per|                     //
// ------------------------------------------------------------------ //
static u128_host sat_mul(u128_host a, u128_host b) {
  if (a == 0 || b == 0) return 0;
  const u128_host lim = ~(u128_host)0;
  if (a > lim / b) return lim;
  return a * b;
}

// The exact-integer product's chunk selector (int_chunk_count in
// device_common.h): the fewest chunks of K = ceil(n / NCH) consecutive
// factors whose bound products all stay below 2^52; -1 if a single factor
// can reach 2^52.
int int_prod_selector(const std::vector<uint64_t> &bounds) {
  const u128_host lim = (u128_host)1 << 52;
  const int nv = (int)bounds.size();
  for (uint64_t b : bounds)
    if ((u128_host)b >= lim) return -1;
  for (int sel = kIntProdSelectors - 1; sel >= 0; --sel) {
    const int nch = std::min(int_chunk_count(sel, nv), std::max(nv, 1));
    const int K = (nv + nch - 1) / nch;
    bool ok = true;
    for (int s0 = 0; s0 < nv && ok; s0 += K) {
      u128_host prod = 1;
      for (int i = s0; i < std::min(nv, s0 + K); ++i) prod = sat_mul(prod, bounds[i]);
      if (prod >= lim) ok = false;
    }
    if (ok) return sel;
  }
  return 0;
}

// Row and column magnitudes and row nonzero masks (launch_int_stats), read
// back in one round trip.
struct IntStats {
  std::vector<uint64_t> rows, cols, sq_rows, sq_cols, masks;
};
static int read_int_stats(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
                          IntStats &st, hipStream_t s) {
  const size_t cnt = 2 * (size_t)(M + N) + (size_t)M;
  std::vector<uint64_t> h(cnt, 0);
  uint64_t *d = nullptr;
  if (hipMallocAsync((void **)&d, sizeof(uint64_t) * std::max<size_t>(cnt, 1), s) != hipSuccess)
    return PERM_E_HIP;
  hipError_t e = launch_int_stats(M, N, dt, dA, lda, tr, d, s);
  if (e == hipSuccess && cnt)
    e = hipMemcpyAsync(h.data(), d, sizeof(uint64_t) * cnt, hipMemcpyDeviceToHost, s);
  hipError_t e2 = hipFreeAsync(d, s);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return PERM_E_HIP;
  const auto at = h.begin();
  st.rows.assign(at, at + M);
  st.cols.assign(at + M, at + M + N);
  st.sq_rows.assign(at + M + N, at + 2 * M + N);
  st.sq_cols.assign(at + 2 * M + N, at + 2 * (M + N));
  st.masks.assign(at + 2 * (M + N), at + 2 * (M + N) + M);
  return PERM_OK;
}

// Fills `pl` and checks overflow for an integer run of `algo` (0 Glynn,
// 1 Ryser square/rect, 2 the e_m form) on the logical M x N matrix.
int int_precheck(int algo, int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
                 perm_out ot, uint32_t flags, hipStream_t s, int &pl,
                 std::vector<uint64_t> *row_masks) {
  const bool wrap = (flags & PERM_FLAG_WRAP) != 0;
  IntStats st;
  // one read of every magnitude (0/1 input under PERM_FLAG_WRAP needs none,
  // unless the caller wants the nonzero masks)
  if (!(dt == PERM_B8 && wrap) || row_masks) {
    int rc = read_int_stats(M, N, dt, dA, lda, tr, st, s);
    if (rc) return rc;
    if (row_masks) *row_masks = st.masks;
  }
  std::vector<uint64_t> &rows = st.rows, &cols = st.cols;
  if (dt == PERM_B8 && wrap) {
    // the bounds from the shape alone
    rows.assign(M, (uint64_t)N);
    cols.assign(N, (uint64_t)N);
  }
  if (algo == 0)  // the padding rows of ones
    for (auto &c : cols) c = (c > ~0ull - (uint64_t)N) ? ~0ull : c + (uint64_t)(N - M);
  // Glynn and Ryser form binary64 chunk products; the e_m form only needs
  // every column sum exact in binary64 (the selector is < 0 iff one is not)
  pl = int_prod_selector(algo == 1 ? rows : cols);
  if (pl < 0) return PERM_E_OVERFLOW;
  if (wrap) return PERM_OK;
  // log2 of an upper bound on |per(A)| <= per(|A|):
  //   any matrix:  prod_i sum_j |a_ij|  (each row sum bounds that row's choices)
  //   0/1 matrix:  Bregman's theorem on the square 0/1 matrix A' = [A; J] padded
  //                with N-M rows of ones, per(A') = (N-M)! per(A) and
  //                per(A') <= prod_rows (r!)^(1/r).
  double lg = 0.0;
  for (uint64_t r : rows) {
    if (r == 0) return PERM_OK;  // a zero row: per = 0
    lg += std::log2((double)r);
  }
  if (M == N) {
    // Carlen-Lieb-Loss: |per(A)| <= n!/n^(n/2) prod_j ||a_j||_2 over the columns
    // (and, applied to A^T, over the rows)
    const std::vector<uint64_t> &sq_rows = st.sq_rows, &sq_cols = st.sq_cols;
    const double base = std::lgamma((double)N + 1.0) / std::log(2.0) -
                        0.5 * (double)N * std::log2((double)N);
    double lr = base, lc = base;
    for (int i = 0; i < N; ++i) {
      double qr, qc;
      std::memcpy(&qr, &sq_rows[i], 8);
      std::memcpy(&qc, &sq_cols[i], 8);
      // each sum of squares is rounded (relative error below N u)
      lr += 0.5 * std::log2(qr * (1.0 + 1e-12));
      lc += 0.5 * std::log2(qc * (1.0 + 1e-12));
    }
    lg = std::min(lg, std::min(lr, lc));
  }
  if (dt == PERM_B8) {
    double lb = 0.0;
    for (uint64_t r : rows) lb += std::lgamma((double)r + 1.0) / std::log(2.0) / (double)r;
    lb += (double)(N - M) * std::lgamma((double)N + 1.0) / std::log(2.0) / (double)N;
    lb -= std::lgamma((double)(N - M) + 1.0) / std::log(2.0);
    lg = std::min(lg, lb);
  }
  lg = lg * (1.0 + 1e-12) + 1e-9;  // margin for rounding in the logarithms
  if (ot == PERM_OUT_I64 && lg >= 63.0) return PERM_E_OVERFLOW;
  if (lg >= 127.0) return PERM_E_OVERFLOW;
  if (algo == 0) {
    // the Glynn sum itself is 2^(N-1) (N-M)! per(A)
    double lx = lg + (double)(N - 1) + std::lgamma((double)(N - M) + 1.0) / std::log(2.0);
    if (lx >= 127.0) return PERM_E_OVERFLOW;
  } else if (algo == 2) {
    // the e_m sum is 2^(M-1) per(A)
    if (lg + (double)(M - 1) >= 127.0) return PERM_E_OVERFLOW;
  }
  return PERM_OK;
}

// ------------------------------------------------------------------ //
// validation                                                          //
// ------------------------------------------------------------------ //
int engine_kind_for(perm_dtype dt, perm_out ot, int &kind) {
  switch (dt) {
    case PERM_F64:
      if (ot != PERM_OUT_F64 && ot != PERM_OUT_DD) return PERM_E_INVALID;
      kind = ENGINE_REAL;
      return PERM_OK;
    case PERM_C128:
      if (ot != PERM_OUT_C128 && ot != PERM_OUT_CDD) return PERM_E_INVALID;
      kind = ENGINE_CPLX;
      return PERM_OK;
    case PERM_I64:
    case PERM_B8:
      if (ot == PERM_OUT_I64 || ot == PERM_OUT_I128) kind = ENGINE_INT;
      else if (ot == PERM_OUT_F64 || ot == PERM_OUT_DD) kind = ENGINE_REAL;
      else return PERM_E_INVALID;
      return PERM_OK;
    default:
      return PERM_E_INVALID;
  }
}

int validate(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot, void *dOut,
             int &kind) {
  if (m < 0 || n < 0 || dOut == nullptr) return PERM_E_INVALID;
  if ((int)ot < 0 || (int)ot > (int)PERM_OUT_CDD) return PERM_E_INVALID;
  int rc = engine_kind_for(dt, ot, kind);
  if (rc) return rc;
  if (m > 0 && n > 0) {
    if (dA == nullptr || lda < n) return PERM_E_INVALID;
  }
  return PERM_OK;
}

// ------------------------------------------------------------------ //
// square Ryser: pruning by a window of columns                       //
// ------------------------------------------------------------------ //
// Row i's sum over a column subset S is empty -- the term is zero -- when S
// misses every nonzero column of row i.  Put the columns U that hold all
// the nonzeros of some sparse rows on the top Gray bits, constant over the
// blocks of a wave: of the 2^|U| states of those bits, only the ones that
// meet every such row can give a nonzero term, and the walk visits only
// those.  Exact for any values: the skipped terms have an empty row sum.
struct RyserWindow {
  std::vector<int32_t> col_order;  // Gray bit q toggles column col_order[q]
  std::vector<uint32_t> states;    // bit p = column col_order[n - fw + p]
  int fw = 0;                      // window width
  int wlow = 0;                    // block index bits below the window state
  uint64_t wblocks = 0;            // states << wlow
  GrayPlan plan;
};

// Each row's nonzero mask (any input type), read back in one round trip.
static int read_row_masks(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
                          std::vector<uint64_t> &out, hipStream_t s) {
  out.assign(M, 0);
  uint64_t *d = nullptr;
  if (hipMallocAsync((void **)&d, sizeof(uint64_t) * (size_t)std::max(M, 1), s) != hipSuccess)
    return PERM_E_HIP;
  hipError_t e = launch_row_masks(M, N, dt, dA, lda, tr, d, s);
  if (e == hipSuccess && M > 0)
    e = hipMemcpyAsync(out.data(), d, sizeof(uint64_t) * (size_t)M, hipMemcpyDeviceToHost, s);
  hipError_t e2 = hipFreeAsync(d, s);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

// Relative time of an engine walk: blocks per lane times one block (2^b
// steps of an update and a product over nv entries, plus the closed-form
// seed of nbits - b + 1 table rows).
static double engine_walk_cost(uint64_t bpl, int nv, int nbits, int b) {
  return (double)bpl * (std::ldexp(2.0 * nv + 20.0, b) + (double)(nbits - b + 1) * nv);
}

// The window: the sparsest rows, taken while their columns fit, with the
// block length that keeps every lane busy; false if it does not save at
// least a fifth of the whole walk's time.
static bool plan_ryser_window(const std::vector<uint64_t> &masks, int n, uint64_t lanes_max,
                              bool force, RyserWindow &out) {
  const int m = (int)masks.size();
  // wave-uniform window states need 7 block-index bits below them (64
  // lanes, two block parities), and blocks are at least 8 steps
  const int fw_cap = std::min(16, n - 7 - 3);
  if (fw_cap < 0 || lanes_max < 256 || n > 64 || m != n) return false;
  // the whole walk's plan (as plan_gray_bpc makes it)
  const int b0 = std::min(n, std::max(3, std::min(n - ilog2(lanes_max) - 1, 12)));
  const uint64_t nblk = 1ull << (n - b0);
  const uint64_t bpl0 = nblk == 1 ? 1 : nblk / std::min<uint64_t>(lanes_max, nblk / 2);
  std::vector<int> rows(m);
  for (int i = 0; i < m; ++i) rows[i] = i;
  std::stable_sort(rows.begin(), rows.end(), [&](int x, int y) {
    return __builtin_popcountll(masks[x]) < __builtin_popcountll(masks[y]);
  });
  const double dense_cost = engine_walk_cost(bpl0, n, n, b0);
  // force: any window that prunes, at its best block length
  double best = force ? HUGE_VAL : 0.8 * dense_cost;
  bool found = false;
  uint64_t U = 0;
  std::vector<uint64_t> st{0};  // surviving states, as column masks within U
  for (int i : rows) {
    const uint64_t mr = masks[i];
    const uint64_t nu = U | mr;
    if (__builtin_popcountll(nu) > fw_cap) continue;
    // extend every state by each subset x of the new columns, keep those
    // that meet row i
    const uint64_t nb = mr & ~U;
    std::vector<uint64_t> nx;
    for (uint64_t t : st) {
      uint64_t x = 0;
      do {
        if ((t | x) & mr) nx.push_back(t | x);
        x = (x - nb) & nb;
      } while (x != 0);
    }
    if (nx.size() > (1u << 16)) break;
    U = nu;
    st.swap(nx);
    const int fw = __builtin_popcountll(U);
    for (int b = 3; b <= 12; ++b) {
      const int L = n - fw - b;
      if (L < 7) break;
      const uint64_t T = (uint64_t)st.size() << L;
      const uint64_t lanes = std::min<uint64_t>(lanes_max, std::max<uint64_t>(256, ((T / 2 + 255) / 256) * 256));
      const uint64_t bpl = 2 * ((T + 2 * lanes - 1) / (2 * lanes));
      const double cost = T == 0 ? 0.0 : engine_walk_cost(bpl, n, n, b);
      if (cost < best && st.size() < (1ull << fw)) {
        best = cost;
        found = true;
        out.fw = fw;
        out.wlow = L;
        out.wblocks = T;
        out.plan.b = b;
        out.plan.lanes = lanes;
        out.plan.blocks_per_lane = std::max<uint64_t>(2, bpl);
        out.plan.block = (int)std::min<uint64_t>(256, lanes);
        out.plan.grid = (int)(lanes / (uint64_t)out.plan.block);
        // window columns in ascending order on Gray bits n - fw .. n - 1
        std::vector<int> ucols;
        for (int j = 0; j < n; ++j)
          if ((U >> j) & 1u) ucols.push_back(j);
        out.col_order.clear();
        for (int j = 0; j < n; ++j)
          if (!((U >> j) & 1u)) out.col_order.push_back(j);
        for (int j : ucols) out.col_order.push_back(j);
        out.states.resize(st.size());
        for (size_t k = 0; k < st.size(); ++k) {
          uint32_t v = 0;
          for (int p = 0; p < fw; ++p)
            if ((st[k] >> ucols[p]) & 1u) v |= 1u << p;
          out.states[k] = v;
        }
      }
    }
    if (st.empty()) break;  // a row with no nonzero: nothing is left to walk
  }
  return found;
}

extern "C" int perm_ryser_window_plan(int n, const uint64_t *row_masks, uint64_t lanes_max,
                                      int force, int *fw, int *b, int *wlow, uint64_t *nstates,
                                      int32_t *col_order, uint32_t *states,
                                      uint64_t states_cap) {
  if (n < 0 || n > 64 || (n > 0 && !row_masks) || !fw || !b || !wlow || !nstates)
    return PERM_E_INVALID;
  RyserWindow win;
  const bool use = plan_ryser_window(std::vector<uint64_t>(row_masks, row_masks + n), n,
                                     lanes_max, force != 0, win);
  *fw = use ? win.fw : 0;
  *b = use ? win.plan.b : 0;
  *wlow = use ? win.wlow : 0;
  *nstates = use ? win.states.size() : 0;
  if (!use) return 0;
  if (col_order) std::copy(win.col_order.begin(), win.col_order.end(), col_order);
  if (states) {
    if (win.states.size() > states_cap) return PERM_E_TOO_LARGE;
    std::copy(win.states.begin(), win.states.end(), states);
  }
  return 1;
}

// ------------------------------------------------------------------ //
// the Gray-walk path (Glynn square/rectangular, Ryser square)        //
// ------------------------------------------------------------------ //
int run_gray(int algo, int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
             perm_out ot, void *dOut, uint32_t flags, hipStream_t s, int kind, int chunk_log2,
             uint64_t chunk, void *ext_scratch, size_t ext_bytes) {
  // algo 0: Glynn (NV = N, nbits = N-1); algo 1: square Ryser (NV = M = N, nbits = N)
  const int nv = algo == 0 ? N : M;
  const int nbits_all = algo == 0 ? N - 1 : N;
  // a chunk walks the low chunk_log2 bits from the seed of its first index
  const int nbits = chunk_log2 < 0 ? nbits_all : chunk_log2;
  const uint64_t k_first = chunk_log2 < 0 ? 0 : (chunk << chunk_log2);
  const uint64_t g_start = k_first ^ (k_first >> 1);
  const int nv_max = kind == ENGINE_REAL ? ENGINE_MAX_NV_REAL
                     : kind == ENGINE_CPLX ? ENGINE_MAX_NV_CPLX
                                           : ENGINE_MAX_NV_INT;
  if (nv > nv_max) return PERM_E_TOO_LARGE;
  // square Ryser over the whole walk: prune the column subsets that leave a
  // sparse row empty.  Integer outputs get the nonzero masks with their
  // pre-check; floating-point outputs read them (one more wait for the
  // stream, about 0.1 ms of lost overlap between calls) when the caller says
  // the input is sparse, or when the whole walk takes 2 ms or more (real
  // n >= 30, complex n >= 29), where that wait costs a dense input under 6%.
  // PERM_RYSER_WINDOW: 0 = always the whole walk, 2 = a window whenever one
  // prunes (for tests at orders where the model keeps the walk)
  const int win_mode = env_int("PERM_RYSER_WINDOW", 1);
  const bool fp_long = (kind == ENGINE_REAL && N >= 30) || (kind == ENGINE_CPLX && N >= 29);
  const bool try_win = algo == 1 && chunk_log2 < 0 && nbits >= 3 && win_mode != 0 &&
                       (kind == ENGINE_INT || fp_long || (flags & PERM_FLAG_SPARSE) != 0 ||
                        win_mode == 2);
  std::vector<uint64_t> masks;
  int pl = 3;
  if (kind == ENGINE_INT) {
    int rc = int_precheck(algo, M, N, dt, dA, lda, tr, ot, flags, s, pl,
                          try_win ? &masks : nullptr);
    if (rc) return rc;
  } else if (try_win) {
    int rc = read_row_masks(M, N, dt, dA, lda, tr, masks, s);
    if (rc) return rc;
  }
  GrayPlan plan;
  int rc = plan_gray(kind, nv, nbits, plan);
  if (rc) return rc;
  RyserWindow win;
  bool use_win = false;
  if (try_win) {
    const int bpc = kind == ENGINE_REAL   ? gray_engine_blocks_per_cu_real(nv)
                    : kind == ENGINE_CPLX ? gray_engine_blocks_per_cu_cplx(nv)
                                          : gray_engine_blocks_per_cu_int(nv);
    const uint64_t lanes_max = pow2_floor((uint64_t)device_cus() * (uint64_t)bpc * 256u);
    use_win = plan_ryser_window(masks, N, lanes_max, win_mode == 2, win);
    if (use_win) plan = win.plan;
  }
  // small square walks: one workgroup stages, walks, reduces and writes the
  // result in one launch, with no scratch memory
  if (chunk_log2 < 0 && M == N && nbits <= SMALL_WALK_MAX_BITS && nv <= SMALL_WALK_MAX_NV &&
      !use_win) {
    tune_record(1.0);
    SmallWalk sw;
    sw.algo = algo;
    sw.n = N;
    sw.dt = dt;
    sw.dA = dA;
    sw.lda = lda;
    sw.tr = tr;
    sw.ot = ot;
    sw.nonneg = kind == ENGINE_INT && dt == PERM_B8 && algo == 1;
    profile_begin(s);
    const hipError_t e = launch_small_walk(kind, sw, dOut, s);
    profile_end(s);
    return e == hipSuccess ? PERM_OK : PERM_E_HIP;
  }
  // real walks without a window: the paired kernel (one scalar row load for
  // two blocks) wherever it fills the device
  bool pair = false;
  if (kind == ENGINE_REAL && !use_win && env_int("PERM_ENGINE_PAIR", 1) != 0) {
    GrayPlan pp;
    if (plan_gray_pair(nv, nbits, pp)) {
      plan = pp;
      pair = true;
    }
  }
  uint64_t bpl_run = plan.blocks_per_lane;
  const double f = tune_fraction();
  if (f < 1.0 && plan.blocks_per_lane >= 4) {
    // keep an even count (the engine pairs blocks of opposite parity), a
    // multiple of 4 for the paired kernel
    const uint64_t unit = pair ? 4 : 2;
    bpl_run = (uint64_t)std::llround((double)plan.blocks_per_lane * f / (double)unit) * unit;
    bpl_run = std::max<uint64_t>(unit, std::min(bpl_run, plan.blocks_per_lane));
  }
  tune_record((double)bpl_run / (double)plan.blocks_per_lane);
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  const size_t tbl_n = (size_t)2 * nbits_all * nv * C;
  const size_t base_n = (size_t)nv * C;
  const size_t part_n = (size_t)plan.grid * 2 * C;
  const size_t win_n = use_win ? win.col_order.size() + win.states.size() : 0;
  const size_t bytes = sizeof(double) * (tbl_n + base_n + part_n) + 256 + sizeof(int32_t) * win_n;
  char *scratch = nullptr;
  if (ext_scratch) {
    if (bytes > ext_bytes) return PERM_E_TOO_LARGE;
    scratch = (char *)ext_scratch;
  } else if (hipMallocAsync((void **)&scratch, bytes, s) != hipSuccess) {
    return PERM_E_HIP;
  }
  double *tbl = (double *)scratch;
  double *base = tbl + tbl_n;
  double *part = base + base_n;
  // floating-point rectangular Glynn: padding rows of 2^e (chosen on the
  // device from the data) instead of ones, unless the caller asks for ones
  int *pad_exp = nullptr;
  hipError_t e = hipSuccess;
  if (algo == 0 && M < N && kind != ENGINE_INT && !(flags & PERM_FLAG_PAD_ONES)) {
    pad_exp = (int *)(part + part_n);
    e = launch_pad_scale(M, N, dt, dA, lda, tr, pad_exp, s);
  }
  int32_t *dcol = nullptr;
  uint32_t *dstates = nullptr;
  if (use_win && e == hipSuccess) {
    // column order and states: one copy, waited for before the host
    // vectors go out of scope
    std::vector<int32_t> host(win_n);
    std::copy(win.col_order.begin(), win.col_order.end(), host.begin());
    for (size_t i = 0; i < win.states.size(); ++i)
      host[win.col_order.size() + i] = (int32_t)win.states[i];
    dcol = (int32_t *)((char *)(part + part_n) + 256);
    dstates = (uint32_t *)(dcol + win.col_order.size());
    e = hipMemcpyAsync(dcol, host.data(), sizeof(int32_t) * win_n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e == hipSuccess)
    e = launch_stage_gray(algo, M, N, dt, dA, lda, tr, tbl, base, C == 2, s, pad_exp, g_start,
                          dcol);
  if (e == hipSuccess) {
    GrayWalk w;
    w.tbl = tbl;
    w.base = base;
    w.nv = nv;
    w.nbits = nbits;
    w.b = plan.b;
    w.prod_levels = pl;
    // 0/1 Ryser: row sums are never negative
    w.nonneg = kind == ENGINE_INT && dt == PERM_B8 && algo == 1;
    w.blocks_per_lane = bpl_run;
    if (use_win) {
      // never read when no state survives (wblocks = 0), but non-null
      w.wlist = win.states.empty() ? (const uint32_t *)dcol : dstates;
      w.wblocks = win.wblocks;
      w.wlow = win.wlow;
      w.wshift = N - win.fw;
    }
    profile_begin(s);
    if (nbits < 3) {
      e = launch_gray_tiny(kind, w, part, s);
    } else {
      switch (kind) {
        case ENGINE_REAL:
          e = pair ? launch_gray_engine_real_pair(w, plan.grid, plan.block, part, s)
                   : launch_gray_engine_real(w, plan.grid, plan.block, part, s);
          break;
        case ENGINE_CPLX: e = launch_gray_engine_cplx(w, plan.grid, plan.block, part, s); break;
        default: e = launch_gray_engine_int(w, plan.grid, plan.block, part, s); break;
      }
    }
    profile_end(s);
  }
  if (e == hipSuccess) {
    Finish f;
    f.mode = algo == 0 ? FINISH_GLYNN : FINISH_RYSER_SQ;
    f.m = M;
    f.n = N;
    f.ot = ot;
    f.pad_exp = pad_exp;
    e = launch_finish(kind, part, nbits < 3 ? 1 : plan.grid, f, dOut, s);
  }
  if (!ext_scratch) {
    hipError_t e2 = hipFreeAsync(scratch, s);
    if (e == hipSuccess) e = e2;
  }
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

// ------------------------------------------------------------------ //
// the e_m form of the rectangular Glynn sum                          //
// ------------------------------------------------------------------ //
int run_esym(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr, perm_out ot,
             void *dOut, uint32_t flags, hipStream_t s, int kind) {
  if (M > ESYM_MAX_M || N > 48) return PERM_E_TOO_LARGE;
  if (kind == ENGINE_INT) {
    int pl = 0;
    int rc = int_precheck(2, M, N, dt, dA, lda, tr, ot, flags, s, pl);
    if (rc) return rc;
  }
  const int nv = N, nbits = M - 1;
  // exact-degree (banded) kernels exist for the floating-point kinds at m >= 14
  // (PERM_ESYM_GENERIC=1 keeps the generic kernels: a cross-check of the two)
  const int band_bpc = kind == ENGINE_INT || env_int("PERM_ESYM_GENERIC", 0) == 1
                           ? 0
                           : esym_band_blocks_per_cu(kind, nv, M);
  const int bpc = band_bpc > 0            ? band_bpc
                  : kind == ENGINE_CPLX ? esym_blocks_per_cu_cplx(nv)
                  : kind == ENGINE_INT  ? esym_blocks_per_cu_int(nv)
                                        : esym_blocks_per_cu_real(nv);
  GrayPlan plan;
  int rc = plan_esym(bpc, nbits, esym_term_ops(kind, nv, M, band_bpc > 0),
                     (double)(nv * (kind == ENGINE_CPLX ? 2 : 1)), plan);
  if (rc) return rc;
  uint64_t bpl_run = plan.blocks_per_lane;
  const double f = tune_fraction();
  if (f < 1.0 && plan.blocks_per_lane >= 4) {
    bpl_run = (uint64_t)std::llround((double)plan.blocks_per_lane * f / 2.0) * 2;
    bpl_run = std::max<uint64_t>(2, std::min(bpl_run, plan.blocks_per_lane));
  }
  tune_record((double)bpl_run / (double)plan.blocks_per_lane);
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  const size_t tbl_n = (size_t)2 * nbits * nv * C;
  const size_t base_n = (size_t)nv * C;
  const size_t part_n = (size_t)plan.grid * 2 * C;
  char *scratch = nullptr;
  if (hipMallocAsync((void **)&scratch, sizeof(double) * (tbl_n + base_n + part_n) + 256, s) !=
      hipSuccess)
    return PERM_E_HIP;
  double *tbl = (double *)scratch;
  double *base = tbl + tbl_n;
  double *part = base + base_n;
  hipError_t e = launch_stage_gray(2, M, N, dt, dA, lda, tr, tbl, base, C == 2, s);
  if (e == hipSuccess) {
    GrayWalk w;
    w.tbl = tbl;
    w.base = base;
    w.nv = nv;
    w.nbits = nbits;
    w.b = plan.b;
    w.prod_levels = 0;
    w.nonneg = 0;
    w.blocks_per_lane = bpl_run;
    w.m = M;
    profile_begin(s);
    e = band_bpc > 0         ? launch_esym_band(kind, w, plan.grid, plan.block, part, s)
        : kind == ENGINE_CPLX ? launch_esym_cplx(w, plan.grid, plan.block, part, s)
        : kind == ENGINE_INT  ? launch_esym_int(w, plan.grid, plan.block, part, s)
                              : launch_esym_real(w, plan.grid, plan.block, part, s);
    profile_end(s);
  }
  if (e == hipSuccess) {
    Finish fin;
    fin.mode = FINISH_GLYNN;  // E / 2^(M-1): no padding rows
    fin.m = M;
    fin.n = M;
    fin.ot = ot;
    e = launch_finish(kind, part, plan.grid, fin, dOut, s);
  }
  hipError_t e2 = hipFreeAsync(scratch, s);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

// ------------------------------------------------------------------ //
// the column sweep                                                    //
// ------------------------------------------------------------------ //
int run_sweep(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr, perm_out ot,
              void *dOut, uint32_t flags, hipStream_t s, int kind) {
  if (M > SWEEP_MAX_M) return PERM_E_TOO_LARGE;
  if (kind == ENGINE_INT) {
    // the states are permanents of submatrices, kept modulo 2^128: the value
    // is exact when |per| < 2^127 (the Ryser bound of the pre-check)
    int pl = 0;
    int rc = int_precheck(1, M, N, dt, dA, lda, tr, ot, flags, s, pl);
    if (rc == PERM_E_OVERFLOW && (flags & PERM_FLAG_WRAP)) rc = PERM_OK;
    if (rc) return rc;
  }
  // perm_time runs the sweep whole: its cost is bounded (at most 28 rows,
  // about 0.2 s), and a cut through its first columns -- the cheapest ones,
  // the state band still narrow -- leaves only the fixed costs to time
  const int ncols = N;
  tune_record(1.0);
  const size_t sb = kind == ENGINE_REAL ? 8 : 16;
  const size_t bytes = sb << M;
  char *buf = nullptr;
  if (hipMallocAsync((void **)&buf, 2 * bytes, s) != hipSuccess) return PERM_E_HIP;
  profile_begin(s);
  hipError_t e = launch_sweep(kind, M, N, dt, dA, lda, tr, buf, buf + bytes, sb, ot, dOut, s, ncols);
  profile_end(s);
  hipError_t e2 = hipFreeAsync(buf, s);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

}  // namespace permgpu

// ==================================================================== //
// public entry points                                                  //
// ==================================================================== //
extern "C" {

int perm_version(void) { return PERM_VERSION; }

int perm_workspace_release(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PERM_E_HIP;
  if (hipDeviceSynchronize() != hipSuccess) return PERM_E_HIP;
  int rc = release_rect_tables(dev);
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess || hipMemPoolTrimTo(pool, 0) != hipSuccess)
    rc = PERM_E_HIP;
  return rc;
}

int perm_profile_enable(int on) {
  g_profile.store(on ? 1 : 0);
  if (on) t_prof.used = 0;
  return PERM_OK;
}

int perm_profile_last(double *ms) {
  if (!ms) return PERM_E_INVALID;
  if (t_prof.used == 0) return PERM_E_INVALID;
  return profile_ms(t_prof.used - 1, ms);
}

int perm_profile_durations(double *ms, int capacity, int *count) {
  if (!count || capacity < 0 || (capacity > 0 && !ms)) return PERM_E_INVALID;
  *count = (int)t_prof.used;
  for (size_t i = 0; i < t_prof.used && i < (size_t)capacity; ++i) {
    int rc = profile_ms(i, &ms[i]);
    if (rc) return rc;
  }
  return PERM_OK;
}

const char *perm_status_string(int status) {
  switch (status) {
    case PERM_OK: return "success";
    case PERM_E_INVALID: return "invalid argument";
    case PERM_E_TOO_LARGE: return "matrix too large for this algorithm";
    case PERM_E_OVERFLOW: return "integer result may overflow the output type";
    case PERM_E_HIP: return "HIP runtime error";
    case PERM_E_UNSUPPORTED: return "unsupported combination of arguments";
    default: return "unknown status";
  }
}

int perm_glynn(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot, void *dOut,
               uint32_t flags, void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = std::min(m, n), N = std::max(m, n);
  if (M == 0) return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  if (N > kMaxN) return PERM_E_TOO_LARGE;
  return run_gray(0, M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind);
}

int perm_glynn_esym(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                    void *dOut, uint32_t flags, void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = std::min(m, n), N = std::max(m, n);
  if (M == 0) return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  return run_esym(M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind);
}

int perm_gray_chunk(perm_algo algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                    perm_out ot, void *dOut, uint32_t flags, int chunk_log2, uint64_t chunk,
                    void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  if (algo != PERM_ALGO_GLYNN && algo != PERM_ALGO_RYSER) return PERM_E_UNSUPPORTED;
  if (kind == ENGINE_INT) return PERM_E_UNSUPPORTED;  // partial sums are not divisible
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = std::min(m, n), N = std::max(m, n);
  if (algo == PERM_ALGO_RYSER && M != N) return PERM_E_UNSUPPORTED;
  if (M == 0) {
    if (chunk_log2 != 0 || chunk != 0) return PERM_E_INVALID;
    return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  }
  if (N > kMaxN) return PERM_E_TOO_LARGE;
  const int nbits = algo == PERM_ALGO_GLYNN ? N - 1 : N;
  // a chunk starts at an even index (its terms keep their signs): at least
  // 2 indices, unless the whole walk is a single term
  if (chunk_log2 < (nbits > 0 ? 1 : 0) || chunk_log2 > nbits) return PERM_E_INVALID;
  if (chunk >= (1ull << (nbits - chunk_log2))) return PERM_E_INVALID;
  return run_gray(algo == PERM_ALGO_GLYNN ? 0 : 1, M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind,
                  chunk_log2, chunk);
}

int perm_column_sweep(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                      void *dOut, uint32_t flags, void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = std::min(m, n), N = std::max(m, n);
  if (M == 0) return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  if (N > kMaxN) return PERM_E_TOO_LARGE;
  return run_sweep(M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind);
}

int perm_ryser(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot, void *dOut,
               uint32_t flags, void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = std::min(m, n), N = std::max(m, n);
  if (M == 0) return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  if (N > kMaxN) return PERM_E_TOO_LARGE;
  if (M == N) return run_gray(1, M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind);
  return run_ryser_rect(M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind);
}

}  // extern "C"
