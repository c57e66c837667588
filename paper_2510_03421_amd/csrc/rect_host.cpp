// Host planning of the rectangular Ryser-by-size walk: column split, the
// revolving-door transition tables, class costs and weights, scratch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "runtime.h"

namespace permgpu {
namespace {

uint64_t binom_u64(int x, int t) {
  if (t < 0 || t > x) return 0;
  u128_host r = 1;
  for (int i = 1; i <= t; ++i) r = r * (u128_host)(x - t + i) / (u128_host)i;
  return (uint64_t)r;
}

// Revolving-door walks over the k-subsets of {0..l-1}: the weight-k words in
// the order of the reflected binary Gray code.  Consecutive words differ by
// one column leaving and one entering; a transition is stored as out*l + in.
struct DoorTables {
  std::vector<uint32_t> trans;     // all walks, k = 0..l
  std::vector<uint32_t> offset;    // l + 2 entries
  std::vector<uint32_t> start;     // first word of each walk
};

const DoorTables &door_tables(int l) {
  static std::mutex mu;
  static std::map<int, DoorTables> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(l);
  if (it != cache.end()) return it->second;
  DoorTables t;
  std::vector<std::vector<uint32_t>> walks(l + 1);
  std::vector<int64_t> last(l + 1, -1);
  t.start.assign(l + 1, 0);
  for (uint64_t i = 0; i < (1ull << l); ++i) {
    const uint32_t gword = (uint32_t)(i ^ (i >> 1));
    const int k = __builtin_popcount(gword);
    if (last[k] < 0) {
      t.start[k] = gword;
    } else {
      const uint32_t prev = (uint32_t)last[k];
      const uint32_t diff = prev ^ gword;
      const int out = __builtin_ctz(prev & diff);
      const int in = __builtin_ctz(gword & diff);
      walks[k].push_back((uint32_t)(out * l + in));
    }
    last[k] = gword;
  }
  t.offset.assign(l + 2, 0);
  for (int k = 0; k <= l; ++k) {
    t.offset[k + 1] = t.offset[k] + (uint32_t)walks[k].size();
    t.trans.insert(t.trans.end(), walks[k].begin(), walks[k].end());
  }
  return cache.emplace(l, std::move(t)).first->second;
}

// Device copies of the transition tables (per device and l) and of the
// binomial table (per device), uploaded once and kept until the process ends.
struct DevTables {
  uint32_t *trans = nullptr;
  uint64_t *binom = nullptr;
};

std::mutex g_tables_mu;
std::map<std::pair<int, int>, uint32_t *> g_trans_cache;
std::map<int, uint64_t *> g_binom_cache;

int device_tables(int l, DevTables &out) {
  auto &mu = g_tables_mu;
  auto &trans_cache = g_trans_cache;
  auto &binom_cache = g_binom_cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PERM_E_HIP;
  const DoorTables &t = door_tables(l);
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(dev, l);
  if (!trans_cache.count(key)) {
    uint32_t *d = nullptr;
    const size_t bytes = sizeof(uint32_t) * std::max<size_t>(1, t.trans.size());
    if (hipMalloc((void **)&d, bytes) != hipSuccess) return PERM_E_HIP;
    if (!t.trans.empty() &&
        hipMemcpy(d, t.trans.data(), sizeof(uint32_t) * t.trans.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
      (void)hipFree(d);
      return PERM_E_HIP;
    }
    trans_cache[key] = d;
  }
  if (!binom_cache.count(dev)) {
    std::vector<uint64_t> b(65 * 65);
    for (int x = 0; x <= 64; ++x)
      for (int k = 0; k <= 64; ++k) b[x * 65 + k] = binom_u64(x, k);
    uint64_t *d = nullptr;
    if (hipMalloc((void **)&d, sizeof(uint64_t) * b.size()) != hipSuccess) return PERM_E_HIP;
    if (hipMemcpy(d, b.data(), sizeof(uint64_t) * b.size(), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return PERM_E_HIP;
    }
    binom_cache[dev] = d;
  }
  out.trans = trans_cache[key];
  out.binom = binom_cache[dev];
  return PERM_OK;
}

struct ClassPlan {
  int l, h, a_lo, a_hi;
  uint64_t cost0[65], item_cost[65], items[65], lanes[65];
  uint32_t k_lo[65], k_hi[65];
  uint64_t total_cost, total_items;
};

void plan_classes(int M, int N, int l, ClassPlan &c) {
  std::memset(&c, 0, sizeof c);
  c.l = l;
  c.h = N - l;
  c.a_lo = 0;
  c.a_hi = std::min(c.h, M);
  uint64_t acc = 0;
  for (int a = 0; a <= 64; ++a) {
    c.cost0[a] = acc;
    if (a < c.a_lo || a > c.a_hi) continue;
    const int klo = std::max(0, 1 - a), khi = std::min(l, M - a);
    if (klo > khi) continue;
    c.k_lo[a] = (uint32_t)klo;
    c.k_hi[a] = (uint32_t)khi;
    uint64_t steps = 0;
    // fixed work of an item in step units (a step: m adds, m - 1 multiplies
    // and the accumulation): rebuilding the H row sums, and per walk its first
    // subset, its first term and the weighted accumulation
    const uint64_t step_ops = 2 * (uint64_t)M + 6;
    uint64_t ops = (uint64_t)a * (uint64_t)M + 20;
    for (int k = klo; k <= khi; ++k) {
      steps += binom_u64(l, k);
      ops += (uint64_t)k * (uint64_t)M + 40;
    }
    c.item_cost[a] = steps + (ops + step_ops - 1) / step_ops;
    c.lanes[a] = binom_u64(c.h, a);
    c.items[a] = (c.lanes[a] + 63) / 64;
    c.total_items += c.items[a];
    acc += c.items[a] * c.item_cost[a];
  }
  c.total_cost = acc;
}

}  // namespace

// Frees the cached device tables of `dev` (they are rebuilt on next use).
int release_rect_tables(int dev) {
  std::lock_guard<std::mutex> g(g_tables_mu);
  int rc = PERM_OK;
  for (auto it = g_trans_cache.begin(); it != g_trans_cache.end();) {
    if (it->first.first == dev) {
      if (hipFree(it->second) != hipSuccess) rc = PERM_E_HIP;
      it = g_trans_cache.erase(it);
    } else {
      ++it;
    }
  }
  auto b = g_binom_cache.find(dev);
  if (b != g_binom_cache.end()) {
    if (hipFree(b->second) != hipSuccess) rc = PERM_E_HIP;
    g_binom_cache.erase(b);
  }
  return rc;
}

int run_ryser_rect(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr, perm_out ot,
                   void *dOut, uint32_t flags, hipStream_t s, int kind) {
  if (M > RECT_MAX_M) return PERM_E_TOO_LARGE;
  int pl = 3;
  if (kind == ENGINE_INT) {
    int rc = int_precheck(1, M, N, dt, dA, lda, tr, ot, flags, s, pl);
    if (rc) return rc;
  }
  const int cus = device_cus();
  if (cus <= 0) return PERM_E_HIP;
  const uint64_t P_target = (uint64_t)cus * 16;  // one wave per SIMD slot, 4 per SIMD
  // largest low-part width (<= 20) that still leaves >= 64 items per wave
  int l = std::min(20, N - 1);
  ClassPlan cp;
  for (; l > 1; --l) {
    plan_classes(M, N, l, cp);
    if (cp.total_items >= 64 * P_target) break;
  }
  plan_classes(M, N, l, cp);
  uint64_t waves = std::min<uint64_t>(P_target, std::max<uint64_t>(1, cp.total_items));
  waves = (waves + 3) / 4 * 4;
  const int grid = (int)(waves / 4);

  DevTables dt_;
  int rc = device_tables(l, dt_);
  if (rc) return rc;
  const DoorTables &door = door_tables(l);

  // metadata
  std::vector<uint64_t> meta64(390, 0);
  std::vector<uint32_t> meta32(261, 0);
  for (int a = 0; a < 65; ++a) {
    meta64[a] = cp.cost0[a];
    meta64[65 + a] = cp.item_cost[a];
    meta64[130 + a] = cp.items[a];
    meta64[195 + a] = cp.lanes[a];
    meta32[a] = cp.k_lo[a];
    meta32[65 + a] = cp.k_hi[a];
  }
  for (int s_ = 0; s_ <= M; ++s_) {
    // w(s) = (-1)^(M-s) C(N-s, M-s)
    const uint64_t b = binom_u64(N - s_, M - s_);
    const int64_t wi = ((M - s_) & 1) ? -(int64_t)b : (int64_t)b;
    const double wf = ((M - s_) & 1) ? -(double)b : (double)b;
    std::memcpy(&meta64[260 + s_], &wi, 8);
    std::memcpy(&meta64[325 + s_], &wf, 8);
  }
  for (int k = 0; k <= l + 1 && k < 66; ++k) meta32[130 + k] = door.offset[std::min(k, l + 1)];
  for (int k = 0; k <= l; ++k) meta32[196 + k] = door.start[k];

  const int C = kind == ENGINE_CPLX ? 2 : 1;
  const size_t colT_n = (size_t)N * M * C, D_n = (size_t)l * l * M * C;
  const size_t part_n = (size_t)waves * 2 * C;
  const size_t bytes = 8 * (colT_n + D_n + part_n + meta64.size()) + 4 * meta32.size() + 512;
  char *scratch = nullptr;
  if (hipMallocAsync((void **)&scratch, bytes, s) != hipSuccess) return PERM_E_HIP;
  double *colT = (double *)scratch;
  double *D = colT + colT_n;
  double *part = D + D_n;
  uint64_t *m64 = (uint64_t *)(part + part_n);
  uint32_t *m32 = (uint32_t *)(m64 + meta64.size());
  hipError_t e = hipMemcpyAsync(m64, meta64.data(), 8 * meta64.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m32, meta32.data(), 4 * meta32.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_stage_rect(M, N, l, dt, dA, lda, tr, colT, D, C == 2, s);
  if (e == hipSuccess) {
    RectWalk w;
    w.colT = colT;
    w.D = D;
    w.trans = dt_.trans;
    w.meta32 = m32;
    w.meta64 = m64;
    w.binom = dt_.binom;
    w.m = M;
    w.n = N;
    w.l = l;
    w.h = N - l;
    w.a_lo = cp.a_lo;
    w.a_hi = cp.a_hi;
    w.prod_levels = pl;
    w.nonneg = kind == ENGINE_INT && dt == PERM_B8;  // 0/1 row sums are never negative
    w.total_cost = cp.total_cost;
    w.cut_q = 1ull << 32;
    const double f = tune_fraction();
    if (f < 1.0) {
      // every wave stops after about f of its share, whatever its items
      w.cut_q = std::max<uint64_t>(1, (uint64_t)std::ldexp(f, 32));
      tune_record(std::ldexp((double)w.cut_q, -32));
    } else {
      tune_record(1.0);
    }
    profile_begin(s);
    e = launch_ryser_rect(kind, w, grid, part, s);
    profile_end(s);
  }
  if (e == hipSuccess) {
    Finish f;
    f.mode = FINISH_PLAIN;
    f.m = M;
    f.n = N;
    f.ot = ot;
    e = launch_finish(kind, part, (int)waves, f, dOut, s);
  }
  hipError_t e2 = hipFreeAsync(scratch, s);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

}  // namespace permgpu
