// C ABI of the batched path: planning (descriptors, work items grouped by
// matrix order, scratch), graph capture and replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace permgpu;

struct perm_batch_plan {
  int dev = 0;
  int count = 0;
  int kind = ENGINE_REAL;
  perm_out ot = PERM_OUT_F64;
  std::vector<BatchBucket> buckets;
  BatchMatrix *d_mats = nullptr;
  uint32_t *d_item_matrix = nullptr;
  uint32_t *d_item_chunk = nullptr;
  double *d_slots = nullptr;
  double *d_pad_rows = nullptr;  // constant rows 2^e, e in [-PAD_EXP_MAX, PAD_EXP_MAX]
  int scale_pad = 0;             // rectangular matrices with scaled padding rows
  // the captured launch sequence for one (data, out) pair
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *g_data = nullptr;
  void *g_out = nullptr;
  // PERM_BATCH_AUTOTUNE: the matrices per wave of the small orders are timed
  // on the first run
  bool autotune = false;
  bool tuned = false;
  // staged walks (exact-integer batches, Ryser, the e_m form of rectangular
  // matrices)
  perm_dtype dt = PERM_F64;
  uint32_t flags = 0;
  int wcount = 0;
  std::vector<WalkBucket> wbuckets;
  WalkDesc *d_wdescs = nullptr;
  uint32_t *d_windex = nullptr;
  uint32_t *d_witem_desc = nullptr;
  uint32_t *d_witem_chunk = nullptr;
  double *d_arena = nullptr;
  double *d_wslots = nullptr;
  int *d_wflags = nullptr;
  bool int_check = false;  // run the exact-integer pre-check on the data
  WalkLaunch wl;           // filled per run (data and output pointers)
};

namespace {

void release(perm_batch_plan *p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->capture_stream) hipStreamDestroy(p->capture_stream);
  hipFree(p->d_mats);
  hipFree(p->d_item_matrix);
  hipFree(p->d_item_chunk);
  hipFree(p->d_slots);
  hipFree(p->d_pad_rows);
  hipFree(p->d_wdescs);
  hipFree(p->d_windex);
  hipFree(p->d_witem_desc);
  hipFree(p->d_witem_chunk);
  hipFree(p->d_arena);
  hipFree(p->d_wslots);
  hipFree(p->d_wflags);
  delete p;
}

// log2 of the lane-block length for a matrix with 2^nbits terms: long blocks
// (fewer closed-form seeds) but at least 128 blocks (one wave's two passes)
// when the matrix is large enough.
int batch_block_log2(int nbits) {
  static const int cap = [] {
    const char *e = std::getenv("PERM_BATCH_BLOCK_LOG2");
    const int v = e ? std::atoi(e) : 9;
    return v >= 0 && v <= 16 ? v : 9;
  }();
  int b = nbits - 7;  // 2^7 = 128 blocks per chunk
  return std::max(0, std::min(b, cap));
}

// Orders up to this many columns run several matrices per wave.
int pack_max_n() {
  static const int v = [] {
    const char *e = std::getenv("PERM_BATCH_PACK_MAX_N");
    const int x = e ? std::atoi(e) : BATCH_PACK_MAX_N;
    return x >= 0 && x <= BATCH_PACK_MAX_N ? x : BATCH_PACK_MAX_N;
  }();
  return v;
}

// Matrices per wave for order n: the largest power of two P <= 64 that leaves
// every lane at least one term (64 / P <= 2^(n-1)) and keeps the wave's
// staged rows and column sums within 8 KiB of LDS.  The LDS bound was set by
// a sweep of P at orders 4..14 (200,000 matrices each): more matrices per wave
// mean fewer seeds per term but fewer resident waves, and 8 KiB picks the
// fastest P, or one within 10% of it, at every point measured.
// PERM_BATCH_PACK forces a value when it leaves every lane a term.
constexpr size_t kPackLdsMax = 32768;  // the largest staging measured (and tuned over)

bool pack_admissible(int n, int C, int P, size_t budget) {
  const size_t per = sizeof(double) * (size_t)(n * n + n) * C;
  return P >= 1 && P <= 64 && (P & (P - 1)) == 0 && (64 / P) <= (1 << (n - 1)) &&
         (size_t)P * per <= budget;
}

int pack_for(int n, int C) {
  if (const char *e = std::getenv("PERM_BATCH_PACK")) {
    const int P = std::atoi(e);
    if (pack_admissible(n, C, P, kPackLdsMax)) return P;
  }
  for (int P = 64; P >= 1; P >>= 1)
    if (pack_admissible(n, C, P, 8192)) return P;
  return 0;
}

BatchLaunch make_launch(const perm_batch_plan *p, const void *data, void *out) {
  BatchLaunch L;
  L.kind = p->kind;
  L.mats = p->d_mats;
  L.count = p->count;
  L.item_matrix = p->d_item_matrix;
  L.item_chunk = p->d_item_chunk;
  L.data = data;
  L.pad_rows = p->d_pad_rows;
  L.scale_pad = p->scale_pad;
  L.slots = p->d_slots;
  L.buckets = p->buckets.data();
  L.nbuckets = (int)p->buckets.size();
  L.ot = p->ot;
  L.out = out;
  L.walk = nullptr;
  return L;
}

// The staged walks' launch record for (data, out), kept in the plan (the
// batch launch refers to it).
const WalkLaunch *make_walk(perm_batch_plan *p, const void *data, void *out) {
  if (p->wcount == 0) return nullptr;
  WalkLaunch &w = p->wl;
  w.kind = p->kind;
  w.dt = p->dt;
  w.descs = p->d_wdescs;
  w.index = p->d_windex;
  w.count = p->wcount;
  w.item_desc = p->d_witem_desc;
  w.item_chunk = p->d_witem_chunk;
  w.data = data;
  w.arena = p->d_arena;
  w.slots = p->d_wslots;
  w.buckets = p->wbuckets.data();
  w.nbuckets = (int)p->wbuckets.size();
  w.ot = p->ot;
  w.out = out;
  return &w;
}

BatchLaunch full_launch(perm_batch_plan *p, const void *data, void *out) {
  BatchLaunch L = make_launch(p, data, out);
  L.walk = make_walk(p, data, out);
  return L;
}

// Exact-integer batches whose bounds the shapes alone do not settle: the
// per-matrix pre-check on the device (product-tree depths into the staged
// descriptors) and, unless every result may wrap, the wait for its flags.
int batch_int_precheck(perm_batch_plan *p, const void *data, hipStream_t s) {
  if (!p->int_check) return PERM_OK;
  const WalkLaunch *w = make_walk(p, data, nullptr);
  if (launch_walk_bounds(*w, p->d_wflags, (p->flags & PERM_FLAG_WRAP) != 0, s) != hipSuccess)
    return PERM_E_HIP;
  std::vector<int> flags(p->wcount);
  if (hipMemcpyAsync(flags.data(), p->d_wflags, sizeof(int) * flags.size(), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PERM_E_HIP;
  for (int f : flags)
    if (f) return PERM_E_OVERFLOW;
  return PERM_OK;
}

// log2 of an upper bound on the magnitude of the integer sum a walk forms on
// an m x n 0/1 matrix (|per| <= n!/(n-m)! injective maps), for the shape-only
// overflow check of 0/1 batches; `per_only` gives the bound on |per| itself.
double b8_log2_bound(int walk, int m, int n, bool per_only) {
  double lg = std::lgamma((double)n + 1.0) / std::log(2.0) -
              std::lgamma((double)(n - m) + 1.0) / std::log(2.0);
  if (per_only) return lg;
  if (walk == WALK_GLYNN) lg += (double)(n - 1) + std::lgamma((double)(n - m) + 1.0) / std::log(2.0);
  if (walk == WALK_ESYM) lg += (double)(m - 1);
  return lg;
}

// Times every admissible P of each small order on the caller's data (three
// launches of that order's kernel alone, the first not counted) and keeps the
// fastest.  The launches run on the plan's stream after the work queued on
// `s`; the slots they write are written again by the run that follows.
int autotune_packing(perm_batch_plan *p, const void *dData, void *dOut, hipStream_t s) {
  hipEvent_t ready = nullptr, e0 = nullptr, e1 = nullptr;
  int rc = PERM_OK;
  if (hipEventCreate(&ready) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    rc = PERM_E_HIP;
  hipStream_t cs = p->capture_stream;
  if (!rc && (hipEventRecord(ready, s) != hipSuccess || hipStreamWaitEvent(cs, ready, 0) != hipSuccess))
    rc = PERM_E_HIP;
  const int C = p->kind == ENGINE_CPLX ? 2 : 1;
  BatchLaunch L = make_launch(p, dData, dOut);
  for (size_t i = 0; i < p->buckets.size() && !rc; ++i) {
    BatchBucket &bk = p->buckets[i];
    if (bk.pack <= 0) continue;
    const uint32_t items = bk.item_end - bk.item_begin;
    int best = bk.pack;
    float best_ms = 0.0f;
    for (int P = 1; P <= 64 && !rc; P <<= 1) {
      if (!pack_admissible(bk.n, C, P, kPackLdsMax)) continue;
      bk.pack = P;
      bk.grid = (int)((items + (uint32_t)P - 1) / (uint32_t)P);
      for (int r = 0; r < 3 && !rc; ++r) {
        float ms = 0.0f;
        if (hipEventRecord(e0, cs) != hipSuccess || launch_batched_bucket(L, (int)i, cs) != hipSuccess ||
            hipEventRecord(e1, cs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = PERM_E_HIP;
          break;
        }
        if (r > 0 && (best_ms == 0.0f || ms < best_ms)) {
          best_ms = ms;
          best = P;
        }
      }
    }
    bk.pack = best;
    bk.grid = (int)((items + (uint32_t)best - 1) / (uint32_t)best);
  }
  if (ready) (void)hipEventDestroy(ready);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

template <class T>
int upload(T **dst, const std::vector<T> &src) {
  const size_t bytes = sizeof(T) * std::max<size_t>(1, src.size());
  if (hipMalloc((void **)dst, bytes) != hipSuccess) return PERM_E_HIP;
  if (!src.empty() &&
      hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
    return PERM_E_HIP;
  return PERM_OK;
}

}  // namespace

extern "C" {

int perm_batch_plan_create(int count, const int32_t *hM, const int32_t *hN,
                           const int64_t *hOffset, const int64_t *hLd, perm_dtype dt,
                           perm_out ot, perm_algo algo, uint32_t flags, perm_batch_plan **plan) {
  if (!plan) return PERM_E_INVALID;
  *plan = nullptr;
  if (flags & ~(PERM_BATCH_AUTOTUNE | PERM_FLAG_PAD_ONES | PERM_FLAG_WRAP)) return PERM_E_INVALID;
  if (count < 0 || (count > 0 && (!hM || !hN || !hOffset || !hLd))) return PERM_E_INVALID;
  int kind = 0;
  int rc = engine_kind_for(dt, ot, kind);
  if (rc) return rc;
  if (algo != PERM_ALGO_GLYNN && algo != PERM_ALGO_RYSER && algo != PERM_ALGO_AUTO)
    return PERM_E_UNSUPPORTED;
  for (int i = 0; i < count; ++i) {
    if (hM[i] < 0 || hN[i] < 0 || hOffset[i] < 0) return PERM_E_INVALID;
    if (hM[i] > 0 && hLd[i] < hN[i]) return PERM_E_INVALID;
    if (hM[i] > hN[i]) return PERM_E_UNSUPPORTED;
    if (hN[i] > BATCH_MAX_N) return PERM_E_TOO_LARGE;
    if (algo == PERM_ALGO_RYSER && hM[i] > 0 && hM[i] < hN[i]) return PERM_E_UNSUPPORTED;
  }
  const bool pad_ones = (flags & PERM_FLAG_PAD_ONES) != 0;
  const bool wrap = (flags & PERM_FLAG_WRAP) != 0;
  // Which walk serves matrix i: square floating-point Glynn (and rectangular
  // Glynn with rows of ones) on the per-order kernels below; everything else
  // staged: exact integers, Ryser, and the e_m form of rectangular matrices
  // (the padding rows summed out: the same sum as Eq. glynn_rectangle, without
  // its ill-conditioned padding).
  auto walk_of = [&](int i) -> int {
    const int m = hM[i], n = hN[i];
    if (m == 0) return kind == ENGINE_INT ? WALK_GLYNN : -1;
    if (algo == PERM_ALGO_RYSER) return WALK_RYSER;
    if (m < n) return (algo == PERM_ALGO_GLYNN && pad_ones) ? (kind == ENGINE_INT ? WALK_GLYNN : -1)
                                                             : WALK_ESYM;
    if (kind != ENGINE_INT) return -1;
    return algo == PERM_ALGO_GLYNN ? WALK_GLYNN : WALK_RYSER;
  };
  perm_batch_plan *p = new perm_batch_plan();
  if (hipGetDevice(&p->dev) != hipSuccess) {
    delete p;
    return PERM_E_HIP;
  }
  p->count = count;
  p->kind = kind;
  p->ot = ot;
  p->dt = dt;
  p->flags = flags;
  p->autotune = (flags & PERM_BATCH_AUTOTUNE) != 0;
  // descriptors and slots
  std::vector<BatchMatrix> mats(count);
  uint64_t slot = 0;
  std::vector<std::vector<uint32_t>> by_n(BATCH_MAX_N + 1);
  std::vector<WalkDesc> wdescs;
  std::vector<uint32_t> windex;
  uint64_t wslot = 0, arena = 0;
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  for (int i = 0; i < count; ++i) {
    BatchMatrix &d = mats[i];
    std::memset(&d, 0, sizeof d);
    d.offset = hOffset[i];
    d.ld = hLd[i];
    const int walk = walk_of(i);
    if (walk >= 0) {
      d.n = -1;  // served by a staged walk
      WalkDesc w;
      std::memset(&w, 0, sizeof w);
      w.offset = hOffset[i];
      w.ld = hLd[i];
      w.m = hM[i];
      w.n = hM[i] == 0 ? 0 : hN[i];
      w.walk = walk;
      w.nv = w.n == 0 ? 0 : (walk == WALK_RYSER ? w.m : w.n);
      w.nbits = w.n == 0 ? 0 : (walk == WALK_GLYNN ? w.n - 1 : (walk == WALK_RYSER ? w.n : w.m - 1));
      w.b = w.n == 0 ? 0 : batch_block_log2(w.nbits);
      // 0/1 input: every factor (a row or a signed column sum) is at most n
      w.pl = int_prod_selector(std::vector<uint64_t>(
          (size_t)std::max(1, walk == WALK_RYSER ? w.m : w.n), (uint64_t)std::max(1, w.n)));
      w.nonneg = walk == WALK_RYSER && dt == PERM_B8;
      w.nchunks = w.n == 0 ? 0 : (uint32_t)(((1ull << (w.nbits - w.b)) + 127) / 128);
      w.first_slot = (uint32_t)wslot;
      w.arena = arena;
      wslot += w.nchunks;
      if (w.n > 0) arena += (uint64_t)(2 * w.nbits + 1) * w.nv * C;
      if (kind == ENGINE_INT && w.n > 0) {
        if (dt != PERM_B8) {
          p->int_check = true;  // bounds need the data
        } else if (!wrap) {
          const double lim = ot == PERM_OUT_I64 ? 63.0 : 127.0;
          if (b8_log2_bound(walk, w.m, w.n, true) >= lim || b8_log2_bound(walk, w.m, w.n, false) >= 127.0)
            p->int_check = true;
        }
      }
      windex.push_back((uint32_t)i);
      wdescs.push_back(w);
      continue;
    }
    d.m = hM[i];
    d.n = hM[i] == 0 ? 0 : hN[i];  // an empty product (m = 0) has per = 1
    d.first_slot = (uint32_t)slot;
    if (d.n > 0) {
      const int nbits = d.n - 1;
      if (d.n <= pack_max_n() && pack_for(d.n, C) > 0) {
        d.b = 0;  // whole matrix in one wave's lane group: one slot
        d.nchunks = 1;
      } else {
        d.b = batch_block_log2(nbits);
        const uint64_t nblocks = 1ull << (nbits - d.b);
        d.nchunks = (uint32_t)((nblocks + 127) / 128);
      }
      slot += d.nchunks;
      by_n[d.n].push_back((uint32_t)i);
    }
  }
  if (slot >= (1ull << 32) || wslot >= (1ull << 32)) {
    delete p;
    return PERM_E_TOO_LARGE;
  }
  for (int i = 0; i < count && !pad_ones; ++i)
    if (mats[i].n > 0 && mats[i].m < mats[i].n) p->scale_pad = 1;
  // work items grouped by order, one bucket (one persistent kernel) per order
  std::vector<uint32_t> item_matrix, item_chunk;
  const int cus = device_cus();
  for (int n = BATCH_MAX_N; n >= 1; --n) {
    if (by_n[n].empty()) continue;
    BatchBucket bk;
    bk.n = n;
    bk.item_begin = (uint32_t)item_matrix.size();
    for (uint32_t i : by_n[n])
      for (uint32_t c = 0; c < mats[i].nchunks; ++c) {
        item_matrix.push_back(i);
        item_chunk.push_back(c);
      }
    bk.item_end = (uint32_t)item_matrix.size();
    const int pk = n <= pack_max_n() ? pack_for(n, kind == ENGINE_CPLX ? 2 : 1) : 0;
    if (pk > 0) {
      // one wave (workgroup) per `pk` matrices
      bk.pack = pk;
      bk.grid = (int)((bk.item_end - bk.item_begin + (uint32_t)pk - 1) / (uint32_t)pk);
    } else {
      const int bpc = std::max(1, batched_blocks_per_cu(kind, n));
      const uint64_t waves_needed = bk.item_end - bk.item_begin;
      const uint64_t groups = std::min<uint64_t>((uint64_t)cus * bpc, (waves_needed + 3) / 4);
      bk.grid = (int)std::max<uint64_t>(1, groups);
    }
    p->buckets.push_back(bk);
  }
  // staged walk items, one bucket per (term kind, order)
  std::vector<uint32_t> witem_desc, witem_chunk;
  for (int esym = 0; esym <= 1; ++esym)
    for (int nv = BATCH_MAX_N; nv >= 1; --nv) {
      WalkBucket wb;
      wb.nv = nv;
      wb.esym = esym;
      wb.item_begin = (uint32_t)witem_desc.size();
      for (size_t k = 0; k < wdescs.size(); ++k) {
        const WalkDesc &w = wdescs[k];
        if (w.n == 0 || w.nv != nv || (w.walk == WALK_ESYM) != (esym == 1)) continue;
        for (uint32_t c = 0; c < w.nchunks; ++c) {
          witem_desc.push_back((uint32_t)k);
          witem_chunk.push_back(c);
        }
      }
      wb.item_end = (uint32_t)witem_desc.size();
      if (wb.item_end == wb.item_begin) continue;
      const int bpc = std::max(1, walk_blocks_per_cu(kind, esym, nv));
      const uint64_t waves = wb.item_end - wb.item_begin;
      wb.grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)cus * bpc, (waves + 3) / 4));
      p->wbuckets.push_back(wb);
    }
  p->wcount = (int)wdescs.size();
  if (p->wcount > 0) {
    if ((rc = upload(&p->d_wdescs, wdescs)) || (rc = upload(&p->d_windex, windex)) ||
        (rc = upload(&p->d_witem_desc, witem_desc)) || (rc = upload(&p->d_witem_chunk, witem_chunk))) {
      release(p);
      return rc;
    }
    if (hipMalloc((void **)&p->d_arena, sizeof(double) * std::max<uint64_t>(1, arena)) != hipSuccess ||
        hipMalloc((void **)&p->d_wslots, sizeof(double) * 4 * std::max<uint64_t>(1, wslot)) != hipSuccess ||
        hipMalloc((void **)&p->d_wflags, sizeof(int) * (size_t)p->wcount) != hipSuccess) {
      release(p);
      return PERM_E_HIP;
    }
  }
  // padding rows: row e + PAD_EXP_MAX holds 2^e (complex: (2^e, 0))
  const int Cp = kind == ENGINE_CPLX ? 2 : 1;
  std::vector<double> pad_rows((size_t)(2 * PAD_EXP_MAX + 1) * BATCH_MAX_N * Cp, 0.0);
  for (int e = -PAD_EXP_MAX; e <= PAD_EXP_MAX; ++e)
    for (int j = 0; j < BATCH_MAX_N; ++j)
      pad_rows[((size_t)(e + PAD_EXP_MAX) * BATCH_MAX_N + j) * Cp] = std::ldexp(1.0, e);
  if ((rc = upload(&p->d_mats, mats)) || (rc = upload(&p->d_item_matrix, item_matrix)) ||
      (rc = upload(&p->d_item_chunk, item_chunk)) || (rc = upload(&p->d_pad_rows, pad_rows))) {
    release(p);
    return rc;
  }
  if (hipMalloc((void **)&p->d_slots, sizeof(double) * 2 * (size_t)C * std::max<uint64_t>(1, slot)) !=
          hipSuccess ||
      hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    release(p);
    return PERM_E_HIP;
  }
  *plan = p;
  return PERM_OK;
}

int perm_batch_plan_run(perm_batch_plan *p, const void *dData, void *dOut, void *stream) {
  if (!p || (p->count > 0 && (!dData || !dOut))) return PERM_E_INVALID;
  if (p->count == 0) return PERM_OK;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->dev) return PERM_E_INVALID;
  if (p->autotune && !p->tuned) {
    const int rc = autotune_packing(p, dData, dOut, s);
    if (rc) return rc;
    p->tuned = true;
  }
  const int prc = batch_int_precheck(p, dData, s);
  if (prc) return prc;
  if (!p->exec || p->g_data != dData || p->g_out != dOut) {
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    // capture on the plan's own stream, so that any caller stream (including
    // the default one) can launch the graph
    const BatchLaunch L = full_launch(p, dData, dOut);
    if (hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return PERM_E_HIP;
    hipError_t e = launch_batched(L, p->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->capture_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return PERM_E_HIP;
    }
    if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      hipGraphDestroy(g);
      return PERM_E_HIP;
    }
    p->graph = g;
    p->g_data = dData;
    p->g_out = dOut;
  }
  return hipGraphLaunch(p->exec, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
}

int perm_batch_plan_packing(const perm_batch_plan *p, int n) {
  if (!p || n < 1 || n > BATCH_MAX_N) return 0;
  for (const BatchBucket &bk : p->buckets)
    if (bk.n == n) return bk.pack;
  return 0;
}

int perm_batch_plan_destroy(perm_batch_plan *p) {
  release(p);
  return PERM_OK;
}

}  // extern "C"

namespace {

// One-shot batch: create a plan, run its launch sequence without graph
// capture, wait for the stream, destroy the plan.
int batched_once(perm_algo algo, int count, const int32_t *hM, const int32_t *hN,
                 const int64_t *hOffset, const int64_t *hLd, perm_dtype dt, const void *dData,
                 perm_out ot, void *dOut, uint32_t flags, void *stream) {
  if (count > 0 && (!dOut || !dData)) return PERM_E_INVALID;
  perm_batch_plan *p = nullptr;
  int rc = perm_batch_plan_create(count, hM, hN, hOffset, hLd, dt, ot, algo,
                                  flags & ~PERM_BATCH_AUTOTUNE, &p);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (count == 0) {
    release(p);
    return PERM_OK;
  }
  rc = batch_int_precheck(p, dData, s);
  if (rc) {
    (void)hipStreamSynchronize(s);
    release(p);
    return rc;
  }
  hipError_t e = launch_batched(full_launch(p, dData, dOut), s);
  // the plan's buffers are released only after the work using them is done
  hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  release(p);
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

}  // namespace

extern "C" {

int perm_glynn_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                       const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                       void *dOut, uint32_t flags, void *stream) {
  return batched_once(PERM_ALGO_GLYNN, count, hM, hN, hOffset, hLd, dt, dData, ot, dOut, flags,
                      stream);
}

int perm_ryser_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                       const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                       void *dOut, uint32_t flags, void *stream) {
  return batched_once(PERM_ALGO_RYSER, count, hM, hN, hOffset, hLd, dt, dData, ot, dOut, flags,
                      stream);
}

int perm_auto_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                      const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                      void *dOut, uint32_t flags, void *stream) {
  return batched_once(PERM_ALGO_AUTO, count, hM, hN, hOffset, hLd, dt, dData, ot, dOut, flags,
                      stream);
}

}  // extern "C"
