// C ABI of the library: argument checks, the planner, workspace layout,
// stage sequencing on the caller's stream and per-stage timing.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "index.h"
#include "kernels.h"
#include "rmq.h"

using namespace rmq;

struct rmq_timer_s {
  rmq::StageClock clock[RMQ_NUM_STAGES];
  bool ran[RMQ_NUM_STAGES];
  bool armed;
};

thread_local rmq::StageClock* rmq::tl_clock = nullptr;


namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

rmq_status from_hip(hipError_t e) {
  if (e == hipSuccess) return RMQ_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return RMQ_ERR_OUT_OF_MEMORY;
  return RMQ_ERR_DEVICE;
}

int ilog2_i64(int64_t x) {
  int j = 0;
  while ((x >> (j + 1)) != 0) ++j;
  return j;
}

bool is_pow2_block(int64_t k) {
  return k >= RMQ_MIN_BLOCK && k <= RMQ_MAX_BLOCK && (k & (k - 1)) == 0;
}

bool aligned_to(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int64_t num_blocks(int64_t m, int64_t k) { return (m + k - 1) / k; }

// Default block sizes.  FULL: about sqrt(n) / 8, clamped to [256, 65536] --
// the ST over blocks stays small (a few MB at n = 1e8) while partial scans
// remain rare (Section 3.2 balances k against (n/k) log(n/k)).  CONTRACTED:
// the paper's default of 512 entries of A_Q.
int32_t default_block_full(int64_t n) {
  double t = sqrt((double)n) / 8.0;
  int64_t k = 256;
  while (k < 65536 && (double)(k * 2) <= t) k *= 2;
  return (int32_t)k;
}
// CONTRACTED: the average query cost is O(1 + k^2/q) (Section 3.1, step 4
// analysis), so k ~ sqrt(q); A_Q has 2q - 1 entries and partial scans read k
// of them.  A power of two near sqrt(2q) / 2, clamped to [16, 4096].
int32_t default_block_contracted(int64_t q) {
  const double t = sqrt(2.0 * (double)q) / 2.0;
  int64_t k = 16;
  while (k < 4096 && (double)(k * 2) <= t) k *= 2;
  return (int32_t)k;
}

struct Plan {
  int path;
  int32_t k;
  int kshift;
  int k1shift;  // two block levels (Section 3.3): k1 = 2^k1shift; -1 = one level
  int lg;       // table over powers of l = 2^lg (Section 3.1); 1 = doubling
  bool records;  // query records allowed (opt->no_query_records == 0)
  int k2shift = -1;  // three block levels (plain method): k2 = 2^k2shift; -1 = none
};

// Query records (see launch_records) for a doubling table of nb blocks and
// `levels` levels: whether they are built (not for another arity, not under
// two block levels, nor above kMaxRecordBytes), and their bytes.  Measured
// at n = 1e8 on the planner's two-level plans, whole jobs were faster
// without them (q = 1e5: 0.083 vs 0.086 ms, q = 1e7: 0.162 vs 0.170 ms).
constexpr size_t kMaxRecordBytes = 8u << 20;  // measured: larger records lose to L2 misses
size_t records_bytes(int64_t nb, int levels) { return sizeof(uint64_t) * 4 * (size_t)nb * levels; }
bool records_built(int64_t nb, int levels, int lg, bool allowed, bool two_level) {
  return allowed && !two_level && lg <= 1 && records_bytes(nb, levels) <= kMaxRecordBytes;
}

// opt->table_arity_log2 as lg (0 and 1 both mean doubling); -1 if invalid.
int arity_lg(const rmq_options* opt) {
  const int32_t a = opt ? opt->table_arity_log2 : 0;
  if (a < 0 || a > 5) return -1;
  return a < 1 ? 1 : a;
}

int32_t table_levels(int64_t nb, int lg) { return lary_levels(nb, lg); }

// Section 3.3's choice for two levels: k2 = sqrt(n) log^(2/3) n, as a power
// of two, at least 2 * k1.
int32_t default_block_two_level(int64_t n, int32_t k1) {
  const double ln = log2((double)(n > 2 ? n : 2));
  const double t = sqrt((double)n) * pow(ln, 2.0 / 3.0);
  int64_t k = 2 * (int64_t)k1;
  while (k < RMQ_MAX_BLOCK && (double)(k * 2) <= t * 1.41421356) k *= 2;
  return (int32_t)k;
}

// The contracted method's default is one block level over A_Q below
// q = 2^22 queries.  From there it takes two levels, k1 = 256 under blocks
// of at least 16384 entries, as few as keep the block table within the LDS
// of the query kernel that copies it (see launch_query_contracted).
// Measured at n = 1e8, q = 1e7, whole jobs: uniform queries 0.839 ms (one
// level, k = 2048, gathered table and query records) -> 0.760 ms
// ((16384, 256), table in LDS); (16384, 512) 0.759, (32768, 512) 0.783,
// (8192, 256) 0.806 (table too large for LDS).  A mix with half the ranges of
// at most 1024 elements loses: 1.610 -> 1.730 ms (short ranges are a few
// entries of A_Q whose block minimum rarely lies inside them, so they are
// scanned through the k1-block minima); callers with such mixes can pass
// block_size and sub_block_size.  (Earlier, with the gathered table: k1 = 512
// under k = 8 times the one-level size gained 1.142 -> 1.114 ms at q = 1e7
// and lost on the skewed mix at n = 1e9, 3.25 -> 3.58 ms.)
constexpr int64_t CONTRACTED_TWO_LEVEL_Q = 1 << 22;
int32_t default_sub_block_contracted(int64_t q) { return q >= CONTRACTED_TWO_LEVEL_Q ? 256 : 0; }
int32_t default_block_two_level_contracted(int64_t q) {
  const int64_t m = 2 * q;  // entries of A_Q, at most
  int64_t k = 16384;
  for (;;) {
    const int64_t nb = (m + k - 1) / k;
    int levels = 1;
    if (nb > 3) {
      levels = 0;
      for (int64_t x = nb - 2; x; x >>= 1) ++levels;
    }
    if (nb * levels * 8 <= 144 * 1024 || k >= RMQ_MAX_BLOCK) return (int32_t)k;
    k *= 2;
  }
}

// Batched items: blocks per array, the largest one-level block, and the k1
// given above it.
constexpr int64_t BATCH_MAX_BLOCKS = 1024;
constexpr int64_t BATCH_ONE_LEVEL_MAX_K = 4096;
constexpr int64_t BATCH_SUB_BLOCK = 1024;

// ST-RMQ_CON (Section 2) takes at most 2^29 queries: its doubled endpoint
// list (4q entries) must index in 32 bits.
constexpr int64_t ST_CON_MAX_Q = 1ll << 29;

// single_call: the caller is rmq_query_batch_ex / rmq_workspace_bytes, which
// alone take the comparison system ST-RMQ_CON and three block levels.
rmq_status make_plan(int64_t n, int64_t q, const rmq_options* opt, Plan* p,
                     bool allow_two_level = true, bool single_call = false) {
  int32_t path = opt ? opt->path : RMQ_PATH_AUTO;
  int32_t k = opt ? opt->block_size : 0;
  int32_t k1 = opt ? opt->sub_block_size : 0;
  const int32_t k2 = opt ? opt->sub_block_size2 : 0;
  p->k2shift = -1;
  if (k2 != 0) {
    // three block levels (Section 3.3): the plain method, under a given k1
    if (!single_call || k1 == 0 || !is_pow2_block(k2) || k2 >= k1 ||
        (path != RMQ_PATH_AUTO && path != RMQ_PATH_FULL))
      return RMQ_ERR_INVALID_ARG;
    path = RMQ_PATH_FULL;
    p->k2shift = ilog2_i64(k2);
  }
  if (path == RMQ_PATH_ST_CON) {
    // the comparison system: no blocks, one element table (doubling)
    if (!single_call || k != 0 || k1 != 0 || arity_lg(opt) != 1 || q > ST_CON_MAX_Q)
      return RMQ_ERR_INVALID_ARG;
    p->path = RMQ_PATH_ST_CON;
    p->k = 1;
    p->kshift = 0;
    p->k1shift = -1;
    p->lg = 1;
    p->records = false;
    return RMQ_OK;
  }
  if (path == RMQ_PATH_CONTRACTED && k == 0 && k1 == 0 && allow_two_level)
    k1 = default_sub_block_contracted(q);
  if (path != RMQ_PATH_AUTO && path != RMQ_PATH_FULL && path != RMQ_PATH_CONTRACTED)
    return RMQ_ERR_INVALID_ARG;
  if (k != 0 && !is_pow2_block(k)) return RMQ_ERR_INVALID_ARG;
  p->k1shift = -1;
  p->lg = arity_lg(opt);
  if (p->lg < 0) return RMQ_ERR_INVALID_ARG;
  p->records = !(opt && opt->no_query_records);
  if (k1 != 0) {
    // two block levels (k1 < k): over A, or over A_Q for the contracted method
    if (!is_pow2_block(k1)) return RMQ_ERR_INVALID_ARG;
    const bool con = path == RMQ_PATH_CONTRACTED;
    if (k == 0)
      k = con && k1 == default_sub_block_contracted(q) ? default_block_two_level_contracted(q)
                                                       : default_block_two_level(con ? 2 * q : n, k1);
    if (k1 >= k) return RMQ_ERR_INVALID_ARG;
    p->path = con ? RMQ_PATH_CONTRACTED : RMQ_PATH_FULL;
    p->k = k;
    p->kshift = ilog2_i64(k);
    p->k1shift = ilog2_i64(k1);
    return RMQ_OK;
  }
  if (path == RMQ_PATH_AUTO) {
    int32_t pk = 0, pp = 0, pk1 = 0;
    if (k == 0 && allow_two_level) {
      rmq_plan_ex(n, q, &pk, &pp, &pk1);
      if (pk1 > 0 && pp == RMQ_PATH_FULL && pk1 < pk) {  // two block levels (Section 3.3)
        p->path = RMQ_PATH_FULL;
        p->k = pk;
        p->kshift = ilog2_i64(pk);
        p->k1shift = ilog2_i64(pk1);
        return RMQ_OK;
      }
    } else {
      rmq_plan(n, q, &pk, &pp);
    }
    path = pp;
    if (k == 0) k = pk;
  }
  if (k == 0) k = path == RMQ_PATH_FULL ? default_block_full(n) : default_block_contracted(q);
  p->path = path;
  p->k = k;
  p->kshift = ilog2_i64(k);
  return RMQ_OK;
}

// ---- workspace layouts ----
struct FullLayout {
  int64_t nb, nb1, nb2;
  int levels;
  bool rec;  // query records built
  size_t off_st, off_sub, off_sub2, off_rec, bytes;
};

// The table, then (two block levels) the k1-block minima, then (three) the
// k2-block minima.
FullLayout full_layout(int64_t n, int64_t k, int k1shift, int lg, bool records,
                       int k2shift = -1) {
  FullLayout f{};
  f.nb = num_blocks(n, k);
  f.levels = table_levels(f.nb, lg);
  f.rec = records_built(f.nb, f.levels, lg, records, k1shift >= 0);
  f.off_st = 0;
  f.off_sub = align_up(sizeof(uint64_t) * (size_t)f.nb * (size_t)f.levels);
  f.nb1 = k1shift >= 0 ? num_blocks(n, 1ll << k1shift) : 0;
  f.off_sub2 = f.off_sub + align_up(sizeof(uint64_t) * (size_t)f.nb1);
  f.nb2 = k1shift >= 0 && k2shift >= 0 ? num_blocks(n, 1ll << k2shift) : 0;
  f.off_rec = f.off_sub2 + (f.nb2 ? align_up(sizeof(uint64_t) * (size_t)f.nb2) : 0);
  f.bytes = f.off_rec + (f.rec ? align_up(records_bytes(f.nb, f.levels)) : 0);
  return f;
}

struct ConLayout {
  int64_t M, m, nb, nb1;
  int levels;
  bool rec;  // query records built
  size_t off_E, off_sort, off_lr, off_aq, off_tiles, off_st, off_sub, off_rec, bytes;
};

// k1shift >= 0: two block levels over A_Q (Section 3.3), the k1-block
// minima kept beside the table.
ConLayout con_layout(int64_t n, int64_t q, int64_t k, int k1shift, int lg, bool records) {
  ConLayout c{};
  c.M = 2 * q;
  c.m = c.M - 1;
  c.nb = num_blocks(c.m, k);
  c.nb1 = k1shift >= 0 ? num_blocks(c.m, 1ll << k1shift) : 0;
  c.levels = table_levels(c.nb, lg);
  c.rec = records_built(c.nb, c.levels, lg, records, k1shift >= 0);
  size_t o = 0;
  c.off_E = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.M);
  c.off_sort = o;
  o = align_up(o + sort_workspace_bytes(q));
  c.off_lr = o;
  o = align_up(o + sizeof(int32_t) * (size_t)c.M);
  c.off_aq = o;  // before the contraction also the remap's pair scratch (2q items)
  o = align_up(o + sizeof(uint64_t) * (size_t)c.M);
  c.off_tiles = o;
  o = align_up(o + contract_tile_start_bytes(n));
  c.off_st = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.nb * (size_t)c.levels);
  c.off_sub = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.nb1);
  c.off_rec = o;
  o = align_up(o + (c.rec ? records_bytes(c.nb, c.levels) : 0));
  c.bytes = o;
  return c;
}

// ST-RMQ_CON: the sorted endpoints (as for the contracted method), their
// remap, the doubled list, the contraction's tile table and the element
// table, whose level 0 is A_Q itself (and, before the contraction, the
// remap's pair scratch: 2q items in 4q - 1 keys).
struct StConLayout {
  int64_t M, m;
  int levels;
  size_t off_E, off_sort, off_lr, off_E2, off_tiles, off_st, bytes;
};

StConLayout st_con_layout(int64_t n, int64_t q) {
  StConLayout c{};
  c.M = 2 * q;
  c.m = 2 * c.M - 1;
  c.levels = ilog2_i64(c.m) + 1;  // windows of every length up to m
  size_t o = 0;
  c.off_E = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.M);
  c.off_sort = o;
  o = align_up(o + sort_workspace_bytes(q));
  c.off_lr = o;
  o = align_up(o + sizeof(int32_t) * (size_t)c.M);
  c.off_E2 = o;
  o = align_up(o + sizeof(int32_t) * 2 * (size_t)c.M);
  c.off_tiles = o;
  o = align_up(o + contract_tile_start_bytes(n));
  c.off_st = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.m * (size_t)c.levels);
  c.bytes = o;
  return c;
}

size_t plan_bytes(int64_t n, int64_t q, const Plan& p) {
  if (p.path == RMQ_PATH_ST_CON) return st_con_layout(n, q).bytes;
  if (p.path == RMQ_PATH_FULL)
    return full_layout(n, p.k, p.k1shift, p.lg, p.records, p.k2shift).bytes;
  return con_layout(n, q, p.k, p.k1shift, p.lg, p.records).bytes;
}

std::once_flag g_pool_once[64];

std::mutex g_table_mu;
std::vector<rmq_plan_entry> g_table;  // measured plans, see rmq_planner_set_table

// The measured entry nearest to (n, q) in (log2 n, log2 q); the caller holds
// g_table_mu and has checked that the table is not empty.
const rmq_plan_entry& nearest_entry(int64_t n, int64_t q) {
  const double ln = log2((double)n), lq = log2((double)(q > 0 ? q : 1));
  const rmq_plan_entry* best = &g_table[0];
  double bd = -1;
  for (const rmq_plan_entry& e : g_table) {
    const double dn = log2((double)e.n) - ln, dq = log2((double)e.q) - lq;
    const double d = dn * dn + dq * dq;
    if (bd < 0 || d < bd) {
      best = &e;
      bd = d;
    }
  }
  return *best;
}

// Keep freed stream-ordered memory cached in the device pool, so that
// per-call scratch costs no device allocation after the first call.  Returns
// the device, or -1.
int prepare_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  std::call_once(g_pool_once[dev], [dev] {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
  return dev;
}

// Size of the per-call scratch taken from the pool: the largest any call on
// the device has needed so far, so that jobs of different sizes all ask for
// the same block.  With each job's exact size, a sweep alternating small and
// large jobs (both methods over q = 1e3 .. 1e7 at n = 1e8) took 3.42 instead
// of 2.72 ms per 10 jobs.
std::atomic<size_t> g_scratch_size[64];
size_t pool_request(int dev, size_t need) {
  if (dev < 0) return need;
  size_t cur = g_scratch_size[dev].load(std::memory_order_relaxed);
  while (cur < need &&
         !g_scratch_size[dev].compare_exchange_weak(cur, need, std::memory_order_relaxed)) {
  }
  return cur > need ? cur : need;
}

// Stage i of a timed call: kernels launched until stage_end carry the
// stage's start/stop events.  A stage that launched nothing gets two plain
// event records (zero length).
void stage_begin(rmq_timer* t, int i) {
  if (!t) return;
  t->clock[i].started = false;
  tl_clock = &t->clock[i];
}
void stage_end(rmq_timer* t, int i, hipStream_t s) {
  if (!t) return;
  tl_clock = nullptr;
  if (!t->clock[i].started) {
    hipEventRecord(t->clock[i].start, s);
    hipEventRecord(t->clock[i].stop, s);
  }
  t->ran[i] = true;
  t->armed = true;
}
struct ClockGuard {  // never leave a stage clock armed on an early return
  ~ClockGuard() { tl_clock = nullptr; }
};

bool check_query_ptrs(const int32_t* L, const int32_t* R, int32_t* out, int64_t q) {
  if (q == 0) return true;
  return L && R && out;
}

// Section 3.1's table over the block minima at st[0 .. nb): doubling, or
// powers of l = 2^lg.
hipError_t build_table(uint64_t* st, int64_t nb, int levels, int lg, hipStream_t s) {
  return lg > 1 ? launch_sparse_table_lary(st, nb, lg, s) : launch_sparse_table(st, nb, levels, s);
}

rmq_status run_full(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R, int64_t q,
                    int32_t* out, hipStream_t s, const rmq_options* opt, const Plan& p,
                    char* ws) {
  rmq_timer* t = opt ? opt->timer : nullptr;
  ClockGuard guard;
  if (t) t->ran[0] = false;  // no sort stage on this path
  const FullLayout f = full_layout(n, p.k, p.k1shift, p.lg, p.records, p.k2shift);
  uint64_t* st = reinterpret_cast<uint64_t*>(ws + f.off_st);
  uint64_t* sub = reinterpret_cast<uint64_t*>(ws + f.off_sub);
  uint64_t* sub2 = reinterpret_cast<uint64_t*>(ws + f.off_sub2);
  uint64_t* rec = f.rec ? reinterpret_cast<uint64_t*>(ws + f.off_rec) : nullptr;
  const bool two = p.k1shift >= 0;
  const bool three = two && p.k2shift >= 0;
  // stage 1 is the one pass over A; with two levels (Section 3.3) it takes
  // the k1-block minima (with three, the k2-block minima, and the k1-block
  // minima from those), and the k-block minima are taken from the k1-block
  // minima in stage 2 with the table
  stage_begin(t, 1);
  hipError_t e = three ? launch_blockmin_i32(A, n, p.k2shift, sub2, s)
                 : two ? launch_blockmin_i32(A, n, p.k1shift, sub, s)
                       : launch_blockmin_i32(A, n, p.kshift, st, s);
  if (e == hipSuccess && three)
    e = launch_blockmin_keys(sub2, f.nb2, p.k1shift - p.k2shift, sub, s);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 1, s);
  stage_begin(t, 2);
  if (two) e = launch_blockmin_keys(sub, f.nb1, p.kshift - p.k1shift, st, s);
  if (e == hipSuccess) e = build_table(st, f.nb, f.levels, p.lg, s);
  if (e == hipSuccess && rec) e = launch_records(st, f.nb, f.levels, rec, s);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 2, s);
  stage_begin(t, 3);
  int64_t* bad = opt ? opt->bad_count : nullptr;
  uint64_t* stats = opt ? opt->stats : nullptr;
  e = three ? launch_query_full3(A, n, p.kshift, st, f.nb, sub, p.k1shift, sub2, p.k2shift, L, R,
                                 q, out, bad, stats, s, p.lg)
      : two ? launch_query_full2(A, n, p.kshift, st, f.nb, sub, p.k1shift, L, R, q, out, bad,
                                 stats, s, p.lg, rec, f.levels)
            : launch_query_full(A, n, p.kshift, st, f.nb, L, R, q, out, bad, stats, s, p.lg, rec,
                                f.levels);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 3, s);
  return RMQ_OK;
}

rmq_status run_contracted(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R,
                          int64_t q, int32_t* out, hipStream_t s, const rmq_options* opt,
                          const Plan& p, char* ws) {
  rmq_timer* t = opt ? opt->timer : nullptr;
  const ConLayout c = con_layout(n, q, p.k, p.k1shift, p.lg, p.records);
  uint64_t* E = reinterpret_cast<uint64_t*>(ws + c.off_E);
  uint64_t* rec = c.rec ? reinterpret_cast<uint64_t*>(ws + c.off_rec) : nullptr;
  int32_t* LR = reinterpret_cast<int32_t*>(ws + c.off_lr);
  uint64_t* aq = reinterpret_cast<uint64_t*>(ws + c.off_aq);
  int32_t* tiles = reinterpret_cast<int32_t*>(ws + c.off_tiles);
  uint64_t* st = reinterpret_cast<uint64_t*>(ws + c.off_st);
  const bool two = p.k1shift >= 0;
  uint64_t* sub = two ? reinterpret_cast<uint64_t*>(ws + c.off_sub) : nullptr;
  ClockGuard guard;
  stage_begin(t, 0);
  // the sort's last pass writes the remap as well
  hipError_t e =
      launch_sort_endpoints(L, R, q, n, E, LR, aq, ws + c.off_sort, sort_workspace_bytes(q), s);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 0, s);
  stage_begin(t, 1);
  // the sort left the positions only (int32) in the first half of E
  // (nothing is contracted after a sort that gave up; the queries then
  // report every query as invalid)
  e = launch_contract(A, n, reinterpret_cast<const int32_t*>(E), q, aq, tiles, s,
                      sort_abort_word(ws + c.off_sort, q));
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 1, s);
  stage_begin(t, 2);
  if (two) {
    e = launch_blockmin_keys(aq, c.m, p.k1shift, sub, s);
    if (e == hipSuccess) e = launch_blockmin_keys(sub, c.nb1, p.kshift - p.k1shift, st, s);
  } else {
    e = launch_blockmin_keys(aq, c.m, p.kshift, st, s);
  }
  if (e != hipSuccess) return from_hip(e);
  e = build_table(st, c.nb, c.levels, p.lg, s);
  if (e == hipSuccess && rec) e = launch_records(st, c.nb, c.levels, rec, s);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 2, s);
  stage_begin(t, 3);
  // a sort that gave up on its order (bounded look-back wait exceeded) makes
  // the query kernel answer -1 for every query and count them all as invalid
  e = launch_query_contracted(aq, c.m, n, p.kshift, st, c.nb, L, R, LR, q, out,
                              opt ? opt->bad_count : nullptr, opt ? opt->stats : nullptr, s,
                              p.lg, rec, c.levels, sub, p.k1shift,
                              sort_abort_word(ws + c.off_sort, q));
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 3, s);
  return RMQ_OK;
}

// ST-RMQ_CON (Section 2), re-created with this library's parts: the sort
// and remap of the endpoints, the contraction over the doubled list (its
// A_Q of 4q - 1 entries), the Sparse Table over every entry, two reads per
// query.  Stages as for the contracted method.
rmq_status run_st_con(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R, int64_t q,
                      int32_t* out, hipStream_t s, const rmq_options* opt, char* ws) {
  rmq_timer* t = opt ? opt->timer : nullptr;
  const StConLayout c = st_con_layout(n, q);
  uint64_t* E = reinterpret_cast<uint64_t*>(ws + c.off_E);
  int32_t* LR = reinterpret_cast<int32_t*>(ws + c.off_lr);
  int32_t* E2 = reinterpret_cast<int32_t*>(ws + c.off_E2);
  int32_t* tiles = reinterpret_cast<int32_t*>(ws + c.off_tiles);
  uint64_t* st = reinterpret_cast<uint64_t*>(ws + c.off_st);
  const uint32_t* fail = sort_abort_word(ws + c.off_sort, q);
  ClockGuard guard;
  stage_begin(t, 0);
  hipError_t e =
      launch_sort_endpoints(L, R, q, n, E, LR, st, ws + c.off_sort, sort_workspace_bytes(q), s);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 0, s);
  stage_begin(t, 1);
  e = launch_double_ends(reinterpret_cast<const int32_t*>(E), c.M, E2, s);
  if (e == hipSuccess) e = launch_contract(A, n, E2, c.M, st, tiles, s, fail);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 1, s);
  stage_begin(t, 2);
  e = launch_sparse_table(st, c.m, c.levels, s);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 2, s);
  stage_begin(t, 3);
  e = launch_query_st_elements(st, c.m, c.levels, L, R, LR, q, n, out,
                               opt ? opt->bad_count : nullptr, s, fail);
  if (e != hipSuccess) return from_hip(e);
  stage_end(t, 3, s);
  return RMQ_OK;
}

}  // namespace

extern "C" {

const char* rmq_status_string(rmq_status s) {
  switch (s) {
    case RMQ_OK: return "ok";
    case RMQ_ERR_INVALID_ARG: return "invalid argument";
    case RMQ_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RMQ_ERR_DEVICE: return "HIP runtime error";
    case RMQ_ERR_WORKSPACE_SMALL: return "workspace too small";
    case RMQ_ERR_MISALIGNED: return "misaligned device pointer";
    case RMQ_ERR_SCRATCH_LIMIT: return "needs more than the fixed scratch array";
  }
  return "unknown status";
}

const char* rmq_version(void) { return "rmq-gfx950 1.1"; }

int32_t rmq_table_levels(int64_t nb) {
  if (nb <= 3) return 1;
  return ilog2_i64(nb - 2) + 1;
}

size_t rmq_query_record_bytes(int64_t nb) {
  if (nb < 1 || nb > RMQ_MAX_N) return 0;
  const int lv = rmq_table_levels(nb);
  return records_built(nb, lv, 1, true, false) ? records_bytes(nb, lv) : 0;
}

int32_t rmq_table_levels_ary(int64_t nb, int32_t table_arity_log2) {
  if (nb < 1 || table_arity_log2 < 0 || table_arity_log2 > 5) return 0;
  return table_levels(nb, table_arity_log2 < 1 ? 1 : table_arity_log2);
}

size_t rmq_index_bytes(int64_t n, int32_t k) {
  if (n < 1 || n > RMQ_MAX_N || !is_pow2_block(k)) return 0;
  const int64_t nb = num_blocks(n, k);
  return sizeof(uint64_t) * (size_t)nb * (size_t)rmq_table_levels(nb);
}

rmq_status rmq_planner_set_table(const rmq_plan_entry* entries, int32_t count) {
  if (count < 0 || (count > 0 && !entries)) return RMQ_ERR_INVALID_ARG;
  for (int32_t i = 0; i < count; ++i) {
    const rmq_plan_entry& e = entries[i];
    if (e.n < 1 || e.q < 1 || !is_pow2_block(e.block_size) ||
        (e.path != RMQ_PATH_FULL && e.path != RMQ_PATH_CONTRACTED))
      return RMQ_ERR_INVALID_ARG;
    if (e.sub_block_size != 0 && (e.path != RMQ_PATH_FULL || !is_pow2_block(e.sub_block_size) ||
                                  e.sub_block_size >= e.block_size))
      return RMQ_ERR_INVALID_ARG;
    if (e.one_level_block_size != 0 && !is_pow2_block(e.one_level_block_size))
      return RMQ_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_table_mu);
  g_table.assign(entries, entries + count);
  return RMQ_OK;
}

rmq_status rmq_plan_ex(int64_t n, int64_t q, int32_t* block_size, int32_t* path,
                       int32_t* sub_block_size) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return RMQ_ERR_INVALID_ARG;
  if (sub_block_size) *sub_block_size = 0;
  {
    // measured table: the entry nearest in (log2 n, log2 q)
    std::lock_guard<std::mutex> lock(g_table_mu);
    if (!g_table.empty()) {
      const rmq_plan_entry* best = &nearest_entry(n, q);
      // a two-level plan needs k1 < k <= the array (else one level)
      const bool two = best->sub_block_size > 0 && best->block_size <= n;
      if (block_size)
        *block_size = two || best->one_level_block_size == 0 ? best->block_size
                                                             : best->one_level_block_size;
      if (path) *path = best->path;
      if (sub_block_size && two) *sub_block_size = best->sub_block_size;
      return RMQ_OK;
    }
  }
  // Both methods stream A once (the contracted one between its outermost
  // endpoints, which for queries spread over A is all of it); the contracted
  // one adds a sort of 2q endpoints and a pass over A_Q, so the plain one is
  // the cheaper choice for every batch whose endpoints span A.
  if (block_size) *block_size = default_block_full(n);
  if (path) *path = RMQ_PATH_FULL;
  return RMQ_OK;
}

rmq_status rmq_plan(int64_t n, int64_t q, int32_t* block_size, int32_t* path) {
  int32_t k = 0, p = 0, k1 = 0;
  const rmq_status st = rmq_plan_ex(n, q, &k, &p, &k1);
  if (st != RMQ_OK) return st;
  if (k1 > 0) {
    // the one-level choice of the same entry
    std::lock_guard<std::mutex> lock(g_table_mu);
    const rmq_plan_entry& best = nearest_entry(n, q);
    k = best.one_level_block_size ? best.one_level_block_size : best.block_size;
  }
  if (block_size) *block_size = k;
  if (path) *path = p;
  return RMQ_OK;
}

int32_t rmq_default_sub_block(int64_t n, int64_t q, int32_t path) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return 0;
  return path == RMQ_PATH_CONTRACTED ? default_sub_block_contracted(q) : 0;
}

int32_t rmq_default_block(int64_t n, int64_t q, int32_t path) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return 0;
  if (path == RMQ_PATH_FULL) return default_block_full(n);
  if (path == RMQ_PATH_CONTRACTED) {
    const int32_t k1 = default_sub_block_contracted(q);
    return k1 ? default_block_two_level_contracted(q) : default_block_contracted(q);
  }
  return 0;
}

size_t rmq_workspace_bytes(int64_t n, int64_t q, const rmq_options* opt) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return 0;
  if (q == 0) return 0;
  Plan p;
  if (make_plan(n, q, opt, &p, true, true) != RMQ_OK) return 0;
  return plan_bytes(n, q, p);
}

rmq_status rmq_query_batch_ex(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R,
                              int64_t q, int32_t* out, void* stream, const rmq_options* opt) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q || !A) return RMQ_ERR_INVALID_ARG;
  if (!check_query_ptrs(L, R, out, q)) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(A, 4) || (q && (!aligned_to(L, 4) || !aligned_to(R, 4) || !aligned_to(out, 4))))
    return RMQ_ERR_MISALIGNED;
  if (opt && opt->workspace && !aligned_to(opt->workspace, ALIGN)) return RMQ_ERR_MISALIGNED;
  Plan p;
  rmq_status st = make_plan(n, q, opt, &p, true, true);
  if (st != RMQ_OK) return st;
  if (q == 0) return RMQ_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = plan_bytes(n, q, p);
  char* ws = nullptr;
  bool own = false;
  if (opt && opt->workspace) {
    if (opt->workspace_bytes < need) return RMQ_ERR_WORKSPACE_SMALL;
    ws = static_cast<char*>(opt->workspace);
  } else {
    const int dev = prepare_pool();
    void* w = nullptr;
    hipError_t e = hipMallocAsync(&w, pool_request(dev, need), s);
    if (e != hipSuccess) return from_hip(e);
    ws = static_cast<char*>(w);
    own = true;
  }
  st = p.path == RMQ_PATH_FULL       ? run_full(A, n, L, R, q, out, s, opt, p, ws)
       : p.path == RMQ_PATH_ST_CON ? run_st_con(A, n, L, R, q, out, s, opt, ws)
                                   : run_contracted(A, n, L, R, q, out, s, opt, p, ws);
  if (own) hipFreeAsync(ws, s);
  return st;
}

rmq_status rmq_query_batch(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R,
                           int64_t q, int32_t* out, void* stream) {
  return rmq_query_batch_ex(A, n, L, R, q, out, stream, nullptr);
}

// ---- resident index ----
}  // extern "C"

namespace {

// Shape of a resident index for (n, opt): block sizes, levels, records and
// the device bytes rmq_build allocates for it.
struct IndexShape {
  int kshift, k1shift, lg, levels;
  int64_t nb, nb1;
  bool rec;
  size_t off_rec, bytes;
};

rmq_status index_shape(int64_t n, const rmq_options* opt, IndexShape* sh) {
  if (n < 1 || n > RMQ_MAX_N) return RMQ_ERR_INVALID_ARG;
  int32_t k = opt ? opt->block_size : 0;
  const int32_t k1 = opt ? opt->sub_block_size : 0;
  const int lg = arity_lg(opt);
  if (lg < 0 || (k1 != 0 && !is_pow2_block(k1))) return RMQ_ERR_INVALID_ARG;
  if (opt && opt->sub_block_size2 != 0) return RMQ_ERR_INVALID_ARG;  // single calls only
  if (k == 0 && k1 != 0) {
    k = default_block_two_level(n, k1);
  } else if (k == 0) {
    // Section 3.2: k = Theta(sqrt(n)) keeps both the query time and the
    // space of the index low; a power of two near sqrt(n) / 4.
    const double tgt = sqrt((double)n) / 4.0;
    k = 256;
    while (k < (1 << 20) && (double)(k * 2) <= tgt) k *= 2;
  }
  if (!is_pow2_block(k) || (k1 != 0 && k1 >= k)) return RMQ_ERR_INVALID_ARG;
  sh->kshift = ilog2_i64(k);
  sh->nb = num_blocks(n, k);
  sh->lg = lg;
  sh->levels = table_levels(sh->nb, lg);
  sh->k1shift = k1 != 0 ? ilog2_i64(k1) : -1;
  sh->nb1 = k1 != 0 ? num_blocks(n, k1) : 0;
  sh->rec = records_built(sh->nb, sh->levels, lg, !(opt && opt->no_query_records), k1 != 0);
  const size_t table_bytes = sizeof(uint64_t) * (size_t)sh->nb * (size_t)sh->levels;
  const size_t sub_bytes = sizeof(uint64_t) * (size_t)sh->nb1;
  // the records start on a 256-byte boundary, so that each is whole lines
  sh->off_rec = align_up(table_bytes + sub_bytes);
  sh->bytes = sh->rec ? sh->off_rec + records_bytes(sh->nb, sh->levels) : table_bytes + sub_bytes;
  return RMQ_OK;
}

}  // namespace

extern "C" {

size_t rmq_build_bytes(int64_t n, const rmq_options* opt) {
  IndexShape sh;
  return index_shape(n, opt, &sh) == RMQ_OK ? sh.bytes : 0;
}

rmq_status rmq_build(const int32_t* A, int64_t n, const rmq_options* opt, void* stream,
                     rmq_index* idx) {
  if (!A || !idx || n < 1 || n > RMQ_MAX_N) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(A, 4)) return RMQ_ERR_MISALIGNED;
  IndexShape sh;
  const rmq_status bad = index_shape(n, opt, &sh);
  if (bad != RMQ_OK) return bad;
  rmq_index_s* ix = static_cast<rmq_index_s*>(calloc(1, sizeof(rmq_index_s)));
  if (!ix) return RMQ_ERR_OUT_OF_MEMORY;
  hipGetDevice(&ix->device);
  ix->A = A;
  ix->n = n;
  ix->kshift = sh.kshift;
  ix->nb = sh.nb;
  ix->lg = sh.lg;
  ix->levels = sh.levels;
  ix->k1shift = sh.k1shift;
  ix->nb1 = sh.nb1;
  const bool with_rec = sh.rec;
  const size_t off_rec = sh.off_rec;
  ix->bytes = sh.bytes;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, ix->bytes);
  if (e != hipSuccess) {
    free(ix);
    return from_hip(e);
  }
  ix->st = static_cast<uint64_t*>(mem);
  ix->sub = sh.k1shift >= 0 ? ix->st + (size_t)ix->nb * (size_t)ix->levels : nullptr;
  ix->rec = with_rec ? reinterpret_cast<uint64_t*>(static_cast<char*>(mem) + off_rec) : nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ix->sub) {
    // Section 3.3: k1-block minima, then the k-block minima from them
    e = launch_blockmin_i32(A, n, ix->k1shift, ix->sub, s);
    if (e == hipSuccess) e = launch_blockmin_keys(ix->sub, ix->nb1, ix->kshift - ix->k1shift,
                                                  ix->st, s);
  } else {
    e = launch_blockmin_i32(A, n, ix->kshift, ix->st, s);
  }
  if (e == hipSuccess) e = build_table(ix->st, ix->nb, ix->levels, ix->lg, s);
  if (e == hipSuccess && ix->rec) e = launch_records(ix->st, ix->nb, ix->levels, ix->rec, s);
  if (e != hipSuccess) {
    hipFree(mem);
    free(ix);
    return from_hip(e);
  }
  *idx = ix;
  return RMQ_OK;
}

rmq_status rmq_query_index_ex(rmq_index idx, const int32_t* L, const int32_t* R, int64_t q,
                              int32_t* out, void* stream, const rmq_options* opt) {
  if (!idx || q < 0 || q > RMQ_MAX_Q) return RMQ_ERR_INVALID_ARG;
  if (!check_query_ptrs(L, R, out, q)) return RMQ_ERR_INVALID_ARG;
  if (q && (!aligned_to(L, 4) || !aligned_to(R, 4) || !aligned_to(out, 4)))
    return RMQ_ERR_MISALIGNED;
  if (q == 0) return RMQ_OK;
  int64_t* bad = opt ? opt->bad_count : nullptr;
  uint64_t* stats = opt ? opt->stats : nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e =
      idx->sub ? launch_query_full2(idx->A, idx->n, idx->kshift, idx->st, idx->nb, idx->sub,
                                    idx->k1shift, L, R, q, out, bad, stats, s, idx->lg, idx->rec,
                                    idx->levels)
               : launch_query_full(idx->A, idx->n, idx->kshift, idx->st, idx->nb, L, R, q, out,
                                   bad, stats, s, idx->lg, idx->rec, idx->levels);
  return from_hip(e);
}

rmq_status rmq_query_index(rmq_index idx, const int32_t* L, const int32_t* R, int64_t q,
                           int32_t* out, void* stream) {
  return rmq_query_index_ex(idx, L, R, q, out, stream, nullptr);
}

rmq_status rmq_index_free(rmq_index idx) {
  if (!idx) return RMQ_ERR_INVALID_ARG;
  hipError_t e = hipFree(idx->st);
  free(idx);
  return from_hip(e);
}

rmq_status rmq_index_info(rmq_index idx, int64_t* n, int32_t* block_size, int64_t* nb,
                          int32_t* levels, size_t* bytes) {
  if (!idx) return RMQ_ERR_INVALID_ARG;
  if (n) *n = idx->n;
  if (block_size) *block_size = (int32_t)(1 << idx->kshift);
  if (nb) *nb = idx->nb;
  if (levels) *levels = idx->levels;
  if (bytes) *bytes = idx->bytes;
  return RMQ_OK;
}

rmq_status rmq_index_copy_table(rmq_index idx, uint64_t* st, void* stream) {
  if (!idx || !st) return RMQ_ERR_INVALID_ARG;
  const size_t table_bytes = sizeof(uint64_t) * (size_t)idx->nb * (size_t)idx->levels;
  return from_hip(hipMemcpyAsync(st, idx->st, table_bytes, hipMemcpyDeviceToDevice,
                                 static_cast<hipStream_t>(stream)));
}

// ---- single stages ----
rmq_status rmq_block_minima(const int32_t* A, int64_t n, int32_t k, uint64_t* keys,
                            void* stream) {
  if (!A || !keys || n < 1 || n > RMQ_MAX_N || !is_pow2_block(k)) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(A, 4) || !aligned_to(keys, 8)) return RMQ_ERR_MISALIGNED;
  return from_hip(launch_blockmin_i32(A, n, ilog2_i64(k), keys, static_cast<hipStream_t>(stream)));
}

rmq_status rmq_block_minima_keys(const uint64_t* src, int64_t m, int32_t k, uint64_t* keys,
                                 void* stream) {
  if (!src || !keys || m < 1 || m > 2 * RMQ_MAX_Q || !is_pow2_block(k)) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(src, 8) || !aligned_to(keys, 8)) return RMQ_ERR_MISALIGNED;
  return from_hip(
      launch_blockmin_keys(src, m, ilog2_i64(k), keys, static_cast<hipStream_t>(stream)));
}

rmq_status rmq_sparse_table_build(uint64_t* st, int64_t nb, int32_t levels, void* stream) {
  if (!st || nb < 1 || levels < 1 || levels > 62) return RMQ_ERR_INVALID_ARG;
  if ((levels > 1) && ((int64_t)1 << (levels - 1)) > nb) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(st, 8)) return RMQ_ERR_MISALIGNED;
  return from_hip(launch_sparse_table(st, nb, levels, static_cast<hipStream_t>(stream)));
}

// The sort's own workspace, then the packed list it leaves before splitting
// it into positions and tags.
static size_t stage_sort_bytes(int64_t q) {
  return q > 0 ? align_up(sort_workspace_bytes(q)) + sizeof(uint64_t) * 2 * (size_t)q : 0;
}

size_t rmq_sort_workspace_bytes(int64_t q) {
  if (q < 0 || q > RMQ_MAX_Q) return 0;
  return stage_sort_bytes(q);
}

rmq_status rmq_sort_endpoints(const int32_t* L, const int32_t* R, int64_t q, int64_t n,
                              int32_t* pos, int32_t* tag, void* workspace, size_t ws_bytes,
                              void* stream) {
  if (q < 0 || q > RMQ_MAX_Q || n < 1 || n > RMQ_MAX_N) return RMQ_ERR_INVALID_ARG;
  if (q == 0) return RMQ_OK;
  if (!L || !R || !pos || !tag || !workspace) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(L, 4) || !aligned_to(R, 4) || !aligned_to(pos, 4) || !aligned_to(tag, 4) ||
      !aligned_to(workspace, ALIGN))
    return RMQ_ERR_MISALIGNED;
  if (ws_bytes < stage_sort_bytes(q)) return RMQ_ERR_WORKSPACE_SMALL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t sort_b = align_up(sort_workspace_bytes(q));
  uint64_t* E = reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + sort_b);
  hipError_t e = launch_sort_endpoints(L, R, q, n, E, nullptr, nullptr, workspace, sort_b, s);
  if (e == hipSuccess) e = launch_unpack_endpoints(E, q, pos, tag, sort_abort_word(workspace, q), s);
  return from_hip(e);
}

rmq_status rmq_contract(const int32_t* A, int64_t n, const int32_t* pos, const int32_t* tag,
                        int64_t q, int32_t* LR, uint64_t* aq, void* stream) {
  if (!A || n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return RMQ_ERR_INVALID_ARG;
  if (q == 0) return RMQ_OK;
  if (!pos || !tag || !LR || !aq) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(A, 4) || !aligned_to(pos, 4) || !aligned_to(tag, 4) || !aligned_to(LR, 8) ||
      !aligned_to(aq, 8))
    return RMQ_ERR_MISALIGNED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  prepare_pool();
  const size_t sort_b = align_up(sort_workspace_bytes(q));
  const size_t list_b = align_up(sizeof(uint64_t) * 2 * (size_t)q);
  void* scratch = nullptr;
  hipError_t e = hipMallocAsync(&scratch, sort_b + list_b + contract_tile_start_bytes(n), s);
  if (e != hipSuccess) return from_hip(e);
  char* w = static_cast<char*>(scratch);
  uint64_t* E = reinterpret_cast<uint64_t*>(w + sort_b);
  e = launch_pack_endpoints(pos, tag, q, E, s);
  if (e == hipSuccess) e = launch_remap(E, q, LR, w, sort_b, s);
  if (e == hipSuccess)
    e = launch_contract(A, n, pos, q, aq, reinterpret_cast<int32_t*>(w + sort_b + list_b), s,
                        nullptr);
  hipFreeAsync(scratch, s);
  return from_hip(e);
}

rmq_status rmq_test_sort_abort(int32_t on) {
  set_sort_abort_preset(on != 0);
  return RMQ_OK;
}

// ---- timers ----
rmq_status rmq_timer_create(rmq_timer** t) {
  if (!t) return RMQ_ERR_INVALID_ARG;
  rmq_timer_s* x = new (std::nothrow) rmq_timer_s();
  if (!x) return RMQ_ERR_OUT_OF_MEMORY;
  for (int i = 0; i < RMQ_NUM_STAGES; ++i) {
    hipError_t e = hipEventCreate(&x->clock[i].start);
    if (e == hipSuccess) e = hipEventCreate(&x->clock[i].stop);
    if (e != hipSuccess) {
      for (int j = 0; j <= i; ++j) {
        if (x->clock[j].start) hipEventDestroy(x->clock[j].start);
        if (x->clock[j].stop) hipEventDestroy(x->clock[j].stop);
      }
      delete x;
      return from_hip(e);
    }
  }
  *t = x;
  return RMQ_OK;
}

rmq_status rmq_timer_read(rmq_timer* t, float* stage_ms, float* total_ms) {
  if (!t || !t->armed) return RMQ_ERR_INVALID_ARG;
  int first = -1, last = -1;
  for (int i = 0; i < RMQ_NUM_STAGES; ++i)
    if (t->ran[i]) {
      if (first < 0) first = i;
      last = i;
    }
  if (first < 0) return RMQ_ERR_INVALID_ARG;
  hipError_t e = hipEventSynchronize(t->clock[last].stop);
  if (e != hipSuccess) return from_hip(e);
  for (int i = 0; i < RMQ_NUM_STAGES; ++i) {
    float ms = 0.f;
    if (t->ran[i]) {
      e = hipEventElapsedTime(&ms, t->clock[i].start, t->clock[i].stop);
      if (e != hipSuccess) return from_hip(e);
    }
    if (stage_ms) stage_ms[i] = ms;
  }
  if (total_ms) {
    e = hipEventElapsedTime(total_ms, t->clock[first].start, t->clock[last].stop);
    if (e != hipSuccess) return from_hip(e);
  }
  return RMQ_OK;
}

rmq_status rmq_timer_destroy(rmq_timer* t) {
  if (!t) return RMQ_ERR_INVALID_ARG;
  for (int i = 0; i < RMQ_NUM_STAGES; ++i) {
    hipEventDestroy(t->clock[i].start);
    hipEventDestroy(t->clock[i].stop);
  }
  delete t;
  return RMQ_OK;
}

}  // extern "C"

// ---- batches of arrays ----
// A batched launch's job table on the device (see ChunkJob and friends).
template <class Job>
struct JobTable {
  const Job* jobs = nullptr;
  int64_t count = 0;
};

struct rmq_batch_s {
  int device;
  std::vector<rmq_batch_item> items;
  std::vector<Plan> plans;
  std::vector<size_t> ws_off;  // per item, into ws
  char* ws = nullptr;          // device scratch for every item, then the job tables
  size_t ws_bytes = 0;
  std::vector<int> full_items;  // plain-path items, run together by the batched kernels
  JobTable<ChunkJob> blockmin, keys;
  int rounds = 0;
  JobTable<TileJob> round[ST_MAX_ROUNDS];
  // query waves: those of arrays with two block levels first, then the others
  JobTable<WaveJob> queries;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
};

namespace {

rmq_status batch_enqueue(rmq_batch b, int mode, hipStream_t s) {
  if (mode == RMQ_BATCH_FUSED && !b->full_items.empty()) {
    hipError_t e = launch_blockmin_multi(b->blockmin.jobs, b->blockmin.count, s);
    if (e == hipSuccess) e = launch_blockmin_keys_multi(b->keys.jobs, b->keys.count, s);
    for (int r = 0; e == hipSuccess && r < b->rounds; ++r)
      e = launch_sparse_table_multi(b->round[r].jobs, r, b->round[r].count, s);
    if (e == hipSuccess) e = launch_query_multi(b->queries.jobs, b->queries.count, s);
    if (e != hipSuccess) return from_hip(e);
  }
  for (size_t i = 0; i < b->items.size(); ++i) {
    const Plan& p = b->plans[i];
    if (mode == RMQ_BATCH_FUSED && p.path == RMQ_PATH_FULL) continue;
    const rmq_batch_item& it = b->items[i];
    if (it.q == 0) continue;
    char* w = b->ws + b->ws_off[i];
    rmq_status st = p.path == RMQ_PATH_FULL
                        ? run_full(it.A, it.n, it.L, it.R, it.q, it.out, s, nullptr, p, w)
                        : run_contracted(it.A, it.n, it.L, it.R, it.q, it.out, s, nullptr, p, w);
    if (st != RMQ_OK) return st;
  }
  return RMQ_OK;
}

}  // namespace

extern "C" {

rmq_status rmq_batch_create(const rmq_batch_item* items, int32_t count, rmq_batch* out) {
  if (!items || !out || count < 1) return RMQ_ERR_INVALID_ARG;
  for (int32_t i = 0; i < count; ++i) {
    const rmq_batch_item& it = items[i];
    if (!it.A || it.n < 1 || it.n > RMQ_MAX_N || it.q < 0 || it.q > RMQ_MAX_Q)
      return RMQ_ERR_INVALID_ARG;
    if (it.q > 0 && (!it.L || !it.R || !it.out)) return RMQ_ERR_INVALID_ARG;
    if (!aligned_to(it.A, 4) ||
        (it.q && (!aligned_to(it.L, 4) || !aligned_to(it.R, 4) || !aligned_to(it.out, 4))))
      return RMQ_ERR_MISALIGNED;
  }
  rmq_batch_s* b = new (std::nothrow) rmq_batch_s();
  if (!b) return RMQ_ERR_OUT_OF_MEMORY;
  hipGetDevice(&b->device);
  b->items.assign(items, items + count);
  b->plans.resize(count);
  b->ws_off.resize(count);
  size_t off = 0;
  for (int32_t i = 0; i < count; ++i) {
    rmq_options o{};
    o.block_size = items[i].block_size;
    o.path = items[i].path;
    // the planner's choice, two block levels (Section 3.3) included
    rmq_status st = make_plan(items[i].n, items[i].q, &o, &b->plans[i]);
    if (st != RMQ_OK) {
      delete b;
      return st;
    }
    // Two adjustments of the plain-method plans for one launch per phase,
    // unless the caller fixed the block size or the path:
    // * at most 2^10 blocks per array: then the first Sparse Table round
    //   (levels 1 .. 10) builds every table and the batch needs no second
    //   round launch;
    // * in one launch a wave reads its lanes' partial blocks one range at a
    //   time, so an item over large one-level blocks sets the launch's tail:
    //   blocks over 4096 elements get the k1-block level (scans then stay
    //   within k1 elements).
    Plan& pl = b->plans[i];
    if (items[i].block_size == 0 && items[i].path == RMQ_PATH_AUTO &&
        pl.path == RMQ_PATH_FULL) {
      while ((((int64_t)items[i].n + pl.k - 1) >> pl.kshift) > BATCH_MAX_BLOCKS) {
        pl.k *= 2;
        pl.kshift += 1;
      }
      if (pl.k1shift < 0 && pl.k > BATCH_ONE_LEVEL_MAX_K) pl.k1shift = ilog2_i64(BATCH_SUB_BLOCK);
    }
    b->plans[i].records = false;  // the batched kernels read the level-major table
    b->ws_off[i] = off;
    off = align_up(off + plan_bytes(items[i].n, items[i].q, b->plans[i]));
    if (b->plans[i].path == RMQ_PATH_FULL) b->full_items.push_back(i);
  }
  b->ws_bytes = off;

  // job tables of the plain-path items (their device addresses are filled
  // in once the scratch exists; offsets into the scratch until then)
  std::vector<ChunkJob> jb_min, jb_keys;
  std::vector<TileJob> jb_round[ST_MAX_ROUNDS];
  std::vector<WaveJob> jb_q2, jb_q1;
  std::vector<ArrayDesc> desc;
  for (int i : b->full_items) {
    const rmq_batch_item& it = items[i];
    const Plan& p = b->plans[i];
    const FullLayout f = full_layout(it.n, p.k, p.k1shift, 1, false);
    const bool two = p.k1shift >= 0;
    desc.push_back(ArrayDesc{it.A, it.n, p.kshift, f.levels, f.nb, nullptr, it.L, it.R, it.q,
                             it.out, 1, nullptr, 0, nullptr, f.nb1, p.k1shift});
    const int64_t g = blockmin_grid(it.n, two ? p.k1shift : p.kshift, 4);
    for (int64_t c = 0; c < g; ++c)
      jb_min.push_back(ChunkJob{it.A, nullptr, it.n, two ? p.k1shift : p.kshift, (int32_t)c});
    if (two) {
      const int64_t gk = blockmin_keys_grid(f.nb1, p.kshift - p.k1shift);
      for (int64_t c = 0; c < gk; ++c)
        jb_keys.push_back(ChunkJob{nullptr, nullptr, f.nb1, p.kshift - p.k1shift, (int32_t)c});
    }
    const int rounds = st_rounds(f.levels);
    if (rounds > ST_MAX_ROUNDS) {
      delete b;
      return RMQ_ERR_INVALID_ARG;
    }
    if (rounds > b->rounds) b->rounds = rounds;
    for (int r = 0; r < rounds; ++r) {
      const int64_t tiles = st_round_tiles(f.nb, f.levels, r);
      for (int64_t t = 0; t < tiles; ++t)
        jb_round[r].push_back(TileJob{nullptr, f.nb, f.levels, (int32_t)t});
    }
    for (int64_t q0 = 0; q0 < it.q; q0 += 64) (two ? jb_q2 : jb_q1).push_back(WaveJob{{}, q0});
  }
  // where each job's array and pointers are: record the item per job
  size_t tbytes = 0;
  auto tsize = [](size_t bytes) { return align_up(bytes ? bytes : 1); };
  tbytes += tsize(sizeof(ChunkJob) * jb_min.size()) + tsize(sizeof(ChunkJob) * jb_keys.size());
  for (int r = 0; r < ST_MAX_ROUNDS; ++r) tbytes += tsize(sizeof(TileJob) * jb_round[r].size());
  tbytes += tsize(sizeof(WaveJob) * jb_q2.size()) + tsize(sizeof(WaveJob) * jb_q1.size());

  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, b->ws_bytes + tbytes);
  if (e != hipSuccess) {
    delete b;
    return from_hip(e);
  }
  b->ws = static_cast<char*>(mem);
  // fill in the device pointers: per item its table and k1-block minima
  {
    size_t a = 0, k = 0, q2 = 0, q1 = 0;
    size_t rr[ST_MAX_ROUNDS] = {};
    for (size_t c = 0; c < b->full_items.size(); ++c) {
      const int i = b->full_items[c];
      const Plan& p = b->plans[i];
      const FullLayout f = full_layout(items[i].n, p.k, p.k1shift, 1, false);
      char* w = b->ws + b->ws_off[i];
      ArrayDesc& d = desc[c];
      d.st = reinterpret_cast<uint64_t*>(w + f.off_st);
      d.sub = p.k1shift >= 0 ? reinterpret_cast<uint64_t*>(w + f.off_sub) : nullptr;
      const bool two = d.sub != nullptr;
      const int64_t g = blockmin_grid(items[i].n, two ? p.k1shift : p.kshift, 4);
      for (int64_t j = 0; j < g; ++j) jb_min[a++].keys = two ? d.sub : d.st;
      if (two) {
        const int64_t gk = blockmin_keys_grid(f.nb1, p.kshift - p.k1shift);
        for (int64_t j = 0; j < gk; ++j, ++k) {
          jb_keys[k].src = d.sub;
          jb_keys[k].keys = d.st;
        }
      }
      for (int r = 0; r < st_rounds(f.levels); ++r) {
        const int64_t tiles = st_round_tiles(f.nb, f.levels, r);
        for (int64_t t = 0; t < tiles; ++t) jb_round[r][rr[r]++].st = d.st;
      }
      for (int64_t q0 = 0; q0 < items[i].q; q0 += 64) (two ? jb_q2[q2++] : jb_q1[q1++]).d = d;
    }
  }
  std::vector<char> img(tbytes);
  size_t at = 0;
  char* dbase = b->ws + b->ws_bytes;
  auto place = [&](const void* src, size_t bytes) {
    if (bytes) memcpy(img.data() + at, src, bytes);
    const char* dev = dbase + at;
    at += tsize(bytes);
    return dev;
  };
  auto put = [&](auto& table, const auto& host) {
    using Job = typename std::remove_reference<decltype(host)>::type::value_type;
    table.jobs = reinterpret_cast<const Job*>(place(host.data(), sizeof(Job) * host.size()));
    table.count = (int64_t)host.size();
  };
  put(b->blockmin, jb_min);
  put(b->keys, jb_keys);
  for (int r = 0; r < ST_MAX_ROUNDS; ++r) put(b->round[r], jb_round[r]);
  // waves over larger blocks first (longer partial scans, slower waves), so
  // that the launch ends on short ones (the benchmark's 256-array batch: the
  // query launch 62 -> 56 us, the fused batch 0.303-0.315 -> 0.296-0.314 ms)
  jb_q2.insert(jb_q2.end(), jb_q1.begin(), jb_q1.end());
  std::stable_sort(jb_q2.begin(), jb_q2.end(),
                   [](const WaveJob& x, const WaveJob& y) { return x.d.kshift > y.d.kshift; });
  put(b->queries, jb_q2);
  e = hipMemcpy(dbase, img.data(), tbytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(mem);
    delete b;
    return from_hip(e);
  }
  *out = b;
  return RMQ_OK;
}

rmq_status rmq_batch_run(rmq_batch b, int32_t mode, int32_t use_graph, void* stream) {
  if (!b || (mode != RMQ_BATCH_FUSED && mode != RMQ_BATCH_PER_ITEM)) return RMQ_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!use_graph) return batch_enqueue(b, mode, s);
  if (!s) return RMQ_ERR_INVALID_ARG;  // capture needs a stream of its own
  if (!b->graph[mode]) {
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return from_hip(e);
    rmq_status st = batch_enqueue(b, mode, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != RMQ_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return from_hip(e);
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return from_hip(e);
    b->graph[mode] = x;
  }
  return from_hip(hipGraphLaunch(b->graph[mode], s));
}

rmq_status rmq_batch_item_plan(rmq_batch b, int32_t i, int32_t* block_size, int32_t* path) {
  return rmq_batch_item_plan_ex(b, i, block_size, path, nullptr);
}

rmq_status rmq_batch_item_plan_ex(rmq_batch b, int32_t i, int32_t* block_size, int32_t* path,
                                  int32_t* sub_block_size) {
  if (!b || i < 0 || i >= (int32_t)b->items.size()) return RMQ_ERR_INVALID_ARG;
  if (block_size) *block_size = b->plans[i].k;
  if (path) *path = b->plans[i].path;
  if (sub_block_size)
    *sub_block_size = b->plans[i].k1shift >= 0 ? (int32_t)(1 << b->plans[i].k1shift) : 0;
  return RMQ_OK;
}

size_t rmq_batch_workspace_bytes(rmq_batch b) { return b ? b->ws_bytes : 0; }

rmq_status rmq_batch_free(rmq_batch b) {
  if (!b) return RMQ_ERR_INVALID_ARG;
  for (int m = 0; m < 2; ++m)
    if (b->graph[m]) hipGraphExecDestroy(b->graph[m]);
  hipError_t e = hipFree(b->ws);
  delete b;
  return from_hip(e);
}

}  // extern "C"
