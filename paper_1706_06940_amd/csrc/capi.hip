// C ABI of the library: argument checks, the planner, workspace layout,
// stage sequencing on the caller's stream and per-stage timing.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "kernels.h"
#include "rmq.h"

using namespace rmq;

struct rmq_timer_s {
  hipEvent_t ev[RMQ_NUM_STAGES + 1];
  bool ran[RMQ_NUM_STAGES];
  bool armed;
};

struct rmq_index_s {
  int device;
  const int32_t* A;
  int64_t n;
  int kshift;
  int64_t nb;
  int levels;
  uint64_t* st;
  size_t bytes;
};

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
constexpr int32_t DEFAULT_BLOCK_CONTRACTED = 512;

struct Plan {
  int path;
  int32_t k;
  int kshift;
};

rmq_status make_plan(int64_t n, int64_t q, const rmq_options* opt, Plan* p) {
  int32_t path = opt ? opt->path : RMQ_PATH_AUTO;
  int32_t k = opt ? opt->block_size : 0;
  if (path != RMQ_PATH_AUTO && path != RMQ_PATH_FULL && path != RMQ_PATH_CONTRACTED)
    return RMQ_ERR_INVALID_ARG;
  if (k != 0 && !is_pow2_block(k)) return RMQ_ERR_INVALID_ARG;
  if (path == RMQ_PATH_AUTO) {
    int32_t pk = 0, pp = 0;
    rmq_plan(n, q, &pk, &pp);
    path = pp;
    if (k == 0) k = pk;
  }
  if (k == 0) k = path == RMQ_PATH_FULL ? default_block_full(n) : DEFAULT_BLOCK_CONTRACTED;
  p->path = path;
  p->k = k;
  p->kshift = ilog2_i64(k);
  return RMQ_OK;
}

// ---- workspace layouts ----
struct FullLayout {
  int64_t nb;
  int levels;
  size_t off_st, bytes;
};

FullLayout full_layout(int64_t n, int64_t k) {
  FullLayout f{};
  f.nb = num_blocks(n, k);
  f.levels = rmq_table_levels(f.nb);
  f.off_st = 0;
  f.bytes = align_up(sizeof(uint64_t) * (size_t)f.nb * (size_t)f.levels);
  return f;
}

struct ConLayout {
  int64_t M, m, nb;
  int levels;
  size_t off_pos, off_tag, off_sort, off_lc, off_rc, off_aq, off_tiles, off_st, bytes;
};

ConLayout con_layout(int64_t n, int64_t q, int64_t k) {
  ConLayout c{};
  c.M = 2 * q;
  c.m = c.M - 1;
  c.nb = num_blocks(c.m, k);
  c.levels = rmq_table_levels(c.nb);
  size_t o = 0;
  c.off_pos = o;
  o = align_up(o + sizeof(int32_t) * (size_t)c.M);
  c.off_tag = o;
  o = align_up(o + sizeof(int32_t) * (size_t)c.M);
  c.off_sort = o;
  o = align_up(o + sort_workspace_bytes(q));
  c.off_lc = o;
  o = align_up(o + sizeof(int32_t) * (size_t)q);
  c.off_rc = o;
  o = align_up(o + sizeof(int32_t) * (size_t)q);
  c.off_aq = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.m);
  c.off_tiles = o;
  o = align_up(o + contract_tile_start_bytes(n));
  c.off_st = o;
  o = align_up(o + sizeof(uint64_t) * (size_t)c.nb * (size_t)c.levels);
  c.bytes = o;
  return c;
}

size_t plan_bytes(int64_t n, int64_t q, const Plan& p) {
  if (p.path == RMQ_PATH_FULL) return full_layout(n, p.k).bytes;
  return con_layout(n, q, p.k).bytes;
}

std::once_flag g_pool_once[64];

// Keep freed stream-ordered memory cached in the device pool, so that
// per-call scratch costs no device allocation after the first call.
void prepare_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::call_once(g_pool_once[dev], [dev] {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
}

void timer_mark(rmq_timer* t, int i, hipStream_t s) {
  if (t) hipEventRecord(t->ev[i], s);
}

bool check_query_ptrs(const int32_t* L, const int32_t* R, int32_t* out, int64_t q) {
  if (q == 0) return true;
  return L && R && out;
}

rmq_status run_full(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R, int64_t q,
                    int32_t* out, hipStream_t s, const rmq_options* opt, const Plan& p,
                    char* ws) {
  rmq_timer* t = opt ? opt->timer : nullptr;
  const FullLayout f = full_layout(n, p.k);
  uint64_t* st = reinterpret_cast<uint64_t*>(ws + f.off_st);
  timer_mark(t, 0, s);
  timer_mark(t, 1, s);  // no sort stage on this path
  hipError_t e = launch_blockmin_i32(A, n, p.kshift, st, s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 2, s);
  e = launch_sparse_table(st, f.nb, f.levels, s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 3, s);
  e = launch_query_full(A, n, p.kshift, st, f.nb, L, R, q, out, opt ? opt->bad_count : nullptr,
                        opt ? opt->stats : nullptr, s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 4, s);
  if (t) {
    t->ran[0] = false;
    t->ran[1] = t->ran[2] = t->ran[3] = true;
    t->armed = true;
  }
  return RMQ_OK;
}

rmq_status run_contracted(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R,
                          int64_t q, int32_t* out, hipStream_t s, const rmq_options* opt,
                          const Plan& p, char* ws) {
  rmq_timer* t = opt ? opt->timer : nullptr;
  const ConLayout c = con_layout(n, q, p.k);
  int32_t* pos = reinterpret_cast<int32_t*>(ws + c.off_pos);
  int32_t* tag = reinterpret_cast<int32_t*>(ws + c.off_tag);
  int32_t* Lc = reinterpret_cast<int32_t*>(ws + c.off_lc);
  int32_t* Rc = reinterpret_cast<int32_t*>(ws + c.off_rc);
  uint64_t* aq = reinterpret_cast<uint64_t*>(ws + c.off_aq);
  int32_t* tiles = reinterpret_cast<int32_t*>(ws + c.off_tiles);
  uint64_t* st = reinterpret_cast<uint64_t*>(ws + c.off_st);
  timer_mark(t, 0, s);
  hipError_t e = launch_sort_endpoints(L, R, q, n, pos, tag, ws + c.off_sort,
                                       sort_workspace_bytes(q), s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 1, s);
  e = launch_contract(A, n, pos, tag, q, Lc, Rc, aq, tiles, s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 2, s);
  e = launch_blockmin_keys(aq, c.m, p.kshift, st, s);
  if (e != hipSuccess) return from_hip(e);
  e = launch_sparse_table(st, c.nb, c.levels, s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 3, s);
  e = launch_query_contracted(aq, c.m, n, p.kshift, st, c.nb, L, R, Lc, Rc, q, out,
                              opt ? opt->bad_count : nullptr, opt ? opt->stats : nullptr, s);
  if (e != hipSuccess) return from_hip(e);
  timer_mark(t, 4, s);
  if (t) {
    t->ran[0] = t->ran[1] = t->ran[2] = t->ran[3] = true;
    t->armed = true;
  }
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
  }
  return "unknown status";
}

const char* rmq_version(void) { return "rmq-gfx950 1.0"; }

int32_t rmq_table_levels(int64_t nb) {
  if (nb <= 3) return 1;
  return ilog2_i64(nb - 2) + 1;
}

size_t rmq_index_bytes(int64_t n, int32_t k) {
  if (n < 1 || n > RMQ_MAX_N || !is_pow2_block(k)) return 0;
  const int64_t nb = num_blocks(n, k);
  return sizeof(uint64_t) * (size_t)nb * (size_t)rmq_table_levels(nb);
}

rmq_status rmq_plan(int64_t n, int64_t q, int32_t* block_size, int32_t* path) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return RMQ_ERR_INVALID_ARG;
  // Both methods stream A once (the contracted one between its outermost
  // endpoints, which for queries spread over A is all of it); the contracted
  // one adds a sort of 2q endpoints and a pass over A_Q, so the plain one is
  // the cheaper choice for every batch whose endpoints span A.
  if (block_size) *block_size = default_block_full(n);
  if (path) *path = RMQ_PATH_FULL;
  return RMQ_OK;
}

size_t rmq_workspace_bytes(int64_t n, int64_t q, const rmq_options* opt) {
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return 0;
  if (q == 0) return 0;
  Plan p;
  if (make_plan(n, q, opt, &p) != RMQ_OK) return 0;
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
  rmq_status st = make_plan(n, q, opt, &p);
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
    prepare_pool();
    void* w = nullptr;
    hipError_t e = hipMallocAsync(&w, need, s);
    if (e != hipSuccess) return from_hip(e);
    ws = static_cast<char*>(w);
    own = true;
  }
  st = p.path == RMQ_PATH_FULL ? run_full(A, n, L, R, q, out, s, opt, p, ws)
                               : run_contracted(A, n, L, R, q, out, s, opt, p, ws);
  if (own) hipFreeAsync(ws, s);
  return st;
}

rmq_status rmq_query_batch(const int32_t* A, int64_t n, const int32_t* L, const int32_t* R,
                           int64_t q, int32_t* out, void* stream) {
  return rmq_query_batch_ex(A, n, L, R, q, out, stream, nullptr);
}

// ---- resident index ----
rmq_status rmq_build(const int32_t* A, int64_t n, const rmq_options* opt, void* stream,
                     rmq_index* idx) {
  if (!A || !idx || n < 1 || n > RMQ_MAX_N) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(A, 4)) return RMQ_ERR_MISALIGNED;
  int32_t k = opt ? opt->block_size : 0;
  if (k == 0) {
    // Section 3.2: k = Theta(sqrt(n)) keeps both the query time and the
    // space of the index low; a power of two near sqrt(n) / 4.
    const double tgt = sqrt((double)n) / 4.0;
    k = 256;
    while (k < (1 << 20) && (double)(k * 2) <= tgt) k *= 2;
  }
  if (!is_pow2_block(k)) return RMQ_ERR_INVALID_ARG;
  rmq_index_s* ix = static_cast<rmq_index_s*>(calloc(1, sizeof(rmq_index_s)));
  if (!ix) return RMQ_ERR_OUT_OF_MEMORY;
  hipGetDevice(&ix->device);
  ix->A = A;
  ix->n = n;
  ix->kshift = ilog2_i64(k);
  ix->nb = num_blocks(n, k);
  ix->levels = rmq_table_levels(ix->nb);
  ix->bytes = sizeof(uint64_t) * (size_t)ix->nb * (size_t)ix->levels;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, ix->bytes);
  if (e != hipSuccess) {
    free(ix);
    return from_hip(e);
  }
  ix->st = static_cast<uint64_t*>(mem);
  hipStream_t s = static_cast<hipStream_t>(stream);
  e = launch_blockmin_i32(A, n, ix->kshift, ix->st, s);
  if (e == hipSuccess) e = launch_sparse_table(ix->st, ix->nb, ix->levels, s);
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
  hipError_t e = launch_query_full(idx->A, idx->n, idx->kshift, idx->st, idx->nb, L, R, q, out,
                                   opt ? opt->bad_count : nullptr, opt ? opt->stats : nullptr,
                                   static_cast<hipStream_t>(stream));
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
  return from_hip(hipMemcpyAsync(st, idx->st, idx->bytes, hipMemcpyDeviceToDevice,
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

size_t rmq_sort_workspace_bytes(int64_t q) {
  if (q < 0 || q > RMQ_MAX_Q) return 0;
  return sort_workspace_bytes(q);
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
  if (ws_bytes < sort_workspace_bytes(q)) return RMQ_ERR_WORKSPACE_SMALL;
  return from_hip(launch_sort_endpoints(L, R, q, n, pos, tag, workspace, ws_bytes,
                                        static_cast<hipStream_t>(stream)));
}

rmq_status rmq_contract(const int32_t* A, int64_t n, const int32_t* pos, const int32_t* tag,
                        int64_t q, int32_t* Lc, int32_t* Rc, uint64_t* aq, void* stream) {
  if (!A || n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q) return RMQ_ERR_INVALID_ARG;
  if (q == 0) return RMQ_OK;
  if (!pos || !tag || !Lc || !Rc || !aq) return RMQ_ERR_INVALID_ARG;
  if (!aligned_to(A, 4) || !aligned_to(aq, 8)) return RMQ_ERR_MISALIGNED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  prepare_pool();
  void* tiles = nullptr;
  hipError_t e = hipMallocAsync(&tiles, contract_tile_start_bytes(n), s);
  if (e != hipSuccess) return from_hip(e);
  e = launch_contract(A, n, pos, tag, q, Lc, Rc, aq, static_cast<int32_t*>(tiles), s);
  hipFreeAsync(tiles, s);
  return from_hip(e);
}

// ---- timers ----
rmq_status rmq_timer_create(rmq_timer** t) {
  if (!t) return RMQ_ERR_INVALID_ARG;
  rmq_timer_s* x = static_cast<rmq_timer_s*>(calloc(1, sizeof(rmq_timer_s)));
  if (!x) return RMQ_ERR_OUT_OF_MEMORY;
  for (int i = 0; i <= RMQ_NUM_STAGES; ++i) {
    hipError_t e = hipEventCreate(&x->ev[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) hipEventDestroy(x->ev[j]);
      free(x);
      return from_hip(e);
    }
  }
  *t = x;
  return RMQ_OK;
}

rmq_status rmq_timer_read(rmq_timer* t, float* stage_ms, float* total_ms) {
  if (!t || !t->armed) return RMQ_ERR_INVALID_ARG;
  hipError_t e = hipEventSynchronize(t->ev[RMQ_NUM_STAGES]);
  if (e != hipSuccess) return from_hip(e);
  for (int i = 0; i < RMQ_NUM_STAGES; ++i) {
    float ms = 0.f;
    if (t->ran[i]) {
      e = hipEventElapsedTime(&ms, t->ev[i], t->ev[i + 1]);
      if (e != hipSuccess) return from_hip(e);
    }
    if (stage_ms) stage_ms[i] = ms;
  }
  if (total_ms) {
    e = hipEventElapsedTime(total_ms, t->ev[0], t->ev[RMQ_NUM_STAGES]);
    if (e != hipSuccess) return from_hip(e);
  }
  return RMQ_OK;
}

rmq_status rmq_timer_destroy(rmq_timer* t) {
  if (!t) return RMQ_ERR_INVALID_ARG;
  for (int i = 0; i <= RMQ_NUM_STAGES; ++i) hipEventDestroy(t->ev[i]);
  free(t);
  return RMQ_OK;
}

}  // extern "C"
