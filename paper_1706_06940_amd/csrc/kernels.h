// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <tuple>

namespace rmq {

// Optional per-stage clock: while set (by the host API, per thread), every
// launch of a stage records `stop` at its end, and the first one also
// records `start` at its beginning -- the events sit on the kernels
// themselves, so a stage's time is pure kernel time.
struct StageClock {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  bool started = false;
};
extern thread_local StageClock* tl_clock;

// Launch on `stream`.  With a stage clock armed the launch goes through
// hipExtLaunchKernel, which records the clock's events on the kernel itself;
// otherwise through hipLaunchKernel (the form stream capture records as a
// plain kernel node).
template <typename... KArgs, typename... Args>
inline hipError_t launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t lds,
                         hipStream_t stream, Args... args) {
  StageClock* c = tl_clock;
  if (c) {
    hipEvent_t start = c->started ? nullptr : c->start;
    c->started = true;
    hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, start, c->stop, 0u,
                          static_cast<KArgs>(args)...);
    return hipGetLastError();
  }
  std::tuple<KArgs...> vals{static_cast<KArgs>(args)...};
  void* ptrs[sizeof...(KArgs)];
  std::apply(
      [&ptrs](auto&... x) {
        int i = 0;
        ((ptrs[i++] = static_cast<void*>(&x)), ...);
      },
      vals);
  return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, lds, stream);
}

#define RMQ_TRY(expr)                       \
  do {                                      \
    hipError_t rmq_err_ = (expr);           \
    if (rmq_err_ != hipSuccess) return rmq_err_; \
  } while (0)

// One array of a batch on the device: its input, its block Sparse Table
// (level-major, levels x nb keys), with two block levels (Section 3.3) its
// k1-block minima, and its queries.
struct ArrayDesc {
  const int32_t* A;
  int64_t n;
  int32_t kshift;
  int32_t levels;
  int64_t nb;
  uint64_t* st;
  const int32_t* L;
  const int32_t* R;
  int64_t q;
  int32_t* out;
  int32_t lg;  // table arity l = 2^lg (1: doubling)
  const uint64_t* rec;  // query records of the doubling table, or null
  int32_t rlev;         // levels of the records' table
  uint64_t* sub;        // two block levels: the k1-block minima, else null
  int64_t nb1;          // number of k1-blocks
  int32_t k1shift;      // k1 = 2^k1shift (when sub is set)
};

// Sparse Table rounds: round r builds levels j0(r)+1 .. j0(r)+t; j0 = 0,
// 10, 16, 22, ... for every table (see sparse_table.hip).
constexpr int ST_MAX_ROUNDS = 6;
int st_round_j0(int r);
int st_rounds(int levels);
int64_t st_round_tiles(int64_t nb, int levels, int r);
size_t st_round_lds(int r);

// ---- non-contracted path (Section 3.2) ----
hipError_t launch_blockmin_i32(const int32_t* A, int64_t n, int kshift, uint64_t* keys,
                               hipStream_t stream);
hipError_t launch_blockmin_keys(const uint64_t* S, int64_t m, int kshift, uint64_t* keys,
                                hipStream_t stream);
hipError_t launch_sparse_table(uint64_t* st, int64_t nb, int levels, hipStream_t stream);
// l-ary table (Section 3.1), l = 2^lg >= 4: level i holds the minima over
// l^i blocks (truncated at nb); levels = lary_levels(nb, lg).  Level 0 given.
// Levels i >= 1 are stored by residue class mod l^i (lary_addr in device.h).
int lary_levels(int64_t nb, int lg);
hipError_t launch_sparse_table_lary(uint64_t* st, int64_t nb, int lg, hipStream_t stream);
// Query records of a doubling table (levels x nb, level-major), pairs of
// keys on 16-byte boundaries: forward pair (b, t) at rec + 2 (b levels + t)
// holds st[0][b] and st[t][b + 1]; backward pair (b, t) at
// rec + 2 ((nb + b) levels + t) holds st[0][b] and st[t][b - 2^t]; a pair
// without a window holds the min identity there.  4 nb levels keys in all.
hipError_t launch_records(const uint64_t* st, int64_t nb, int levels, uint64_t* rec,
                          hipStream_t stream);
int64_t blockmin_grid(int64_t n, int kshift, int elems_per_lane_load);
// Batched forms: one launch per phase for all arrays of a batch.  Every
// workgroup (block minima, table tiles) or wave (queries) of such a launch
// reads its whole assignment from one record of a job table built on the
// host -- a single load before its first load of data.
struct ChunkJob {            // block minima of one chunk of one array
  const void* src;           //   int32 A, or uint64 k1-block minima
  uint64_t* keys;            //   its blocks' minima go here
  int64_t len;               //   elements of src
  int32_t shift;             //   blocks of 2^shift elements
  int32_t chunk;             //   the chunk (workgroup) index within the array
};
struct TileJob {             // one tile of a table round
  uint64_t* st;
  int64_t nb;
  int32_t levels;
  int32_t tile;
};
struct WaveJob {             // 64 queries of one array (each array's queries
  ArrayDesc d;               //   padded to whole waves)
  int64_t q0;                //   the wave's first query within the array
};
// Block minima over int32 arrays (the k1-block minima for arrays with two
// block levels, else the k-block minima), one workgroup per job.
hipError_t launch_blockmin_multi(const ChunkJob* jobs, int64_t count, hipStream_t stream);
// Two block levels: the k-block minima (st level 0) from the k1-block minima.
hipError_t launch_blockmin_keys_multi(const ChunkJob* jobs, int64_t count, hipStream_t stream);
hipError_t launch_sparse_table_multi(const TileJob* jobs, int round, int64_t count,
                                     hipStream_t stream);
// Each wave's array may have two block levels or one (its job says which).
hipError_t launch_query_multi(const WaveJob* jobs, int64_t waves, hipStream_t stream);
// Serving: one launch over a coalesced batch of requests on resident tables
// (two_level: every table has two block levels, else none has).
hipError_t launch_query_segments(const ArrayDesc* tables, const int64_t* seg_prefix,
                                 const int32_t* seg_table, int nseg, const int32_t* L,
                                 const int32_t* R, int32_t* out, int64_t total, bool two_level,
                                 hipStream_t stream);
// Block count of launch_blockmin_keys for m keys and blocks of 2^kshift.
int64_t blockmin_keys_grid(int64_t m, int kshift);
// lg: the table's arity l = 2^lg (1: doubling; see launch_sparse_table_lary).
hipError_t launch_query_full(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                             int64_t nb, const int32_t* L, const int32_t* R, int64_t q,
                             int32_t* out, int64_t* bad_count, uint64_t* stats,
                             hipStream_t stream, int lg = 1, const uint64_t* rec = nullptr,
                             int rlev = 0);
// LCA queries (Section 1) over the depth array D of an Euler tour.
hipError_t launch_query_lca(const int32_t* D, int64_t len, int kshift, const uint64_t* st,
                            int64_t nb, const uint64_t* sub, int k1shift, const int32_t* first,
                            const int32_t* node, int64_t N, const int32_t* U, const int32_t* V,
                            int64_t q, int32_t* out, int64_t* bad_count, hipStream_t stream,
                            int lg = 1, const uint64_t* rec = nullptr, int rlev = 0);
// Two block levels (Section 3.3): sub holds the minima of the 2^k1shift-blocks.
hipError_t launch_query_full2(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                              int64_t nb, const uint64_t* sub, int k1shift, const int32_t* L,
                              const int32_t* R, int64_t q, int32_t* out, int64_t* bad_count,
                              uint64_t* stats, hipStream_t stream, int lg = 1,
                              const uint64_t* rec = nullptr, int rlev = 0);

// Three block levels (Section 3.3, h = 3): sub holds the k1-block minima,
// sub2 the k2-block minima (k2 < k1 < k, powers of two).
hipError_t launch_query_full3(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                              int64_t nb, const uint64_t* sub, int k1shift, const uint64_t* sub2,
                              int k2shift, const int32_t* L, const int32_t* R, int64_t q,
                              int32_t* out, int64_t* bad_count, uint64_t* stats,
                              hipStream_t stream, int lg = 1);

// Compute units of the current device (cached per device).
int device_cu_count();

// ---- contracted path (Section 3.1) ----
// Device LSD radix sort of the 2q endpoints by (position, tag).  The sorted
// list E holds (position << 32) | tag per slot.  With LR non-null the last
// pass also writes the remap (as launch_remap does) and, since the tags are
// then used up, writes only the positions, as int32 in the first half of E;
// pair_scratch, when given, is 2q 8-byte items through which long sorts
// stage the remap.
size_t sort_workspace_bytes(int64_t q);
hipError_t launch_sort_endpoints(const int32_t* L, const int32_t* R, int64_t q, int64_t n,
                                 uint64_t* E, int32_t* LR, uint64_t* pair_scratch, void* ws,
                                 size_t ws_bytes, hipStream_t stream);
// Remap: LR[2i] = Lc[i], LR[2i+1] = Rc[i] from the sorted list; uses the
// sort's workspace.
hipError_t launch_remap(const uint64_t* E, int64_t q, int32_t* LR, void* ws, size_t ws_bytes,
                        hipStream_t stream);
// Stable sort of N 8-byte items by their high 32 bits (key < 2^key_bits),
// the low 32 bits carried along.  items and out must not alias the
// workspace of sort_pairs_workspace_bytes(N).
size_t sort_pairs_workspace_bytes(int64_t N);
hipError_t launch_sort_pairs(const uint64_t* items, int64_t N, int key_bits, uint64_t* out,
                             void* ws, size_t ws_bytes, hipStream_t stream);
// The sort's abort word inside its workspace (for q queries, or N items of
// sort_pairs): nonzero after a sort whose bounded look-back wait gave up, so
// that its order cannot be trusted.  Device pointer; null for an empty sort.
const uint32_t* sort_abort_word(const void* ws, int64_t q);
const uint32_t* sort_pairs_abort_word(const void* ws, int64_t N);
// Tests of the failure report: every later sort's abort word starts set.
void set_sort_abort_preset(bool on);
// Split E into positions and tags (all -1 if the sort's abort word is set),
// or join them into E.
hipError_t launch_unpack_endpoints(const uint64_t* E, int64_t q, int32_t* pos, int32_t* tag,
                                   const uint32_t* abort_word, hipStream_t stream);
hipError_t launch_pack_endpoints(const int32_t* pos, const int32_t* tag, int64_t q, uint64_t* E,
                                 hipStream_t stream);
// Contraction: A_Q over the closed areas between consecutive endpoints,
// given the 2q sorted endpoint positions E (int32).
// tile_start: scratch of contract_tile_start_bytes(n).  fail (may be null):
// the endpoint sort's abort word; when it is set nothing is done.  A list
// that is not sorted positions of A gives meaningless A_Q but never an
// access out of bounds.
size_t contract_tile_start_bytes(int64_t n);
hipError_t launch_contract(const int32_t* A, int64_t n, const int32_t* E, int64_t q,
                           uint64_t* aq, int32_t* tile_start, hipStream_t stream,
                           const uint32_t* fail);
// ST-RMQ_CON (Section 2): the 2q sorted endpoint positions E, each written
// twice into E2 (4q entries, 8-byte aligned).
hipError_t launch_double_ends(const int32_t* E, int64_t M, int32_t* E2, hipStream_t stream);
// ST-RMQ_CON's queries: st is the Sparse Table over every entry of its A_Q
// (m = 4q - 1 entries, `levels` levels); query i reads entries 2 LR[2i] ..
// 2 LR[2i + 1] + 2.  fail as below.
hipError_t launch_query_st_elements(const uint64_t* st, int64_t m, int levels, const int32_t* L,
                                    const int32_t* R, const int32_t* LR, int64_t q, int64_t n,
                                    int32_t* out, int64_t* bad_count, hipStream_t stream,
                                    const uint32_t* fail);
// fail: the endpoint sort's abort word; when it is set every query is
// answered -1 and counted in bad_count.
hipError_t launch_query_contracted(const uint64_t* aq, int64_t m, int64_t n, int kshift,
                                   const uint64_t* st, int64_t nb, const int32_t* L,
                                   const int32_t* R, const int32_t* LR, int64_t q, int32_t* out,
                                   int64_t* bad_count, uint64_t* stats, hipStream_t stream,
                                   int lg, const uint64_t* rec, int rlev, const uint64_t* sub,
                                   int k1shift, const uint32_t* fail);

}  // namespace rmq
