// Lowest common ancestors through RMQ (Section 1): in the Euler tour of a
// rooted tree, LCA(u, v) is the node of minimum depth between the first
// occurrences of u and v.  This file builds the tour on the device.
//
// Arcs: node c != root has a down arc 2c (parent -> c) and an up arc 2c+1
// (c -> parent).  With the children of every node in increasing id, the
// tour's arc list is
//   next(down c) = down(first child of c), or up c if c is a leaf;
//   next(up c)   = down(next sibling of c), or up(parent) -- or the end when
//                  the parent is the root;
// starting at down(first child of root).  The tour is the root followed by
// the head node of each arc in list order (2N - 1 nodes); the depth changes
// by +1 on a down arc and -1 on an up arc.
//
// Steps:
//   1. check the parent array (one root, parents in range);
//   2. stable radix sort of (parent + 1, child) -> children grouped by
//      parent, in increasing id; first child and next sibling of each node;
//   3. arc successors;
//   4. list ranking: every arc whose index is a multiple of SPLIT (and the
//      list head) starts a walk that numbers the arcs up to the next such
//      arc, summing counts and depth steps; pointer jumping over the walks'
//      sublists gives each sublist's offset from the head;
//   5. each arc's tour position and depth, then the tour's node and depth
//      arrays and every node's first position;
//   6. a resident RMQ index over the depth array.
// Every walk and jump loop is bounded; the host checks that the list from
// the head has 2(N - 1) arcs and ends (no cycle) before accepting the tour.
#include <stdlib.h>

#include "device.h"
#include "index.h"
#include "kernels.h"
#include "rmq.h"

struct rmq_lca_s {
  int device;
  int64_t N;
  int32_t root;
  int32_t* depth;  // 2N - 1
  int32_t* node;   // 2N - 1
  int32_t* first;  // N
  void* mem;       // the three arrays above
  size_t bytes;
  rmq_index idx;   // RMQ index over depth
};

namespace rmq {

namespace {
typedef int32_t v2i32 __attribute__((ext_vector_type(2)));  // (count, depth sum)

constexpr int WG = 256;
constexpr int32_t END = -1;      // successor of the last arc
constexpr int32_t NOT_ARC = -2;  // the root's two arc slots
constexpr int64_t SPLIT = 64;    // one sampled arc per SPLIT arc indices

int64_t blocks(int64_t n) { return (n + WG - 1) / WG; }

// stat[0] += roots, stat[1] += parents out of range, stat[2] = a root
__global__ __launch_bounds__(WG) void k_lca_check(const int32_t* __restrict__ parent, int64_t N,
                                                  unsigned long long* __restrict__ stat) {
  const int64_t v = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (v >= N) return;
  const int32_t p = parent[v];
  if (p == -1) {
    atomicAdd(&stat[0], 1ull);
    atomicExch(&stat[2], (unsigned long long)v);
  } else if (p < 0 || p >= N || p == v) {
    atomicAdd(&stat[1], 1ull);
  }
}

__global__ __launch_bounds__(WG) void k_lca_items(const int32_t* __restrict__ parent, int64_t N,
                                                  uint64_t* __restrict__ items) {
  const int64_t v = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (v < N) items[v] = ((uint64_t)(uint32_t)(parent[v] + 1) << 32) | (uint32_t)v;
}

__global__ __launch_bounds__(WG) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t x) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) p[i] = x;
}

// Slot s of the sorted (parent + 1, child) list; slot 0 holds the root
// (key 0), then the children of each node in increasing id.
__global__ __launch_bounds__(WG) void k_lca_links(const uint64_t* __restrict__ sorted, int64_t N,
                                                  int32_t* __restrict__ first_child,
                                                  int32_t* __restrict__ next_sibling) {
  const int64_t s = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (s < 1 || s >= N) return;
  const uint64_t x = sorted[s];
  const uint32_t key = (uint32_t)(x >> 32);
  const int32_t c = (int32_t)(uint32_t)x;
  if ((uint32_t)(sorted[s - 1] >> 32) != key) first_child[key - 1] = c;
  int32_t ns = -1;
  if (s + 1 < N) {
    const uint64_t y = sorted[s + 1];
    if ((uint32_t)(y >> 32) == key) ns = (int32_t)(uint32_t)y;
  }
  next_sibling[c] = ns;
}

__global__ __launch_bounds__(WG) void k_lca_next(const int32_t* __restrict__ parent, int64_t N,
                                                 int32_t root,
                                                 const int32_t* __restrict__ first_child,
                                                 const int32_t* __restrict__ next_sibling,
                                                 int32_t* __restrict__ nxt) {
  const int64_t c = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (c >= N) return;
  if (c == root) {
    nxt[2 * c] = NOT_ARC;
    nxt[2 * c + 1] = NOT_ARC;
    return;
  }
  const int32_t fc = first_child[c], ns = next_sibling[c], p = parent[c];
  nxt[2 * c] = fc >= 0 ? 2 * fc : (int32_t)(2 * c + 1);
  nxt[2 * c + 1] = ns >= 0 ? 2 * ns : (p == root ? END : 2 * p + 1);
}

__device__ __forceinline__ bool sampled(int64_t a, int64_t head) {
  return a == head || (a % SPLIT == 0);
}
__device__ __forceinline__ int64_t sample_id(int64_t a, int64_t head, int64_t S) {
  return a == head ? S : a / SPLIT;
}

// Walk from sample sid (sid < S: arc sid * SPLIT; sid == S: the head) to
// the next sample.  Each arc on the way gets its sample, its count and its
// depth sum within the walk (both exclusive).  A walk is bounded by the
// number of arcs; an overlong one sets stat[1].
__global__ __launch_bounds__(WG) void k_lca_walk(const int32_t* __restrict__ nxt, int64_t NA,
                                                 const int32_t* __restrict__ first_child,
                                                 int32_t root, int64_t S,
                                                 v4i32* __restrict__ arc,
                                                 int32_t* __restrict__ s_next,
                                                 v2i32* __restrict__ s_lw,
                                                 unsigned long long* __restrict__ stat) {
  const int64_t sid = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (sid > S) return;
  const int64_t head = 2 * (int64_t)first_child[root];  // negative: no list (rejected)
  const int64_t a0 = sid == S ? head : sid * SPLIT;
  if (a0 < 0 || a0 >= NA || nxt[a0] == NOT_ARC || (sid < S && a0 == head)) {
    s_lw[sid] = v2i32{-1, 0};  // no walk starts here
    s_next[sid] = END;
    return;
  }
  int64_t a = a0;
  int32_t cnt = 0, w = 0;
  int32_t nx = END;
  bool ended = false;
  for (int64_t guard = 0; guard <= NA; ++guard) {
    // the arc's sample, count and depth sum: one 16-byte store (three 4-byte
    // stores to as many arrays made three scattered writes per arc)
    arc[a] = v4i32{(int32_t)sid, cnt, w, 0};
    cnt += 1;
    w += (a & 1) ? -1 : 1;
    nx = nxt[a];
    if (nx < 0 || nx >= NA || sampled(nx, head)) {
      ended = true;
      break;
    }
    a = nx;
  }
  if (!ended) atomicExch(&stat[1], 1ull);  // longer than the whole list: a cycle
  s_lw[sid] = v2i32{cnt, w};
  s_next[sid] = (nx >= 0 && nx < NA) ? (int32_t)sample_id(nx, head, S) : END;
  atomicAdd(&stat[0], (unsigned long long)cnt);
}

// One round of pointer jumping over the samples: sums (count, depth step)
// from each sample to the end of the list.
__global__ __launch_bounds__(WG) void k_lca_jump(const int32_t* __restrict__ in_next,
                                                 const v2i32* __restrict__ in_lw,
                                                 int32_t* __restrict__ out_next,
                                                 v2i32* __restrict__ out_lw, int64_t S1) {
  const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (j >= S1) return;
  const int32_t nx = in_next[j];
  // (count, depth sum) of a sample as one 8-byte word: one gather per jump
  const v2i32 lw = in_lw[j];
  int32_t len = lw.x, w = lw.y, nn = nx;
  if (len >= 0 && nx >= 0 && nx < S1) {
    const v2i32 o = in_lw[nx];
    len += o.x;
    w += o.y;
    nn = in_next[nx];
  }
  out_next[j] = nn;
  out_lw[j] = v2i32{len, w};
}

// Tour position and depth of every arc; the tour's node and depth arrays,
// first occurrences.  suf: (count, depth sum) from each sample to the end.
__global__ __launch_bounds__(WG) void k_lca_place(const int32_t* __restrict__ parent, int64_t NA,
                                                  int32_t root, int64_t S,
                                                  const v4i32* __restrict__ arc,
                                                  const v2i32* __restrict__ suf,
                                                  const int32_t* __restrict__ nxt,
                                                  int32_t* __restrict__ depth,
                                                  int32_t* __restrict__ node,
                                                  int32_t* __restrict__ first) {
  const int64_t a = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (a == 0) {
    depth[0] = 0;
    node[0] = root;
    first[root] = 0;
  }
  if (a >= NA || nxt[a] == NOT_ARC) return;
  // every arc of the list was walked: the host checked the count before
  // this launch (the sample is still range-checked)
  const v4i32 x = arc[a];
  const int32_t sid = x.x;
  if (sid < 0 || sid > S) return;
  const v2i32 all = suf[S], mine = suf[sid];
  const int64_t pos = (int64_t)all.x - mine.x + x.y + 1;
  const int64_t d = ((int64_t)all.y - mine.y) + x.z + ((a & 1) ? -1 : 1);
  if (pos < 1 || pos > NA - 2) return;
  const int32_t c = (int32_t)(a >> 1);
  depth[pos] = (int32_t)d;
  node[pos] = (a & 1) ? parent[c] : c;
  if (!(a & 1)) first[c] = (int32_t)pos;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

rmq_status status_of(hipError_t e) {
  if (e == hipSuccess) return RMQ_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return RMQ_ERR_OUT_OF_MEMORY;
  return RMQ_ERR_DEVICE;
}

int bits_for(uint64_t x) {
  int b = 1;
  while (b < 32 && (x >> b) != 0) ++b;
  return b;
}

// Builds the tour arrays of h (allocated) from parent; temporaries from one
// allocation, freed before return.
rmq_status build_tour(const int32_t* parent, int64_t N, int32_t root, rmq_lca_s* h,
                      hipStream_t s) {
  const int64_t NA = 2 * N;
  const int64_t S = (NA + SPLIT - 1) / SPLIT;
  const int64_t S1 = S + 1;
  const size_t sort_ws = sort_pairs_workspace_bytes(N);
  size_t off = 0;
  auto take = [&off](size_t b) {
    const size_t at = off;
    off = align256(off + b);
    return at;
  };
  const size_t o_items = take(8 * (size_t)N), o_sorted = take(8 * (size_t)N),
               o_sort = take(sort_ws), o_fc = take(4 * (size_t)N), o_ns = take(4 * (size_t)N),
               o_nxt = take(4 * (size_t)NA), o_arc = take(16 * (size_t)NA),
               o_sa = take(12 * (size_t)S1), o_sb = take(12 * (size_t)S1),
               o_stat = take(4 * 8);
  void* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, off);
  if (e != hipSuccess) return status_of(e);
  char* t = static_cast<char*>(tmp);
  uint64_t* items = reinterpret_cast<uint64_t*>(t + o_items);
  uint64_t* sorted = reinterpret_cast<uint64_t*>(t + o_sorted);
  int32_t* fc = reinterpret_cast<int32_t*>(t + o_fc);
  int32_t* ns = reinterpret_cast<int32_t*>(t + o_ns);
  int32_t* nxt = reinterpret_cast<int32_t*>(t + o_nxt);
  v4i32* arc = reinterpret_cast<v4i32*>(t + o_arc);  // per arc: sample, count, depth sum
  // per sample, ping and pong: (count, depth sum) pairs, then next samples
  struct Samples {
    v2i32* lw;
    int32_t* next;
  };
  const Samples sa{reinterpret_cast<v2i32*>(t + o_sa),
                   reinterpret_cast<int32_t*>(t + o_sa + 8 * (size_t)S1)};
  const Samples sb{reinterpret_cast<v2i32*>(t + o_sb),
                   reinterpret_cast<int32_t*>(t + o_sb + 8 * (size_t)S1)};
  unsigned long long* stat = reinterpret_cast<unsigned long long*>(t + o_stat);

  rmq_status st = RMQ_OK;
  auto run = [&]() -> hipError_t {
    RMQ_TRY(hipMemsetAsync(stat, 0, 4 * 8, s));
    RMQ_TRY(launch(k_lca_items, dim3((unsigned)blocks(N)), dim3(WG), 0, s, parent, N, items));
    RMQ_TRY(launch_sort_pairs(items, N, bits_for((uint64_t)N), sorted, t + o_sort, sort_ws, s));
    {
      // a sort whose bounded look-back wait gave up leaves no usable order:
      // report it before anything reads the list
      uint32_t h_abort = 0;
      RMQ_TRY(hipMemcpyAsync(&h_abort, sort_pairs_abort_word(t + o_sort, N), 4,
                             hipMemcpyDeviceToHost, s));
      RMQ_TRY(hipStreamSynchronize(s));
      if (h_abort) {
        st = RMQ_ERR_DEVICE;
        return hipSuccess;
      }
    }
    RMQ_TRY(launch(k_fill_i32, dim3((unsigned)blocks(N)), dim3(WG), 0, s, fc, N, -1));
    RMQ_TRY(launch(k_fill_i32, dim3((unsigned)blocks(N)), dim3(WG), 0, s, ns, N, -1));
    RMQ_TRY(launch(k_lca_links, dim3((unsigned)blocks(N)), dim3(WG), 0, s, sorted, N, fc, ns));
    RMQ_TRY(launch(k_lca_next, dim3((unsigned)blocks(N)), dim3(WG), 0, s, parent, N, root, fc, ns,
                   nxt));
    RMQ_TRY(launch(k_lca_walk, dim3((unsigned)blocks(S1)), dim3(WG), 0, s, nxt, NA, fc, root, S,
                   arc, sa.next, sa.lw, stat));
    int rounds = 1;
    while ((1ll << rounds) < S1) ++rounds;
    Samples in = sa, outb = sb;
    for (int r = 0; r <= rounds; ++r) {
      RMQ_TRY(launch(k_lca_jump, dim3((unsigned)blocks(S1)), dim3(WG), 0, s, in.next,
                     static_cast<const v2i32*>(in.lw), outb.next, outb.lw, S1));
      const Samples x = in;
      in = outb;
      outb = x;
    }
    // `in` holds the sums to the end; check: the head's sample reaches the
    // end, the walks cover 2(N - 1) arcs and the head's sum is 2(N - 1)
    int32_t head_next = 0, head_len = 0;
    unsigned long long h_stat[2] = {0, 0};
    RMQ_TRY(hipMemcpyAsync(&head_next, in.next + S, 4, hipMemcpyDeviceToHost, s));
    RMQ_TRY(hipMemcpyAsync(&head_len, in.lw + S, 4, hipMemcpyDeviceToHost, s));  // its count
    RMQ_TRY(hipMemcpyAsync(h_stat, stat, 16, hipMemcpyDeviceToHost, s));
    RMQ_TRY(hipStreamSynchronize(s));
    if (head_next != END || h_stat[1] != 0 || (int64_t)h_stat[0] != NA - 2 ||
        (int64_t)head_len != NA - 2) {
      st = RMQ_ERR_INVALID_ARG;  // not one list of 2(N - 1) arcs from the head
      return hipSuccess;
    }
    RMQ_TRY(launch(k_lca_place, dim3((unsigned)blocks(NA)), dim3(WG), 0, s, parent, NA, root, S,
                   arc, static_cast<const v2i32*>(in.lw), nxt, h->depth, h->node, h->first));
    return hipStreamSynchronize(s);
  };
  e = run();
  hipFree(tmp);
  if (e != hipSuccess) return status_of(e);
  return st;
}

}  // namespace

}  // namespace rmq

using namespace rmq;

extern "C" {

rmq_status rmq_lca_build(const int32_t* parent, int64_t num_nodes, const rmq_options* opt,
                         void* stream, rmq_lca* out) {
  if (!parent || !out || num_nodes < 1 || num_nodes > (1ll << 30)) return RMQ_ERR_INVALID_ARG;
  if ((uintptr_t)parent % 4) return RMQ_ERR_MISALIGNED;
  const int64_t N = num_nodes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // 1. one root, parents in range
  unsigned long long* dstat = nullptr;
  hipError_t e = hipMalloc(&dstat, 3 * sizeof(unsigned long long));
  if (e != hipSuccess) return status_of(e);
  unsigned long long hstat[3] = {0, 0, 0};
  e = hipMemsetAsync(dstat, 0, sizeof(hstat), s);
  if (e == hipSuccess)
    e = launch(k_lca_check, dim3((unsigned)blocks(N)), dim3(WG), 0, s, parent, N, dstat);
  if (e == hipSuccess) e = hipMemcpyAsync(hstat, dstat, sizeof(hstat), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(dstat);
  if (e != hipSuccess) return status_of(e);
  if (hstat[0] != 1 || hstat[1] != 0) return RMQ_ERR_INVALID_ARG;
  const int32_t root = (int32_t)hstat[2];

  rmq_lca_s* h = static_cast<rmq_lca_s*>(calloc(1, sizeof(rmq_lca_s)));
  if (!h) return RMQ_ERR_OUT_OF_MEMORY;
  hipGetDevice(&h->device);
  h->N = N;
  h->root = root;
  const int64_t len = 2 * N - 1;
  const size_t o_depth = 0, o_node = align256(4 * (size_t)len),
               o_first = o_node + align256(4 * (size_t)len);
  h->bytes = o_first + align256(4 * (size_t)N);
  e = hipMalloc(&h->mem, h->bytes);
  if (e != hipSuccess) {
    free(h);
    return status_of(e);
  }
  char* m = static_cast<char*>(h->mem);
  h->depth = reinterpret_cast<int32_t*>(m + o_depth);
  h->node = reinterpret_cast<int32_t*>(m + o_node);
  h->first = reinterpret_cast<int32_t*>(m + o_first);

  rmq_status st = RMQ_OK;
  if (N == 1) {
    const int32_t zero = 0;
    e = hipMemcpyAsync(h->depth, &zero, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h->node, &zero, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h->first, &zero, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = status_of(e);
  } else {
    st = build_tour(parent, N, root, h, s);
  }
  // 6. the RMQ index over the depth array
  if (st == RMQ_OK) {
    rmq_options o{};
    if (opt) {
      o.block_size = opt->block_size;
      o.sub_block_size = opt->sub_block_size;
      o.table_arity_log2 = opt->table_arity_log2;
      o.no_query_records = opt->no_query_records;
    }
    st = rmq_build(h->depth, len, &o, stream, &h->idx);
  }
  if (st != RMQ_OK) {
    hipFree(h->mem);
    free(h);
    return st;
  }
  *out = h;
  return RMQ_OK;
}

rmq_status rmq_lca_query(rmq_lca h, const int32_t* u, const int32_t* v, int64_t q, int32_t* out,
                         void* stream, const rmq_options* opt) {
  if (!h || q < 0 || q > RMQ_MAX_Q) return RMQ_ERR_INVALID_ARG;
  if (q == 0) return RMQ_OK;
  if (!u || !v || !out) return RMQ_ERR_INVALID_ARG;
  if ((uintptr_t)u % 4 || (uintptr_t)v % 4 || (uintptr_t)out % 4) return RMQ_ERR_MISALIGNED;
  const rmq_index_s* ix = h->idx;
  return status_of(launch_query_lca(h->depth, ix->n, ix->kshift, ix->st, ix->nb, ix->sub,
                                    ix->k1shift, h->first, h->node, h->N, u, v, q, out,
                                    opt ? opt->bad_count : nullptr,
                                    static_cast<hipStream_t>(stream), ix->lg, ix->rec,
                                    ix->levels));
}

rmq_status rmq_lca_copy_tour(rmq_lca h, int32_t* depth, int32_t* node, int32_t* first,
                             void* stream) {
  if (!h) return RMQ_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t len = 4 * (size_t)(2 * h->N - 1);
  hipError_t e = hipSuccess;
  if (depth) e = hipMemcpyAsync(depth, h->depth, len, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && node) e = hipMemcpyAsync(node, h->node, len, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && first)
    e = hipMemcpyAsync(first, h->first, 4 * (size_t)h->N, hipMemcpyDeviceToDevice, s);
  return status_of(e);
}

rmq_status rmq_lca_info(rmq_lca h, int64_t* num_nodes, size_t* bytes) {
  if (!h) return RMQ_ERR_INVALID_ARG;
  if (num_nodes) *num_nodes = h->N;
  if (bytes) *bytes = h->bytes + h->idx->bytes;
  return RMQ_OK;
}

rmq_status rmq_lca_free(rmq_lca h) {
  if (!h) return RMQ_ERR_INVALID_ARG;
  rmq_status st = rmq_index_free(h->idx);
  hipError_t e = hipFree(h->mem);
  free(h);
  return st != RMQ_OK ? st : status_of(e);
}

}  // extern "C"
