// Query answering on a block Sparse Table (Section 3.1 step 4; Section 3.2
// second stage), with the partial-block scans done cooperatively by the wave.
//
// One lane per query.  For a query over index range [li, ri] of the source
// (A itself, or A_Q for the contracted path), with end blocks bl = li/k and
// br = ri/k:
//   * inner span: m' = min of the two overlapping 2^t-block windows that cover
//     blocks bl+1 .. br-1, t = floor(log2(br - bl - 1)) (none if br - bl < 2);
//   * speculative reads of the two end-block minima kl, kr:
//       - if the block minimum lies inside the query, it is the exact minimum
//         of that partial block;
//       - else if it is not below the best known so far, the partial block
//         cannot hold the answer and is skipped;
//       - else the partial block must be scanned;
//   * a query inside one block uses that block's minimum if it lies inside
//     the query, else scans the query range.
// Keys are unique, so every comparison above is exact and the answer is the
// leftmost minimum.  Scans are rare for uniform queries; instead of diverging
// one lane at a time they are queued per wave (ballot) and each queued range
// is read by all 64 lanes with coalesced 16-byte loads and a DPP min.  Left
// scans run first, and a pending right scan is re-checked against the best
// key after them.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;

// --- sources -----------------------------------------------------------------
// The plain array: index == position in A, key built from the int32 value.
struct SrcA {
  const int32_t* __restrict__ A;
  int64_t len;
  __device__ __forceinline__ uint32_t pos_of(uint64_t key) const { return key_pos(key); }
  // A[p..p+3] for 4-aligned p <= hi; entries past the array read as INT32_MAX
  // (the caller masks positions outside [lo, hi]).
  __device__ __forceinline__ v4i32 load4(int64_t p, int64_t hi) const {
    v4i32 x = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    if (p + 3 < len) {
      if (p <= hi) x = *reinterpret_cast<const v4i32*>(A + p);
    } else {
      for (int c = 0; c < 4; ++c)
        if (p + c < len && p + c <= hi) x[c] = A[p + c];
    }
    return x;
  }
  // This lane's source as seen by the whole wave (for a wave-wide scan).
  __device__ __forceinline__ SrcA broadcast(int src_lane) const {
    return {reinterpret_cast<const int32_t*>(readlane64((int64_t)(uintptr_t)A, src_lane)),
            readlane64(len, src_lane)};
  }
  // min key over A[lo..hi], whole wave cooperating (everything wave-uniform).
  __device__ uint64_t scan(int64_t lo, int64_t hi, int lane) const {
    uint64_t best = KEY_NONE;
    if (((uintptr_t)A & 15) == 0) {
      const int64_t a0 = lo & ~3ll;
      for (int64_t base = a0; base <= hi; base += 512) {
        const int64_t p0 = base + lane * 4, p1 = p0 + 256;
        v4i32 x0 = load4(p0, hi), x1 = load4(p1, hi);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t q0 = p0 + c, q1 = p1 + c;
          if (p0 <= hi && q0 >= lo && q0 <= hi) best = umin64(best, make_key(x0[c], (uint32_t)q0));
          if (p1 <= hi && q1 >= lo && q1 <= hi) best = umin64(best, make_key(x1[c], (uint32_t)q1));
        }
      }
    } else {
      for (int64_t p = lo + lane; p <= hi; p += 64) best = umin64(best, make_key(A[p], (uint32_t)p));
    }
    return wave_min_u64(best);
  }
};

// The contracted array A_Q: entries are already keys whose low half is the
// position in A.
struct SrcKeys {
  const uint64_t* __restrict__ S;
  int64_t len;
  __device__ __forceinline__ v2u64 load2(int64_t p, int64_t hi) const {
    v2u64 x = {KEY_NONE, KEY_NONE};
    if (p + 1 < len) {
      if (p <= hi) x = *reinterpret_cast<const v2u64*>(S + p);
    } else if (p < len && p <= hi) {
      x[0] = S[p];
    }
    return x;
  }
  __device__ __forceinline__ uint32_t pos_of(uint64_t key) const { return key_pos(key); }
  __device__ __forceinline__ SrcKeys broadcast(int src_lane) const {
    return {reinterpret_cast<const uint64_t*>(readlane64((int64_t)(uintptr_t)S, src_lane)),
            readlane64(len, src_lane)};
  }
  __device__ uint64_t scan(int64_t lo, int64_t hi, int lane) const {
    uint64_t best = KEY_NONE;
    if (((uintptr_t)S & 15) == 0) {
      const int64_t a0 = lo & ~1ll;
      for (int64_t base = a0; base <= hi; base += 256) {
        const int64_t p0 = base + lane * 2, p1 = p0 + 128;
        v2u64 x0 = load2(p0, hi), x1 = load2(p1, hi);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int64_t q0 = p0 + c, q1 = p1 + c;
          if (p0 <= hi && q0 >= lo && q0 <= hi) best = umin64(best, x0[c]);
          if (p1 <= hi && q1 >= lo && q1 <= hi) best = umin64(best, x1[c]);
        }
      }
    } else {
      for (int64_t p = lo + lane; p <= hi; p += 64) best = umin64(best, S[p]);
    }
    return wave_min_u64(best);
  }
};

// --- the query step ----------------------------------------------------------
// One lane's query [l, r] (positions in A, validated here) over source
// entries [li, ri] of its table (st: level-major, nb blocks of 2^kshift
// entries).  All 64 lanes of the wave must call this together: the partial
// scans are done by the whole wave.  Lanes may belong to different tables
// (batched launches); `live` is false for padding lanes.
template <class Src>
__device__ __forceinline__ void query_core(const Src& src, int64_t src_len, int64_t n,
                                           int kshift, const uint64_t* __restrict__ st,
                                           int64_t nb, int64_t l, int64_t r, int64_t li,
                                           int64_t ri, bool live, int32_t* outp,
                                           unsigned long long* __restrict__ bad_count,
                                           unsigned long long* __restrict__ stats) {
  const int lane = lane_id();
  const bool ok = live && 0 <= l && l <= r && r < n && 0 <= li && li <= ri && ri < src_len;

  uint64_t best = KEY_NONE, kr = KEY_NONE;
  bool needL = false, needR = false;
  int64_t loL = 0, hiL = -1, loR = 0, hiR = -1;

  if (ok) {
    const int64_t bl = li >> kshift, br = ri >> kshift;
    const uint64_t kl = st[bl];
    if (bl == br) {
      const int64_t p = src.pos_of(kl);
      if (l <= p && p <= r) {
        best = kl;
      } else {
        needL = true;
        loL = li;
        hiL = ri;
      }
    } else {
      const int64_t inner = br - bl - 1;
      if (inner > 0) {
        const int t = ilog2_u64((uint64_t)inner);
        const uint64_t* lev = st + (size_t)t * nb;
        best = umin64(lev[bl + 1], lev[br - (1ll << t)]);
      }
      kr = st[br];
      if ((int64_t)src.pos_of(kl) >= l) {
        best = umin64(best, kl);
      } else if (kl < best) {
        needL = true;
        loL = li;
        hiL = ((bl + 1) << kshift) - 1;
      }
      if ((int64_t)src.pos_of(kr) <= r) {
        best = umin64(best, kr);
      } else if (kr < best) {
        needR = true;
        loR = br << kshift;
        hiR = ri;
      }
    }
  }

  // ---- wave-cooperative partial-block scans ----
  uint64_t n_scans = 0, n_elems = 0;
  uint64_t pend = ballot(needL);
  while (pend) {
    const int src_lane = __builtin_ctzll(pend);
    pend &= pend - 1;
    const int64_t lo = readlane64(loL, src_lane), hi = readlane64(hiL, src_lane);
    const uint64_t m = src.broadcast(src_lane).scan(lo, hi, lane);
    if (lane == src_lane) best = umin64(best, m);
    n_scans += 1;
    n_elems += (uint64_t)(hi - lo + 1);
  }
  if (needR && !(kr < best)) needR = false;  // the left scan already beat this block
  pend = ballot(needR);
  while (pend) {
    const int src_lane = __builtin_ctzll(pend);
    pend &= pend - 1;
    const int64_t lo = readlane64(loR, src_lane), hi = readlane64(hiR, src_lane);
    const uint64_t m = src.broadcast(src_lane).scan(lo, hi, lane);
    if (lane == src_lane) best = umin64(best, m);
    n_scans += 1;
    n_elems += (uint64_t)(hi - lo + 1);
  }

  if (live) *outp = ok ? (int32_t)src.pos_of(best) : -1;

  if (bad_count) {
    const uint64_t bad = ballot(live && !ok);
    if (bad && lane == 0) atomicAdd(bad_count, (unsigned long long)__popcll(bad));
  }
  if (stats && n_scans && lane == 0) {
    atomicAdd(stats, (unsigned long long)n_scans);
    atomicAdd(stats + 1, (unsigned long long)n_elems);
  }
}

// One table.  L, R: the queries' positions in A.  For the contracted path, LR
// holds their contracted index ranges as interleaved pairs (LR[2i],
// LR[2i+1]); for the plain path LR is null and the ranges are [L[i], R[i]]
// themselves.  src_len: number of source entries (n or 2q - 1).
template <class Src>
__global__ __launch_bounds__(WG) void k_query(Src src, int64_t src_len, int64_t n, int kshift,
                                              const uint64_t* __restrict__ st, int64_t nb,
                                              const int32_t* __restrict__ L,
                                              const int32_t* __restrict__ R,
                                              const int32_t* __restrict__ LR, int64_t q,
                                              int32_t* __restrict__ out,
                                              unsigned long long* __restrict__ bad_count,
                                              unsigned long long* __restrict__ stats) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = i < q;
  int64_t l = 0, r = -1, li = 0, ri = -1;
  if (live) {
    l = L[i];
    r = R[i];
    if (LR) {
      const int2 c = reinterpret_cast<const int2*>(LR)[i];
      li = c.x;
      ri = c.y;
    } else {
      li = l;
      ri = r;
    }
  }
  query_core(src, src_len, n, kshift, st, nb, l, r, li, ri, live, out + (live ? i : 0),
             bad_count, stats);
}

// Every query of a batch of tables (plain path): global query g belongs to
// the table whose range of the concatenated query list holds it.
__global__ __launch_bounds__(WG) void k_query_multi(const ArrayDesc* __restrict__ items,
                                                    const int64_t* __restrict__ q_prefix,
                                                    int count,
                                                    unsigned long long* __restrict__ bad_count,
                                                    unsigned long long* __restrict__ stats) {
  const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = g < q_prefix[count];
  const int j = live ? find_item(q_prefix, count, g) : 0;
  const ArrayDesc& d = items[j];
  const int64_t i = live ? g - q_prefix[j] : 0;
  int64_t l = 0, r = -1;
  if (live) {
    l = d.L[i];
    r = d.R[i];
  }
  query_core(SrcA{d.A, d.n}, d.n, d.n, d.kshift, d.st, d.nb, l, r, l, r, live, d.out + i,
             bad_count, stats);
}

// A coalesced batch of requests (serving): queries g in
// [seg_prefix[s], seg_prefix[s+1]) belong to request s, which targets the
// resident table tables[seg_table[s]].
__global__ __launch_bounds__(WG) void k_query_segments(const ArrayDesc* __restrict__ tables,
                                                       const int64_t* __restrict__ seg_prefix,
                                                       const int32_t* __restrict__ seg_table,
                                                       int nseg, const int32_t* __restrict__ L,
                                                       const int32_t* __restrict__ R,
                                                       int32_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = g < seg_prefix[nseg];
  const int sg = live ? find_item(seg_prefix, nseg, g) : 0;
  const ArrayDesc& d = tables[seg_table[sg]];
  int64_t l = 0, r = -1;
  if (live) {
    l = L[g];
    r = R[g];
  }
  query_core(SrcA{d.A, d.n}, d.n, d.n, d.kshift, d.st, d.nb, l, r, l, r, live,
             out + (live ? g : 0), nullptr, nullptr);
}

}  // namespace

hipError_t launch_query_segments(const ArrayDesc* tables, const int64_t* seg_prefix,
                                 const int32_t* seg_table, int nseg, const int32_t* L,
                                 const int32_t* R, int32_t* out, int64_t total,
                                 hipStream_t stream) {
  if (total <= 0) return hipSuccess;
  const int64_t grid = (total + WG - 1) / WG;
  RMQ_TRY(launch(k_query_segments, dim3((unsigned)grid), dim3(WG), 0, stream, tables, seg_prefix,
                 seg_table, nseg, L, R, out));
  return hipSuccess;
}

hipError_t launch_query_full(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                             int64_t nb, const int32_t* L, const int32_t* R, int64_t q,
                             int32_t* out, int64_t* bad_count, uint64_t* stats,
                             hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t grid = (q + WG - 1) / WG;
  RMQ_TRY(launch(k_query<SrcA>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcA{A, n}, n, n,
                 kshift, st, nb, L, R, static_cast<const int32_t*>(nullptr), q, out,
                 (unsigned long long*)bad_count, (unsigned long long*)stats));
  return hipGetLastError();
}

hipError_t launch_query_contracted(const uint64_t* aq, int64_t m, int64_t n, int kshift,
                                   const uint64_t* st, int64_t nb, const int32_t* L,
                                   const int32_t* R, const int32_t* LR, int64_t q, int32_t* out,
                                   int64_t* bad_count, uint64_t* stats, hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t grid = (q + WG - 1) / WG;
  RMQ_TRY(launch(k_query<SrcKeys>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcKeys{aq, m}, m,
                 n, kshift, st, nb, L, R, LR, q, out, (unsigned long long*)bad_count,
                 (unsigned long long*)stats));
  return hipGetLastError();
}

hipError_t launch_query_multi(const ArrayDesc* items, const int64_t* q_prefix, int count,
                              int64_t total_q, int64_t* bad_count, uint64_t* stats,
                              hipStream_t stream) {
  if (total_q <= 0) return hipSuccess;
  const int64_t grid = (total_q + WG - 1) / WG;
  RMQ_TRY(launch(k_query_multi, dim3((unsigned)grid), dim3(WG), 0, stream, items, q_prefix, count,
                 (unsigned long long*)bad_count, (unsigned long long*)stats));
  return hipSuccess;
}

}  // namespace rmq
