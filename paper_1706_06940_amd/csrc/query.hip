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
  // min key over A[lo..hi], whole wave cooperating (lo, hi wave-uniform).
  __device__ uint64_t scan(int64_t lo, int64_t hi, int lane, bool aligned) const {
    uint64_t best = KEY_NONE;
    if (aligned) {
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
  __device__ uint64_t scan(int64_t lo, int64_t hi, int lane, bool aligned) const {
    uint64_t best = KEY_NONE;
    if (aligned) {
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

// --- the kernel --------------------------------------------------------------
// L, R: the queries' positions in A (validated here).  For the contracted
// path, LI/RI hold their contracted index ranges; for the plain path LI == L
// and RI == R.  src_len: number of source entries (n or 2q - 1).
template <class Src>
__global__ __launch_bounds__(WG) void k_query(Src src, int64_t src_len, int64_t n, int kshift,
                                              const uint64_t* __restrict__ st, int64_t nb,
                                              const int32_t* __restrict__ L,
                                              const int32_t* __restrict__ R,
                                              const int32_t* __restrict__ LI,
                                              const int32_t* __restrict__ RI, int64_t q,
                                              int32_t* __restrict__ out,
                                              unsigned long long* __restrict__ bad_count,
                                              unsigned long long* __restrict__ stats,
                                              bool aligned) {
  const int lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = i < q;

  int64_t l = 0, r = -1, li = 0, ri = -1;
  if (live) {
    l = L[i];
    r = R[i];
    li = LI[i];
    ri = RI[i];
  }
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
    const uint64_t m = src.scan(lo, hi, lane, aligned);
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
    const uint64_t m = src.scan(lo, hi, lane, aligned);
    if (lane == src_lane) best = umin64(best, m);
    n_scans += 1;
    n_elems += (uint64_t)(hi - lo + 1);
  }

  if (live) out[i] = ok ? (int32_t)src.pos_of(best) : -1;

  if (bad_count) {
    const uint64_t bad = ballot(live && !ok);
    if (bad && lane == 0) atomicAdd(bad_count, (unsigned long long)__popcll(bad));
  }
  if (stats && n_scans && lane == 0) {
    atomicAdd(stats, (unsigned long long)n_scans);
    atomicAdd(stats + 1, (unsigned long long)n_elems);
  }
}

}  // namespace

hipError_t launch_query_full(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                             int64_t nb, const int32_t* L, const int32_t* R, int64_t q,
                             int32_t* out, int64_t* bad_count, uint64_t* stats,
                             hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t grid = (q + WG - 1) / WG;
  const bool aligned = ((uintptr_t)A & 15) == 0;
  hipLaunchKernelGGL(k_query<SrcA>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcA{A, n}, n, n,
                     kshift, st, nb, L, R, L, R, q, out, (unsigned long long*)bad_count,
                     (unsigned long long*)stats, aligned);
  return hipGetLastError();
}

hipError_t launch_query_contracted(const uint64_t* aq, int64_t m, int64_t n, int kshift,
                                   const uint64_t* st, int64_t nb, const int32_t* L,
                                   const int32_t* R, const int32_t* Lc, const int32_t* Rc,
                                   int64_t q, int32_t* out, int64_t* bad_count, uint64_t* stats,
                                   hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t grid = (q + WG - 1) / WG;
  const bool aligned = ((uintptr_t)aq & 15) == 0;
  hipLaunchKernelGGL(k_query<SrcKeys>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcKeys{aq, m}, m,
                     n, kshift, st, nb, L, R, Lc, Rc, q, out, (unsigned long long*)bad_count,
                     (unsigned long long*)stats, aligned);
  return hipGetLastError();
}

}  // namespace rmq
