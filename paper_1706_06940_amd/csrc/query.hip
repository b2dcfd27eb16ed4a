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
// On sources that allow it (two block levels), when at least LANE_SCAN_MIN
// lanes of a wave need a partial scan, those whose range reads at most
// LANE_SCAN_MAX entries read it alone, all at once; the others are queued and
// read by the whole wave one range at a time (a step covers 512 elements, so
// a lone scan finishes fast).
constexpr int LANE_SCAN_MIN = 16;
constexpr int64_t LANE_SCAN_MAX = 1024;

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
  // Whole ranges are not scanned lane by lane on this source: one lane's
  // loads touch 64 different lines per instruction, so queued wave-wide
  // scans (8 lines per load) are faster even when every lane has a range.
  static constexpr bool kLaneScans = false;
  // min key over A[lo..hi] by this lane alone (a short piece); 16 elements
  // per step, their loads in flight together.
  __device__ uint64_t lane_scan(int64_t lo, int64_t hi, uint64_t bound, int64_t& reads) const {
    reads += hi - lo + 1;
    uint64_t best = KEY_NONE;
    if (((uintptr_t)A & 15) == 0) {
      for (int64_t p = lo & ~3ll; p <= hi; p += 16) {
        v4i32 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = load4(p + 4 * u, hi);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int64_t e = p + 4 * u + c;
            if (e >= lo && e <= hi) best = umin64(best, make_key(x[u][c], (uint32_t)e));
          }
      }
    } else {
      for (int64_t e = lo; e <= hi; ++e) best = umin64(best, make_key(A[e], (uint32_t)e));
    }
    return best;
  }
  // Queued pieces are read several at a time, each by a group of G lanes
  // (grouped_scans); an entry is 4 bytes.
  static constexpr bool kGroupScans = true;
  static constexpr bool kNested = false;
  static constexpr int kEntryShift = 2;
  // This lane's share of the min key over A[lo..hi] when G lanes read it
  // together: four 16-byte loads per lane in flight, 16 G elements a pass
  // (positions fit 32 bits: n < 2^31).
  template <int G>
  __device__ uint64_t group_part(uint32_t lo, uint32_t hi, int gl) const {
    uint64_t best = KEY_NONE;
    if (((uintptr_t)A & 15) == 0) {
      for (uint32_t base = lo & ~3u; base <= hi; base += 16 * G) {
        v4i32 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = load4(base + (uint32_t)(u * G + gl) * 4, hi);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t e = base + (uint32_t)(u * G + gl) * 4 + c;
            if (e >= lo && e <= hi) best = umin64(best, make_key(x[u][c], e));
          }
      }
    } else {
      for (uint32_t e = lo + gl; e <= hi; e += G) best = umin64(best, make_key(A[e], e));
    }
    return best;
  }
  // lane src_lane's source, per lane (lanes may take different sources)
  __device__ __forceinline__ SrcA gather(int src_lane) const {
    return {reinterpret_cast<const int32_t*>(__shfl((long long)(uintptr_t)A, src_lane)),
            (int64_t)__shfl((long long)len, src_lane)};
  }
  // This lane's source as seen by the whole wave (for a wave-wide scan).
  static constexpr bool kIndexIsPos = true;  // entry index = position in A
  // the source bound to one query's range in A (used by two-level sources)
  __device__ __forceinline__ SrcA with_query(int64_t, int64_t) const { return *this; }
  __device__ __forceinline__ SrcA broadcast(int src_lane) const {
    return {reinterpret_cast<const int32_t*>(readlane64((int64_t)(uintptr_t)A, src_lane)),
            readlane64(len, src_lane)};
  }
  // min key over A[lo..hi], whole wave cooperating (everything wave-uniform).
  // `bound` (the query's best key so far) is not needed here; `reads` counts
  // the entries read.
  __device__ uint64_t scan(int64_t lo, int64_t hi, int lane, uint64_t bound,
                           int64_t& reads) const {
    reads += hi - lo + 1;
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
  static constexpr bool kLaneScans = false;  // as for the plain array
  // min key over S[lo..hi] by this lane alone (a short piece under two block
  // levels); 8 entries per step, their loads in flight together
  __device__ uint64_t lane_scan(int64_t lo, int64_t hi, uint64_t bound, int64_t& reads) const {
    reads += hi - lo + 1;
    uint64_t best = KEY_NONE;
    for (int64_t p = lo; p <= hi; p += 8) {
      uint64_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = p + u <= hi ? S[p + u] : KEY_NONE;
#pragma unroll
      for (int u = 0; u < 8; ++u) best = umin64(best, x[u]);
    }
    return best;
  }
  static constexpr bool kGroupScans = true;  // as for the plain array; 8-byte entries
  static constexpr bool kNested = false;
  static constexpr int kEntryShift = 3;
  // This lane's share of the min over S[lo..hi] when G lanes read it
  // together: four 16-byte loads per lane in flight, 8 G entries a pass
  // (indices fit 32 bits: A_Q has fewer than 2^31 entries).
  template <int G>
  __device__ uint64_t group_part(uint32_t lo, uint32_t hi, int gl) const {
    uint64_t best = KEY_NONE;
    if (((uintptr_t)S & 15) == 0) {
      for (uint32_t base = lo & ~1u; base <= hi; base += 8 * G) {
        v2u64 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = load2(base + (uint32_t)(u * G + gl) * 2, hi);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const uint32_t e = base + (uint32_t)(u * G + gl) * 2 + c;
            if (e >= lo && e <= hi) best = umin64(best, x[u][c]);
          }
      }
    } else {
      for (uint32_t e = lo + gl; e <= hi; e += G) best = umin64(best, S[e]);
    }
    return best;
  }
  __device__ __forceinline__ SrcKeys gather(int src_lane) const {
    return {reinterpret_cast<const uint64_t*>(__shfl((long long)(uintptr_t)S, src_lane)),
            (int64_t)__shfl((long long)len, src_lane)};
  }
  static constexpr bool kIndexIsPos = false;  // keys carry positions in A
  __device__ __forceinline__ SrcKeys with_query(int64_t, int64_t) const { return *this; }
  __device__ __forceinline__ SrcKeys broadcast(int src_lane) const {
    return {reinterpret_cast<const uint64_t*>(readlane64((int64_t)(uintptr_t)S, src_lane)),
            readlane64(len, src_lane)};
  }
  __device__ uint64_t scan(int64_t lo, int64_t hi, int lane, uint64_t bound,
                           int64_t& reads) const {
    reads += hi - lo + 1;
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

// An array with two block levels (Section 3.3): the minima of its k1-blocks
// are kept, so a partial k-block [lo, hi] is read as the k1-block minima of
// the k1-blocks it covers plus at most two partial k1-blocks, and those again
// only when their k1-block minimum can still beat the query's best key (the
// same speculation as at the upper level).  Inner: the plain array A (SrcA)
// or the contracted A_Q (SrcKeys).
//
// Whether a k1-block's minimum lies inside a piece: over A, by the piece's
// bounds; over A_Q, whose keys carry positions in A, in A: every piece read
// here is the query's part of one k1-block, and the block's minimum lies in
// the block, so it lies in the piece exactly when its position in A lies in
// the query's range [ql, qr].
template <class Inner>
struct Src2 {
  Inner a;
  const uint64_t* __restrict__ sub;  // k1-block minima
  int64_t nsub;
  int s1;            // k1 = 2^s1
  int64_t ql = 0;    // the query's range in A (with_query)
  int64_t qr = -1;
  __device__ __forceinline__ uint32_t pos_of(uint64_t key) const { return key_pos(key); }
  __device__ __forceinline__ Src2 with_query(int64_t l, int64_t r) const {
    if constexpr (Inner::kIndexIsPos) return *this;  // the piece's own bounds serve
    Src2 c = *this;
    c.ql = l;
    c.qr = r;
    return c;
  }
  // whether position p (of a k1-block's minimum) lies in the piece lo..hi
  __device__ __forceinline__ bool inside(int64_t p, int64_t lo, int64_t hi) const {
    if constexpr (Inner::kIndexIsPos) return lo <= p && p <= hi;
    return ql <= p && p <= qr;
  }
  __device__ __forceinline__ Src2 broadcast(int src_lane) const {
    Src2 c{a.broadcast(src_lane),
           reinterpret_cast<const uint64_t*>(readlane64((int64_t)(uintptr_t)sub, src_lane)),
           readlane64(nsub, src_lane), __builtin_amdgcn_readlane(s1, src_lane)};
    if constexpr (!Inner::kIndexIsPos) {
      c.ql = readlane64(ql, src_lane);
      c.qr = readlane64(qr, src_lane);
    }
    return c;
  }
  // min over the entries lo..hi, which lie in one k1-block: its minimum if
  // that lies inside, nothing if it cannot beat `bound`, else a scan of the
  // entries
  __device__ __forceinline__ uint64_t part(int64_t lo, int64_t hi, int lane, uint64_t bound,
                           int64_t& reads) const {
    const uint64_t kb = sub[lo >> s1];
    reads += 1;
    const int64_t p = (int64_t)key_pos(kb);
    if (inside(p, lo, hi)) return kb;
    if (!(kb < bound)) return KEY_NONE;
    return a.scan(lo, hi, lane, bound, reads);
  }
  // Dense short ranges are read lane by lane here: the lane reads k1-block
  // minima and at most two pieces of at most k1 elements (only while k1 <=
  // 256: longer pieces read by one lane cost more than wave-wide scans).
  static constexpr bool kLaneScans = true;
  static constexpr bool kGroupScans = false;  // its pieces are read in two steps
  // as an inner source itself (three block levels, Src2<Src2<SrcA>>): entry
  // indices are its inner source's
  static constexpr bool kIndexIsPos = Inner::kIndexIsPos;
  // Entries one lane reads for a piece of `elems` entries inside one block
  // of this level (as the inner source of a third level).
  static constexpr bool kNested = true;
  __device__ __forceinline__ int64_t piece_cost(int64_t elems) const {
    const int64_t k1 = 1ll << s1;
    const int64_t inner = elems < k1 ? elems : k1;
    return (elems >> s1) + 2 + 2 * inner;
  }
  __device__ __forceinline__ int64_t lane_cost(int64_t lo, int64_t hi) const {
    const int64_t elems = hi - lo + 1, k1 = 1ll << s1;
    if constexpr (Inner::kNested) {
      // three levels: a partial k1-block costs its k2-block minima and two
      // partial k2-blocks
      const int64_t piece = a.piece_cost(elems < k1 ? elems : k1);
      return (hi >> s1) - (lo >> s1) + 1 + 2 * piece;
    }
    if (s1 > 8) return INT64_MAX;
    const int64_t two = 2ll << s1;
    return (hi >> s1) - (lo >> s1) + 1 + (elems < two ? elems : two);
  }
  // the same decomposition by this lane alone (short ranges): k1-blocks
  // b_lo+1 .. b_hi-1 whole, then the pieces of b_lo and b_hi in the range
  // (a whole k1-block's minimum always lies inside, so it needs no scan)
  __device__ __forceinline__ uint64_t lane_scan(int64_t lo, int64_t hi, uint64_t bound, int64_t& reads) const {
    const int64_t b_lo = lo >> s1, b_hi = hi >> s1;
    const int64_t k1 = 1ll << s1;
    const uint64_t kh = sub[b_lo], kt = sub[b_hi];  // both loads in flight
    uint64_t best = KEY_NONE;
    for (int64_t b = b_lo + 1; b < b_hi; ++b) best = umin64(best, sub[b]);
    reads += b_hi - b_lo + 1;
    auto piece = [&](uint64_t kb, int64_t p_lo, int64_t p_hi) {
      const int64_t p = (int64_t)key_pos(kb);
      if (inside(p, p_lo, p_hi)) best = umin64(best, kb);
      else if (kb < umin64(best, bound))
        best = umin64(best, a.lane_scan(p_lo, p_hi, bound, reads));
    };
    piece(kh, lo, b_lo == b_hi ? hi : (b_lo + 1) * k1 - 1);
    if (b_hi != b_lo) piece(kt, b_hi * k1, hi);
    return best;
  }
  __device__ __forceinline__ uint64_t scan(int64_t lo, int64_t hi, int lane, uint64_t bound,
                           int64_t& reads) const {
    const int64_t b_lo = lo >> s1, b_hi = hi >> s1;
    if (b_lo == b_hi) return part(lo, hi, lane, bound, reads);
    const int64_t k1 = 1ll << s1;
    // whole k1-blocks inside [lo, hi]
    const int64_t f = (lo & (k1 - 1)) == 0 ? b_lo : b_lo + 1;
    const int64_t g = ((hi + 1) & (k1 - 1)) == 0 ? b_hi : b_hi - 1;
    uint64_t best = KEY_NONE;
    for (int64_t b = f + lane; b <= g; b += 64) best = umin64(best, sub[b]);
    best = wave_min_u64(best);
    reads += g >= f ? g - f + 1 : 0;
    if (f != b_lo)
      best = umin64(best, part(lo, (b_lo + 1) * k1 - 1, lane, umin64(best, bound), reads));
    if (g != b_hi) best = umin64(best, part(b_hi * k1, hi, lane, umin64(best, bound), reads));
    return best;
  }
};
using SrcA2 = Src2<SrcA>;
using SrcKeys2 = Src2<SrcKeys>;
// Three block levels (Section 3.3 with h = 3): the k1-block minima over the
// k2-block minima over A.
using SrcA3 = Src2<SrcA2>;

// --- the query step ----------------------------------------------------------
// The queued partial-block pieces of a wave (pl: lanes with a left piece
// [loL, hiL], pr: with a right piece [loR, hiR]) read 64 / G at a time: group
// g (lanes gG .. gG + G - 1) reads the g-th queued piece, then the group's
// minimum goes to the lane that queued it.  One round of loads serves up to
// 64 / G pieces where a wave-wide scan serves one (G = 16 or 32: pieces of at
// most 1 or 2 KB).
template <int G, class Src>
__device__ __forceinline__ void grouped_scans(const Src& src, uint64_t pl, uint64_t pr,
                                              uint32_t loL, uint32_t hiL, uint32_t loR,
                                              uint32_t hiR, int lane, uint64_t& best,
                                              uint64_t& n_scans, uint64_t& n_elems) {
  constexpr int S = 64 / G;
  const int gi = lane / G, gl = lane % G;
  while (pl | pr) {
    int who[S];
    bool right[S];
#pragma unroll
    for (int g = 0; g < S; ++g) {
      who[g] = -1;
      right[g] = false;
      if (pl) {
        who[g] = __builtin_ctzll(pl);
        pl &= pl - 1;
      } else if (pr) {
        who[g] = __builtin_ctzll(pr);
        pr &= pr - 1;
        right[g] = true;
      }
    }
    int mine = who[0];
    bool mr = right[0];
#pragma unroll
    for (int g = 1; g < S; ++g)
      if (gi == g) {
        mine = who[g];
        mr = right[g];
      }
    const int sl = mine < 0 ? lane : mine;
    const uint32_t l_lo = (uint32_t)__shfl((int)loL, sl), l_hi = (uint32_t)__shfl((int)hiL, sl);
    const uint32_t r_lo = (uint32_t)__shfl((int)loR, sl), r_hi = (uint32_t)__shfl((int)hiR, sl);
    uint32_t lo = mr ? r_lo : l_lo, hi = mr ? r_hi : l_hi;
    if (mine < 0) {  // no piece for this group: a range no pass enters
      lo = 4;
      hi = 0;
    }
    uint64_t m = src.gather(sl).template group_part<G>(lo, hi, gl);
    m = group_min_u64<G>(m);
#pragma unroll
    for (int g = 0; g < S; ++g) {
      if (who[g] < 0) break;
      const uint64_t r = (uint64_t)readlane64((int64_t)m, g * G + G - 1);
      if (lane == who[g]) best = umin64(best, r);
      n_scans += 1;
      n_elems += (uint32_t)__builtin_amdgcn_readlane((int)(hi - lo + 1), g * G);
    }
  }
}

// The end-block step of one lane's query: validity, the inner windows'
// minimum, both end blocks' keys with the speculation of Section 3.1 step 4,
// and the partial pieces still to read (queued below).
struct EndState {
  uint64_t best, kr;
  int64_t loL, hiL, loR, hiR;
  bool ok, needL, needR;
};
template <class Src, class TablePtr = const uint64_t*>
__device__ __forceinline__ EndState query_ends(const Src& src, int64_t src_len, int64_t n,
                                               int kshift, TablePtr __restrict__ st, int64_t nb,
                                               int64_t l, int64_t r, int64_t li, int64_t ri,
                                               bool live, int lg = 1,
                                               const uint64_t* __restrict__ rec = nullptr,
                                               int rlev = 0) {
  const bool ok = live && 0 <= l && l <= r && r < n && 0 <= li && li <= ri && ri < src_len;

  uint64_t best = KEY_NONE, kr = KEY_NONE;
  bool needL = false, needR = false;
  int64_t loL = 0, hiL = -1, loR = 0, hiR = -1;

  if (ok) {
    const int64_t bl = li >> kshift, br = ri >> kshift;
    const int64_t inner = br - bl - 1;
    const int t = inner > 0 ? ilog2_u64((uint64_t)inner) : 0;
    // query records (doubling table): one 16-byte load per end gives the
    // end block's key and the window of 2^t blocks beside it
    v2u64 pl = {KEY_NONE, KEY_NONE}, pr = {KEY_NONE, KEY_NONE};
    if (rec) {
      pl = *reinterpret_cast<const v2u64*>(rec + 2 * (bl * rlev + t));
      if (bl != br) pr = *reinterpret_cast<const v2u64*>(rec + 2 * ((nb + br) * rlev + t));
    }
    // both end blocks' keys are read before the inner windows, so that all
    // of the query's table reads are in flight together (bl == br: the
    // same key twice)
    const uint64_t kl = rec ? pl.x : st[bl];
    const uint64_t kr_end = rec ? pr.x : st[br];
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
      if (inner > 0) {
        if (lg <= 1) {  // doubling (Section 2): two overlapping windows
          const TablePtr lev = st + (size_t)t * nb;
          best = rec ? umin64(pl.y, pr.y) : umin64(lev[bl + 1], lev[br - (1ll << t)]);
        } else {
          // l-ary table (Section 3.1), l = 2^lg: level i holds windows of
          // s = l^i blocks; whole windows from the left, then one ending at
          // the last inner block -- at most l of them.  The whole windows
          // share a residue class mod s, so they are adjacent entries.
          const int sh = (t / lg) * lg;
          const TablePtr lev = st + (size_t)(t / lg) * nb;
          const int64_t whole = inner >> sh;
          const TablePtr w = lev + lary_addr(bl + 1, nb, sh);
#pragma unroll 8
          for (int64_t j = 0; j < whole; ++j) best = umin64(best, w[j]);
          if (inner & ((1ll << sh) - 1))
            best = umin64(best, lev[lary_addr(br - (1ll << sh), nb, sh)]);
        }
      }
      kr = kr_end;
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

  return EndState{best, kr, loL, hiL, loR, hiR, ok, needL, needR};
}

// The same end-block step from a doubling table in LDS without query records
// (at most 18432 words: 32-bit indices), with no branches: every table read
// is made, at clamped indices, and the cases are selected afterwards.
template <class Src, class TablePtr>
__device__ __forceinline__ EndState query_ends_lds(const Src& src, int64_t src_len, int64_t n,
                                                   int kshift, TablePtr __restrict__ st,
                                                   int64_t nb, int64_t l, int64_t r, int64_t li,
                                                   int64_t ri, bool live) {
  const bool ok = live && 0 <= l && l <= r && r < n && 0 <= li && li <= ri && ri < src_len;
  const uint32_t bl = ok ? (uint32_t)(li >> kshift) : 0u;
  const uint32_t br = ok ? (uint32_t)(ri >> kshift) : 0u;
  const bool has_inner = br > bl + 1u;
  const uint32_t inner = has_inner ? br - bl - 1u : 1u;
  const int t = 31 - __clz(inner);
  const uint32_t base = (uint32_t)t * (uint32_t)nb;
  const uint32_t w1 = base + (has_inner ? bl + 1u : bl);
  const uint32_t w2 = base + (has_inner ? br - (1u << t) : bl);
  const uint64_t kl = st[bl], kre = st[br], x1 = st[w1], x2 = st[w2];
  const uint64_t b1 = has_inner ? umin64(x1, x2) : KEY_NONE;  // the inner windows
  const int64_t pl = (int64_t)src.pos_of(kl), pr = (int64_t)src.pos_of(kre);
  const bool same = bl == br;
  // one block: its minimum, or the whole range is a piece
  const bool in_one = l <= pl && pl <= r;
  // two end blocks: each end block's minimum if it lies in the range, else
  // a piece of it while that minimum could still win
  const bool l_in = pl >= l;
  const uint64_t b2 = l_in ? umin64(b1, kl) : b1;
  const bool r_in = pr <= r;
  const uint64_t b3 = r_in ? umin64(b2, kre) : b2;
  EndState e;
  e.ok = ok;
  e.best = !ok ? KEY_NONE : same ? (in_one ? kl : KEY_NONE) : b3;
  e.kr = ok && !same ? kre : KEY_NONE;
  e.needL = ok && (same ? !in_one : (!l_in && kl < b1));
  e.needR = ok && !same && !r_in && kre < b2;
  e.loL = ok ? li : 0;
  e.hiL = !ok ? -1 : same ? ri : (((int64_t)bl + 1) << kshift) - 1;
  e.loR = ok ? ((int64_t)br << kshift) : 0;
  e.hiR = ok ? ri : -1;
  return e;
}

// The partial-block step of one lane's query (all 64 lanes together) and its
// answer: the pieces the end-block step left are read, then out is written.
template <class Src>
__device__ __forceinline__ void query_scans(const Src& src, const EndState& e, int64_t l,
                                            int64_t r, bool live, int32_t* outp,
                                            unsigned long long* __restrict__ bad_count,
                                            unsigned long long* __restrict__ stats) {
  const int lane = lane_id();
  const bool ok = e.ok;
  uint64_t best = e.best;
  const uint64_t kr = e.kr;
  bool needL = e.needL, needR = e.needR;
  const int64_t loL = e.loL, hiL = e.hiL, loR = e.loR, hiR = e.hiR;
  // ---- partial-block scans: a short range is read by its own lane (many
  // of them at once); a long one is queued and read by the whole wave ----
  uint64_t n_scans = 0, n_elems = 0;  // wave-uniform counts of queued scans
  int64_t lane_scans = 0, lane_reads = 0;
  const Src qsrc = src.with_query(l, r);  // this lane's query range in A
  if constexpr (Src::kLaneScans) {
    if (__popcll(ballot(needL)) >= LANE_SCAN_MIN && needL &&
        src.lane_cost(loL, hiL) <= LANE_SCAN_MAX) {
      best = umin64(best, qsrc.lane_scan(loL, hiL, best, lane_reads));
      lane_scans += 1;
      needL = false;
    }
  }
  if constexpr (Src::kGroupScans) {
    const uint64_t pl = ballot(needL), pr = ballot(needR);
    if (pl | pr) {
      // the widest queued piece sets the group size: G lanes read 64 G bytes
      // a pass; pieces over 2 KB are read wave-wide below
      uint32_t len = 0;
      if (needL) len = (uint32_t)(hiL - loL + 1);
      if (needR && (uint32_t)(hiR - loR + 1) > len) len = (uint32_t)(hiR - loR + 1);
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)len, d);
        len = o > len ? o : len;
      }
      const uint64_t bytes = (uint64_t)len << Src::kEntryShift;
      const uint32_t a = (uint32_t)loL, b = (uint32_t)hiL, c = (uint32_t)loR, e = (uint32_t)hiR;
      if (bytes <= 2048) {
        if (bytes <= 1024)
          grouped_scans<16>(qsrc, pl, pr, a, b, c, e, lane, best, n_scans, n_elems);
        else
          grouped_scans<32>(qsrc, pl, pr, a, b, c, e, lane, best, n_scans, n_elems);
        needL = needR = false;
      }
    }
  }
  uint64_t pend = ballot(needL);
  while (pend) {
    const int src_lane = __builtin_ctzll(pend);
    pend &= pend - 1;
    const int64_t lo = readlane64(loL, src_lane), hi = readlane64(hiL, src_lane);
    const uint64_t bound = (uint64_t)readlane64((int64_t)best, src_lane);
    int64_t reads = 0;
    const uint64_t m = qsrc.broadcast(src_lane).scan(lo, hi, lane, bound, reads);
    if (lane == src_lane) best = umin64(best, m);
    n_scans += 1;
    n_elems += (uint64_t)reads;
  }
  if (needR && !(kr < best)) needR = false;  // the left scan already beat this block
  if constexpr (Src::kLaneScans) {
    if (__popcll(ballot(needR)) >= LANE_SCAN_MIN && needR &&
        src.lane_cost(loR, hiR) <= LANE_SCAN_MAX) {
      best = umin64(best, qsrc.lane_scan(loR, hiR, best, lane_reads));
      lane_scans += 1;
      needR = false;
    }
  }
  pend = ballot(needR);
  while (pend) {
    const int src_lane = __builtin_ctzll(pend);
    pend &= pend - 1;
    const int64_t lo = readlane64(loR, src_lane), hi = readlane64(hiR, src_lane);
    const uint64_t bound = (uint64_t)readlane64((int64_t)best, src_lane);
    int64_t reads = 0;
    const uint64_t m = qsrc.broadcast(src_lane).scan(lo, hi, lane, bound, reads);
    if (lane == src_lane) best = umin64(best, m);
    n_scans += 1;
    n_elems += (uint64_t)reads;
  }

  if (live) __builtin_nontemporal_store(ok ? (int32_t)src.pos_of(best) : -1, outp);

  if (bad_count) {
    const uint64_t bad = ballot(live && !ok);
    if (bad && lane == 0) atomicAdd(bad_count, (unsigned long long)__popcll(bad));
  }
  if (stats) {
    for (int d = 1; d < 64; d <<= 1) {
      lane_scans += __shfl_xor(lane_scans, d);
      lane_reads += __shfl_xor(lane_reads, d);
    }
    n_scans += (uint64_t)lane_scans;
    n_elems += (uint64_t)lane_reads;
    if (n_scans && lane == 0) {
      atomicAdd(stats, (unsigned long long)n_scans);
      atomicAdd(stats + 1, (unsigned long long)n_elems);
    }
  }
}

// One lane's query [l, r] (positions in A, validated here) over source
// entries [li, ri] of its table (st: level-major, nb blocks of 2^kshift
// entries).  All 64 lanes of the wave must call this together: the partial
// scans are done by the whole wave.  Lanes may belong to different tables
// (batched launches); `live` is false for padding lanes.
template <class Src, class TablePtr = const uint64_t*>
__device__ __forceinline__ void query_core(const Src& src, int64_t src_len, int64_t n,
                                           int kshift, TablePtr __restrict__ st,
                                           int64_t nb, int64_t l, int64_t r, int64_t li,
                                           int64_t ri, bool live, int32_t* outp,
                                           unsigned long long* __restrict__ bad_count,
                                           unsigned long long* __restrict__ stats,
                                           int lg = 1, const uint64_t* __restrict__ rec = nullptr,
                                           int rlev = 0) {
  const EndState e = query_ends(src, src_len, n, kshift, st, nb, l, r, li, ri, live, lg, rec, rlev);
  query_scans(src, e, l, r, live, outp, bad_count, stats);
}

// One table.  L, R: the queries' positions in A.  For the contracted path, LR
// holds their contracted index ranges as interleaved pairs (LR[2i],
// LR[2i+1]); for the plain path LR is null and the ranges are [L[i], R[i]]
// themselves.  src_len: number of source entries (n or 2q - 1).  fail
// (contracted path): the endpoint sort's abort word; when it is set the
// contracted ranges cannot be trusted, and every query is answered -1 and
// counted as invalid.
template <class Src>
__global__ __launch_bounds__(WG) void k_query(Src src, int64_t src_len, int64_t n, int kshift,
                                              const uint64_t* __restrict__ st, int64_t nb,
                                              const int32_t* __restrict__ L,
                                              const int32_t* __restrict__ R,
                                              const int32_t* __restrict__ LR, int64_t q,
                                              int32_t* __restrict__ out,
                                              unsigned long long* __restrict__ bad_count,
                                              unsigned long long* __restrict__ stats, int lg,
                                              const uint64_t* __restrict__ rec, int rlev,
                                              const uint32_t* __restrict__ fail) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = i < q;
  const bool failed = fail && *fail != 0;  // uniform: one scalar load
  int64_t l = 0, r = -1, li = 0, ri = -1;
  if (live && !failed) {
    // the query streams are read once: non-temporal, so that they do not
    // push the table (gathered at random) out of the caches
    l = __builtin_nontemporal_load(L + i);
    r = __builtin_nontemporal_load(R + i);
    if (LR) {
      const int64_t c = __builtin_nontemporal_load(reinterpret_cast<const int64_t*>(LR) + i);
      li = (int32_t)(uint32_t)c;
      ri = (int32_t)(uint32_t)(c >> 32);
    } else {
      li = l;
      ri = r;
    }
  }
  query_core(src, src_len, n, kshift, st, nb, l, r, li, ri, live, out + (live ? i : 0),
             bad_count, stats, lg, rec, rlev);
}

// Large batches over a small doubling table (plain method): the table
// gathers are the launch's cost -- four 8-byte loads per query at random
// blocks, each wave load touching up to 64 lines, bound by the L2 request
// rate (n = 1e8, q = 1e7, k = 65536: 100 of the kernel's 110 us without its
// partial scans).  Here one 1024-thread workgroup per CU copies the whole
// table (at most LDS_TABLE_BYTES) into LDS once and then walks the query
// waves w, w + stride, ...; the table reads become LDS reads and each wave's
// L and R two rounds ahead are in flight while it answers the current ones.
// Partial scans still read A (and the k1-block minima) from memory.  Below
// 2^21 queries the copy per CU costs more than it saves (q = 1e6: 16-21 us
// against 16 us gathering).
constexpr int LWG = 1024;
constexpr int64_t LDS_TABLE_BYTES = 144 * 1024;
// src_len: source entries (n, or 2q - 1 for A_Q); LR: the contracted ranges
// (null for the plain method); fail: the endpoint sort's abort word (null,
// or when set every query is answered -1 and counted invalid).
template <class Src>
__global__ __launch_bounds__(LWG) void k_query_lds(Src src, int64_t src_len, int64_t n,
                                                   int kshift, const uint64_t* __restrict__ st,
                                                   int64_t nb, int64_t words,
                                                   const int32_t* __restrict__ L,
                                                   const int32_t* __restrict__ R,
                                                   const int32_t* __restrict__ LR, int64_t q,
                                                   int32_t* __restrict__ out,
                                                   unsigned long long* __restrict__ bad_count,
                                                   unsigned long long* __restrict__ stats,
                                                   const uint32_t* __restrict__ fail) {
  __shared__ __align__(16) uint64_t s_st[LDS_TABLE_BYTES / 8];
  const int lane = lane_id();
  const int64_t total = (q + 63) >> 6;
  const int64_t stride = (int64_t)gridDim.x * (LWG / 64);
  int64_t w = (int64_t)blockIdx.x * (LWG / 64) +
              __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool failed = fail && *fail != 0;  // uniform: one scalar load
  // this wave's queries two rounds ahead are in flight while it answers
  // the current ones (the first two go out before the table copy)
  struct Q {
    int32_t l, r;
    int64_t c;  // the contracted range pair (li low, ri high)
  };
  Q q1{0, -1, 0}, q2{0, -1, 0};
  auto fetch = [&](int64_t ww, Q& x) {
    const int64_t i = ww * 64 + lane;
    const bool in = ww < total && i < q && !failed;
    x.l = in ? __builtin_nontemporal_load(L + i) : 0;
    x.r = in ? __builtin_nontemporal_load(R + i) : -1;
    x.c = in && LR ? __builtin_nontemporal_load(reinterpret_cast<const int64_t*>(LR) + i) : 0;
  };
  fetch(w, q1);
  fetch(w + stride, q2);
  // the table, 16 bytes a load, all of a thread's loads in flight together
  // (the table starts on a 256-byte boundary)
  constexpr int PER = (int)(LDS_TABLE_BYTES / 16 / LWG);
  const int64_t pairs = words >> 1;
  v2u64 t[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t idx = threadIdx.x + (int64_t)u * LWG;
    if (idx < pairs) t[u] = reinterpret_cast<const v2u64*>(st)[idx];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t idx = threadIdx.x + (int64_t)u * LWG;
    if (idx < pairs) reinterpret_cast<v2u64*>(s_st)[idx] = t[u];
  }
  if ((words & 1) && threadIdx.x == 0) s_st[words - 1] = st[words - 1];
  __syncthreads();
  // the table reads in the LDS address space (ds loads, not flat ones)
  using LdsPtr = const __attribute__((address_space(3))) uint64_t*;
  const LdsPtr lds_table = (LdsPtr)s_st;
  for (; w < total; w += stride) {  // the same trip count for the whole wave
    const int64_t i = w * 64 + lane;
    const bool live = i < q;
    const int64_t l = q1.l, r = q1.r;
    const int64_t li = LR ? (int64_t)(int32_t)(uint32_t)q1.c : l;
    const int64_t ri = LR ? (int64_t)(int32_t)(uint32_t)(q1.c >> 32) : r;
    q1 = q2;
    fetch(w + 2 * stride, q2);
    const EndState e = query_ends_lds(src, src_len, n, kshift, lds_table, nb, l, r, li, ri, live);
    query_scans(src, e, l, r, live, out + (live ? i : 0), bad_count, stats);
  }
}

typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));

// ST-RMQ_CON's queries (Section 2; the comparison system): its A_Q holds,
// for sorted endpoint slot s, the marked element at entry 2s and the region
// up to slot s + 1 at entry 2s + 1, so query i (left end at slot LR[2i],
// right end at slot LR[2i + 1] + 1) covers entries 2 LR[2i] .. 2 LR[2i + 1]
// + 2, and the Sparse Table over every entry (Bender and Farach's doubling)
// answers it with two reads, of the windows of 2^t entries at both ends.
__global__ __launch_bounds__(WG) void k_query_st_elements(
    const uint64_t* __restrict__ st, int64_t m, int levels, const int32_t* __restrict__ L,
    const int32_t* __restrict__ R, const int32_t* __restrict__ LR, int64_t q, int64_t n,
    int32_t* __restrict__ out, unsigned long long* __restrict__ bad_count,
    const uint32_t* __restrict__ fail) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = i < q;
  const bool failed = fail && *fail != 0;
  bool ok = false;
  uint64_t best = KEY_NONE;
  if (live) {
    const int64_t l = __builtin_nontemporal_load(L + i), r = __builtin_nontemporal_load(R + i);
    const v2u32 c = __builtin_nontemporal_load(reinterpret_cast<const v2u32*>(LR) + i);
    const int64_t lo = 2 * (int64_t)(int32_t)c.x, hi = 2 * (int64_t)(int32_t)c.y + 2;
    ok = !failed && 0 <= l && l <= r && r < n && 0 <= lo && lo <= hi && hi < m;
    if (ok) {
      const int t = ilog2_u64((uint64_t)(hi - lo + 1));
      if (t < levels) {
        const uint64_t* lev = st + (size_t)t * (size_t)m;
        best = umin64(lev[lo], lev[hi - (1ll << t) + 1]);
      } else {
        ok = false;  // never, for a table of ilog2(m) + 1 levels
      }
    }
    __builtin_nontemporal_store(ok ? (int32_t)key_pos(best) : -1, out + i);
  }
  if (bad_count) {
    const uint64_t bad = ballot(live && !ok);
    if (bad && lane_id() == 0) atomicAdd(bad_count, (unsigned long long)__popcll(bad));
  }
}

// Every query of a batch of tables (plain path): global query g belongs to
// the table whose range of the concatenated query list holds it.
// Queries of a batch: wave w does job w, 64 consecutive queries of one
// array (each array's queries padded to whole waves, so a wave never spans
// two arrays).  An array has two block levels (SrcA2) or one (SrcA).
template <class Src>
__device__ __forceinline__ Src array_src(const ArrayDesc& d);
template <>
__device__ __forceinline__ SrcA array_src<SrcA>(const ArrayDesc& d) {
  return SrcA{d.A, d.n};
}
template <>
__device__ __forceinline__ SrcA2 array_src<SrcA2>(const ArrayDesc& d) {
  return SrcA2{SrcA{d.A, d.n}, d.sub, d.nb1, d.k1shift};
}

// One launch for the waves of every array: a wave's job says whether its
// array has two block levels (the branch is uniform over the wave).
__global__ __launch_bounds__(WG) void k_query_multi(const WaveJob* __restrict__ jobs,
                                                    int64_t waves) {
  const int64_t w = (int64_t)blockIdx.x * (WG / 64) +
                    __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const WaveJob& jb = jobs[w < waves ? w : waves - 1];
  const ArrayDesc& d = jb.d;
  const int64_t i = jb.q0 + lane_id();
  const bool live = w < waves && i < d.q;
  int64_t l = 0, r = -1;
  if (live) {
    l = __builtin_nontemporal_load(d.L + i);
    r = __builtin_nontemporal_load(d.R + i);
  }
  if (d.sub)
    query_core(array_src<SrcA2>(d), d.n, d.n, d.kshift, d.st, d.nb, l, r, l, r, live,
               d.out + (live ? i : 0), nullptr, nullptr, d.lg, d.rec, d.rlev);
  else
    query_core(array_src<SrcA>(d), d.n, d.n, d.kshift, d.st, d.nb, l, r, l, r, live,
               d.out + (live ? i : 0), nullptr, nullptr, d.lg, d.rec, d.rlev);
}

// A coalesced batch of requests (serving): queries g in
// [seg_prefix[s], seg_prefix[s+1]) belong to request s, which targets the
// resident table tables[seg_table[s]].
template <class Src>
__global__ __launch_bounds__(WG) void k_query_segments(const ArrayDesc* __restrict__ tables,
                                                       const int64_t* __restrict__ seg_prefix,
                                                       const int32_t* __restrict__ seg_table,
                                                       int nseg, const int32_t* __restrict__ L,
                                                       const int32_t* __restrict__ R,
                                                       int32_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
  const int64_t total = seg_prefix[nseg];
  const bool live = g < total;
  const int64_t gw = (int64_t)blockIdx.x * WG + (threadIdx.x & ~63);  // the wave's first query
  const int sg = find_item_wave(seg_prefix, nseg, gw < total ? gw : total - 1, live ? g : gw);
  const ArrayDesc& d = tables[seg_table[sg]];
  int64_t l = 0, r = -1;
  if (live) {
    l = L[g];
    r = R[g];
  }
  query_core(array_src<Src>(d), d.n, d.n, d.kshift, d.st, d.nb, l, r, l, r, live,
             out + (live ? g : 0), nullptr, nullptr, d.lg, d.rec, d.rlev);
}

// Lowest common ancestors (Section 1): query i is the pair (U[i], V[i]) of
// tree nodes; its range over the Euler tour's depth array runs between their
// first occurrences, and the answer is the tour node at the minimum depth.
template <class Src>
__global__ __launch_bounds__(WG) void k_query_lca(Src src, int64_t len, int kshift,
                                                  const uint64_t* __restrict__ st, int64_t nb,
                                                  const int32_t* __restrict__ first,
                                                  const int32_t* __restrict__ node, int64_t N,
                                                  const int32_t* __restrict__ U,
                                                  const int32_t* __restrict__ V, int64_t q,
                                                  int32_t* __restrict__ out,
                                                  unsigned long long* __restrict__ bad_count,
                                                  int lg, const uint64_t* __restrict__ rec,
                                                  int rlev) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  const bool live = i < q;
  int64_t l = -1, r = -1;  // an invalid node leaves l < 0: answered -1
  if (live) {
    const int64_t u = U[i], v = V[i];
    if (0 <= u && u < N && 0 <= v && v < N) {
      const int64_t fu = first[u], fv = first[v];
      l = fu < fv ? fu : fv;
      r = fu < fv ? fv : fu;
    }
  }
  query_core(src, len, len, kshift, st, nb, l, r, l, r, live, out + (live ? i : 0), bad_count,
             nullptr, lg, rec, rlev);
  if (live) {
    const int32_t p = out[i];
    out[i] = p >= 0 ? node[p] : -1;
  }
}

}  // namespace

hipError_t launch_query_segments(const ArrayDesc* tables, const int64_t* seg_prefix,
                                 const int32_t* seg_table, int nseg, const int32_t* L,
                                 const int32_t* R, int32_t* out, int64_t total, bool two_level,
                                 hipStream_t stream) {
  if (total <= 0) return hipSuccess;
  const int64_t grid = (total + WG - 1) / WG;
  if (two_level)
    RMQ_TRY(launch(k_query_segments<SrcA2>, dim3((unsigned)grid), dim3(WG), 0, stream, tables,
                   seg_prefix, seg_table, nseg, L, R, out));
  else
    RMQ_TRY(launch(k_query_segments<SrcA>, dim3((unsigned)grid), dim3(WG), 0, stream, tables,
                   seg_prefix, seg_table, nseg, L, R, out));
  return hipSuccess;
}

// Whether a plain-method batch takes k_query_lds: a doubling table of at
// most LDS_TABLE_BYTES, and enough queries to pay for one copy of it per CU.
// Returns the table's words (levels x nb), else 0.
constexpr int64_t LDS_MIN_QUERIES = 1 << 21;
int64_t lds_table_words(int64_t nb, int lg, int64_t q) {
  if (lg != 1 || q < LDS_MIN_QUERIES || nb < 1) return 0;
  int levels = 1;  // floor(log2(nb - 2)) + 1 levels (one for nb <= 3)
  if (nb > 3) {
    levels = 0;
    for (int64_t x = nb - 2; x; x >>= 1) ++levels;
  }
  const int64_t words = nb * levels;
  return words * 8 <= LDS_TABLE_BYTES ? words : 0;
}

int lds_grid(int64_t q) {
  const int cus = device_cu_count();
  const int64_t waves = (q + 63) / 64;
  const int64_t need = (waves + LWG / 64 - 1) / (LWG / 64);
  return (int)(need < cus ? need : cus);
}

hipError_t launch_query_full(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                             int64_t nb, const int32_t* L, const int32_t* R, int64_t q,
                             int32_t* out, int64_t* bad_count, uint64_t* stats,
                             hipStream_t stream, int lg, const uint64_t* rec, int rlev) {
  if (q <= 0) return hipSuccess;
  if (const int64_t words = lds_table_words(nb, lg, q)) {
    RMQ_TRY(launch(k_query_lds<SrcA>, dim3((unsigned)lds_grid(q)), dim3(LWG), 0, stream,
                   SrcA{A, n}, n, n, kshift, st, nb, words, L, R,
                   static_cast<const int32_t*>(nullptr), q, out, (unsigned long long*)bad_count,
                   (unsigned long long*)stats, static_cast<const uint32_t*>(nullptr)));
    return hipGetLastError();
  }
  const int64_t grid = (q + WG - 1) / WG;
  RMQ_TRY(launch(k_query<SrcA>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcA{A, n}, n, n,
                 kshift, st, nb, L, R, static_cast<const int32_t*>(nullptr), q, out,
                 (unsigned long long*)bad_count, (unsigned long long*)stats, lg, rec, rlev,
                 static_cast<const uint32_t*>(nullptr)));
  return hipGetLastError();
}

hipError_t launch_query_full2(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                              int64_t nb, const uint64_t* sub, int k1shift, const int32_t* L,
                              const int32_t* R, int64_t q, int32_t* out, int64_t* bad_count,
                              uint64_t* stats, hipStream_t stream, int lg, const uint64_t* rec,
                              int rlev) {
  if (q <= 0) return hipSuccess;
  const int64_t nsub = (n + (1ll << k1shift) - 1) >> k1shift;
  if (const int64_t words = lds_table_words(nb, lg, q)) {
    RMQ_TRY(launch(k_query_lds<SrcA2>, dim3((unsigned)lds_grid(q)), dim3(LWG), 0, stream,
                   SrcA2{SrcA{A, n}, sub, nsub, k1shift}, n, n, kshift, st, nb, words, L, R,
                   static_cast<const int32_t*>(nullptr), q, out, (unsigned long long*)bad_count,
                   (unsigned long long*)stats, static_cast<const uint32_t*>(nullptr)));
    return hipGetLastError();
  }
  const int64_t grid = (q + WG - 1) / WG;
  RMQ_TRY(launch(k_query<SrcA2>, dim3((unsigned)grid), dim3(WG), 0, stream,
                 SrcA2{SrcA{A, n}, sub, nsub, k1shift}, n, n, kshift, st, nb, L, R,
                 static_cast<const int32_t*>(nullptr), q, out, (unsigned long long*)bad_count,
                 (unsigned long long*)stats, lg, rec, rlev, static_cast<const uint32_t*>(nullptr)));
  return hipGetLastError();
}

hipError_t launch_query_full3(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                              int64_t nb, const uint64_t* sub, int k1shift, const uint64_t* sub2,
                              int k2shift, const int32_t* L, const int32_t* R, int64_t q,
                              int32_t* out, int64_t* bad_count, uint64_t* stats,
                              hipStream_t stream, int lg) {
  if (q <= 0) return hipSuccess;
  const int64_t nsub = (n + (1ll << k1shift) - 1) >> k1shift;
  const int64_t nsub2 = (n + (1ll << k2shift) - 1) >> k2shift;
  const SrcA3 src{SrcA2{SrcA{A, n}, sub2, nsub2, k2shift}, sub, nsub, k1shift};
  if (const int64_t words = lds_table_words(nb, lg, q)) {
    RMQ_TRY(launch(k_query_lds<SrcA3>, dim3((unsigned)lds_grid(q)), dim3(LWG), 0, stream, src, n,
                   n, kshift, st, nb, words, L, R, static_cast<const int32_t*>(nullptr), q, out,
                   (unsigned long long*)bad_count, (unsigned long long*)stats,
                   static_cast<const uint32_t*>(nullptr)));
    return hipGetLastError();
  }
  const int64_t grid = (q + WG - 1) / WG;
  RMQ_TRY(launch(k_query<SrcA3>, dim3((unsigned)grid), dim3(WG), 0, stream, src, n, n, kshift, st,
                 nb, L, R, static_cast<const int32_t*>(nullptr), q, out,
                 (unsigned long long*)bad_count, (unsigned long long*)stats, lg,
                 static_cast<const uint64_t*>(nullptr), 0, static_cast<const uint32_t*>(nullptr)));
  return hipGetLastError();
}

hipError_t launch_query_lca(const int32_t* D, int64_t len, int kshift, const uint64_t* st,
                            int64_t nb, const uint64_t* sub, int k1shift, const int32_t* first,
                            const int32_t* node, int64_t N, const int32_t* U, const int32_t* V,
                            int64_t q, int32_t* out, int64_t* bad_count, hipStream_t stream,
                            int lg, const uint64_t* rec, int rlev) {
  if (q <= 0) return hipSuccess;
  const int64_t grid = (q + WG - 1) / WG;
  if (sub) {
    const int64_t nsub = (len + (1ll << k1shift) - 1) >> k1shift;
    RMQ_TRY(launch(k_query_lca<SrcA2>, dim3((unsigned)grid), dim3(WG), 0, stream,
                   SrcA2{SrcA{D, len}, sub, nsub, k1shift}, len, kshift, st, nb, first, node, N,
                   U, V, q, out, (unsigned long long*)bad_count, lg, rec, rlev));
  } else {
    RMQ_TRY(launch(k_query_lca<SrcA>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcA{D, len},
                   len, kshift, st, nb, first, node, N, U, V, q, out,
                   (unsigned long long*)bad_count, lg, rec, rlev));
  }
  return hipSuccess;
}

hipError_t launch_query_contracted(const uint64_t* aq, int64_t m, int64_t n, int kshift,
                                   const uint64_t* st, int64_t nb, const int32_t* L,
                                   const int32_t* R, const int32_t* LR, int64_t q, int32_t* out,
                                   int64_t* bad_count, uint64_t* stats, hipStream_t stream,
                                   int lg, const uint64_t* rec, int rlev, const uint64_t* sub,
                                   int k1shift, const uint32_t* fail) {
  if (q <= 0) return hipSuccess;
  if (const int64_t words = lds_table_words(nb, lg, q)) {
    if (sub) {
      const int64_t nsub = (m + (1ll << k1shift) - 1) >> k1shift;
      RMQ_TRY(launch(k_query_lds<SrcKeys2>, dim3((unsigned)lds_grid(q)), dim3(LWG), 0, stream,
                     SrcKeys2{SrcKeys{aq, m}, sub, nsub, k1shift}, m, n, kshift, st, nb, words, L,
                     R, LR, q, out, (unsigned long long*)bad_count, (unsigned long long*)stats,
                     fail));
    } else {
      RMQ_TRY(launch(k_query_lds<SrcKeys>, dim3((unsigned)lds_grid(q)), dim3(LWG), 0, stream,
                     SrcKeys{aq, m}, m, n, kshift, st, nb, words, L, R, LR, q, out,
                     (unsigned long long*)bad_count, (unsigned long long*)stats, fail));
    }
    return hipGetLastError();
  }
  const int64_t grid = (q + WG - 1) / WG;
  if (sub) {
    const int64_t nsub = (m + (1ll << k1shift) - 1) >> k1shift;
    RMQ_TRY(launch(k_query<SrcKeys2>, dim3((unsigned)grid), dim3(WG), 0, stream,
                   SrcKeys2{SrcKeys{aq, m}, sub, nsub, k1shift}, m, n, kshift, st, nb, L, R, LR,
                   q, out, (unsigned long long*)bad_count, (unsigned long long*)stats, lg, rec,
                   rlev, fail));
  } else {
    RMQ_TRY(launch(k_query<SrcKeys>, dim3((unsigned)grid), dim3(WG), 0, stream, SrcKeys{aq, m},
                   m, n, kshift, st, nb, L, R, LR, q, out, (unsigned long long*)bad_count,
                   (unsigned long long*)stats, lg, rec, rlev, fail));
  }
  return hipGetLastError();
}

hipError_t launch_query_st_elements(const uint64_t* st, int64_t m, int levels, const int32_t* L,
                                    const int32_t* R, const int32_t* LR, int64_t q, int64_t n,
                                    int32_t* out, int64_t* bad_count, hipStream_t stream,
                                    const uint32_t* fail) {
  if (q <= 0) return hipSuccess;
  RMQ_TRY(launch(k_query_st_elements, dim3((unsigned)((q + WG - 1) / WG)), dim3(WG), 0, stream,
                 st, m, levels, L, R, LR, q, n, out, (unsigned long long*)bad_count, fail));
  return hipSuccess;
}

hipError_t launch_query_multi(const WaveJob* jobs, int64_t waves, hipStream_t stream) {
  if (waves <= 0) return hipSuccess;
  const int64_t grid = (waves + WG / 64 - 1) / (WG / 64);
  RMQ_TRY(launch(k_query_multi, dim3((unsigned)grid), dim3(WG), 0, stream, jobs, waves));
  return hipSuccess;
}

// Compute units of the current device (cached per device; 256 if the
// runtime cannot say).
int device_cu_count() {
  static int cus[64] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  if (!cus[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
      c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

}  // namespace rmq
