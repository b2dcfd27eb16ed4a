// Device LSD radix sort of the 2q query endpoints, and the remap that follows
// it (Section 3.1 step 1).
//
// Item j of the endpoint list is (position, tag j): the left end of query i
// is item 2i and its right end item 2i+1.  Sorting by position with a STABLE
// sort keeps equal positions in tag order, so the result is ordered by
// (position, tag) -- the same order any sort on the pair gives.
//
// One sweep per digit of the position (ceil(log2 n) bits in all):
//   k_os_clear  -- clears digit totals, tickets and the first status words;
//   k_os_hist   -- one read of the input: digit totals of every pass at once,
//                  by range of tiles (per workgroup in LDS, then global
//                  atomics);
//   k_os_pass   -- per pass, one workgroup (one thread per digit value) per
//                  tile of 1024, 2048 or 8192 items (by list length), taken
//                  in order from an atomic ticket (in the first pass, the
//                  tiles form 8 ranges of contiguous tiles with a ticket
//                  each).  The tile ranks its items stably (one wave ballot
//                  per digit bit gives the lanes that share a digit),
//                  publishes its per-digit counts at once, stages the tile in
//                  LDS in digit order, and meanwhile finds the number of
//                  same-digit items in the earlier tiles (of its range; the
//                  earlier ranges' counts come from the histogram) by a
//                  decoupled look-back over their published words (count +
//                  "aggregate" or "inclusive" flag in one 64-bit word, read
//                  four predecessors at a time).  It then writes runs of
//                  equal digits contiguously.  A tile only ever waits on tiles
//                  that took their ticket earlier and are therefore running,
//                  so the waits end; each is also bounded, and an exceeded
//                  bound sets an abort word that ends every wait at once.
//                  A sort whose abort word is set has given up on its order:
//                  the word stays set for the kernels after it, which then
//                  report the failure instead of their results (the query
//                  kernel answers -1 for every query and counts each as
//                  invalid; the stand-alone stages write -1; the LCA build
//                  returns an error).
// Items are 8 bytes, (position << 32) | tag; the key bits are split into the
// fewest passes of at most 9 bits with equal widths (27 bits -> 9, 9, 9).
// The passes issue more instructions than they move bytes (the ranking takes
// one ballot per key bit of every item, whatever the split), so fewer, wider
// passes over large tiles cost less: measured at n = 1e8, the sort of 2q
// endpoints took 0.64 / 0.11 / 0.044 ms at q = 1e7 / 1e6 / 1e5 with 9-bit
// digits and 8192-item tiles against 0.65 / 0.135 / 0.054 ms with four
// passes of 7 bits over 4096-item tiles.  Staging the tile in LDS before the
// global writes pays: storing each item straight from registers at its
// digit run (runs written by many store instructions) was slower at
// q = 1e7 (0.71 - 0.77 ms).
// The first pass reads L and R directly (invalid queries sort as position
// 0; the query kernel re-checks them), the last writes the output list E.
//
// Remap: slot s of the sorted list holding tag t gives Lc[t/2] = s (t even)
// or Rc[t/2] = s - 1 (t odd).  Inside the whole pipeline the last sort pass
// writes these 2q scattered 4-byte stores itself, as it places each item;
// for long lists (2q >= 2^22) it instead writes each tile's (tag, slot)
// pairs grouped by window of 32768 tags, and k_remap_windows assembles each
// window of LR in LDS and writes it out whole (a scattered 4-byte store
// costs a partial write to HBM once LR outgrows the L2s).
// The stand-alone remap (from a given sorted list) instead orders the
// (tag, slot) pairs by the top bits of the tag with one more sweep and then
// writes window by window, each window of the interleaved LR array while it
// sits in one XCD's L2.
#include <atomic>

#include "device.h"
#include "kernels.h"

namespace rmq {

// Value every later sort's abort word starts at (tests of the failure
// report set it to 1, so that each wait ends at once; see
// set_sort_abort_preset).
static std::atomic<uint32_t> g_abort_preset{0};

void set_sort_abort_preset(bool on) { g_abort_preset.store(on ? 1u : 0u); }

namespace {

// Digit width and the tile of long lists (build-time choices).
#ifndef RMQ_SORT_RADIX_BITS
#define RMQ_SORT_RADIX_BITS 9
#endif
#ifndef RMQ_SORT_BIG_TILE
#define RMQ_SORT_BIG_TILE 8192
#endif
constexpr int RADIX_BITS = RMQ_SORT_RADIX_BITS;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int WG = RADIX;  // one thread per digit value
constexpr int BIG_TILE = RMQ_SORT_BIG_TILE;
constexpr int BIG_ROUNDS = BIG_TILE / WG;
constexpr int R1K = 1024 / WG > 0 ? 1024 / WG : 1;
constexpr int R2K = 2048 / WG > 0 ? 2048 / WG : 1;
// Items per thread of a tile (a tile is WG * ROUNDS items), chosen by the
// list length N: small lists take small tiles so that more workgroups share
// them, long ones large tiles (fewer look-back steps, longer digit runs):
// 1024-item tiles below 10^5 items, 2048 below 4 * 10^5, BIG_TILE above.
int rounds_for(int64_t N) { return N < 100000 ? R1K : (N < 400000 ? R2K : BIG_ROUNDS); }
constexpr int NXCD = 8;

// Items are 8 bytes: (key << 32) | value, so a digit run of a tile is one
// contiguous run of whole cache lines in the output.
// Where a pass takes its items from:
enum Mode : int {
  ITEMS = 0,    // items_in[j]
  QUERIES = 1,  // item j = ((L[j/2] or R[j/2]) << 32) | j
  E_TAGS = 2,   // item j = (low half of items_in[j] << 32) | j
};

// Tile handled by this workgroup: XCD x = blockIdx % 8 takes the x-th
// contiguous range of tiles.  Returns -1 for the padding workgroups.
__device__ __forceinline__ int64_t xcd_tile(int64_t num_tiles) {
  const int64_t per = (num_tiles + NXCD - 1) / NXCD;
  const int64_t t = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  return t < num_tiles ? t : -1;
}
int64_t xcd_grid(int64_t num_tiles) { return ((num_tiles + NXCD - 1) / NXCD) * NXCD; }

template <int ROUNDS>
__device__ __forceinline__ int64_t item_index(int64_t tile0, int wave, int round, int lane) {
  return tile0 + (int64_t)wave * (64 * ROUNDS) + round * 64 + lane;
}

// Loading item j takes two steps so that a tile's loads can all be in
// flight at once: load_raw reads memory (index clamped to the list, no
// branch), finish_item builds the item.  Items j >= N are never counted.
template <int MODE>
__device__ __forceinline__ uint64_t load_raw(const uint64_t* __restrict__ items_in,
                                             const int32_t* __restrict__ L,
                                             const int32_t* __restrict__ R, int64_t N, int64_t j) {
  const int64_t jc = j < N ? j : N - 1;
  if (MODE == QUERIES) return (uint32_t)((jc & 1) ? R[jc >> 1] : L[jc >> 1]);
  return items_in[jc];
}

// From the queries, item j is (position << 32) | j.  Lanes 2i and 2i+1 of a
// round hold the two ends of one query, so validity is shared through a lane
// swap; an invalid query's ends sort as position 0.
template <int MODE>
__device__ __forceinline__ uint64_t finish_item(uint64_t raw, int64_t n, int64_t j) {
  if (MODE == QUERIES) {
    const int32_t x = (int32_t)(uint32_t)raw;
    const int32_t other = __shfl_xor(x, 1);
    const int32_t l = (j & 1) ? other : x, r = (j & 1) ? x : other;
    const bool ok = 0 <= l && l <= r && (int64_t)r < n;
    return ((uint64_t)(ok ? (uint32_t)x : 0u) << 32) | (uint32_t)j;
  }
  if (MODE == E_TAGS) return (raw << 32) | (uint32_t)j;
  return raw;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t item, int shift, uint32_t mask) {
  return ((uint32_t)(item >> 32) >> shift) & mask;
}
// The same, with the digit width instead of its mask (one bit-field extract).
__device__ __forceinline__ uint32_t digit_bits(uint64_t item, int shift, int bits) {
  return __builtin_amdgcn_ubfe((uint32_t)(item >> 32), (uint32_t)shift, (uint32_t)bits);
}

constexpr int MAX_PASSES = 4;
// Copies of the digit totals, one per range of tiles (below): a histogram
// workgroup adds into the copy of the range its tiles lie in, and a pass
// sums the copies.  Device-scope atomics on one address are serialised;
// with a single copy every address takes one add per workgroup (1221 of
// them at 2e7 items) and the adds, not the reads, set the histogram's time
// (38 us against 26 us with 8 copies at 2e7 items).
constexpr int HCOPIES = 8;
constexpr int HSTRIDE = MAX_PASSES * RADIX;  // words between copies
// The first pass's tiles form CHAINS ranges of contiguous tiles, each with
// its own ticket counter and its own look-back: range x (tiles
// x * range_tiles ..) is taken by the workgroups with blockIdx % CHAINS ==
// x, and its items of digit d start after those of every earlier range, a
// count the histogram gives by range (copy x of the totals holds range x's).
// With one chain over all tiles a tile's look-back walks back about 28
// tiles (7 reads of four predecessors, ~0.9 us each, at 2e7 items): the
// nearest tile with an inclusive count is as far back as the tiles issued
// meanwhile, and with eight chains each issues an eighth of them.  The
// later passes read the previous pass's output, whose per-range digit
// counts nothing has counted, so they run as one chain.
constexpr int CHAINS = HCOPIES;
struct Chains {
  uint32_t* tickets;    // nchains counters of this pass
  int64_t range_tiles;  // tiles per range (a multiple of the histogram's tiles per group)
  int64_t num_tiles;
  int nchains;          // CHAINS in the first pass, else 1 (range_tiles = num_tiles)
};
Chains first_pass_chains(uint32_t* tickets, int64_t range_tiles, int64_t num_tiles) {
  return Chains{tickets, range_tiles, num_tiles, CHAINS};
}
Chains one_chain(uint32_t* tickets, int64_t num_tiles) {
  return Chains{tickets, num_tiles, num_tiles, 1};
}
// Tiles per histogram workgroup: one while the grid is small (every tile's
// loads then start at once), up to 8 for long lists (fewer global atomics).
int hist_tiles(int64_t num_tiles) {
  const int64_t t = num_tiles / 1024;
  return t < 1 ? 1 : (t > 8 ? 8 : (int)t);
}
#ifndef RMQ_SORT_LOOKBACK
#define RMQ_SORT_LOOKBACK 4
#endif
constexpr int LOOKBACK = RMQ_SORT_LOOKBACK;  // predecessors read per look-back step
constexpr uint64_t ST_AGG = 1ull << 62;
constexpr uint64_t ST_INC = 2ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 18;

struct Digits {  // the digit split of one sort: pass p covers key bits
  int passes;    // [shift[p], shift[p] + bits[p])
  int shift[MAX_PASSES];
  int bits[MAX_PASSES];
};

// Balanced split of nbits key bits starting at bit `base` into the fewest
// passes of at most 9 bits (27 bits -> 9, 9, 9; 20 bits -> 7, 7, 6): every pass then has
// digits of similar spread, which keeps LDS counters uncontended and digit
// runs long.
Digits split_digits(int base, int nbits) {
  Digits d{};
  d.passes = (nbits + RADIX_BITS - 1) / RADIX_BITS;
  if (d.passes < 1) d.passes = 1;
  const int w = (nbits + d.passes - 1) / d.passes;
  int at = 0;
  for (int p = 0; p < d.passes; ++p) {
    d.shift[p] = base + at;
    d.bits[p] = nbits - at < w ? nbits - at : w;
    if (d.bits[p] < 1) d.bits[p] = 1;
    at += w;
  }
  return d;
}

__device__ __forceinline__ uint64_t load_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Clears what the sweeps accumulate into: digit totals, tickets, abort word
// (to `preset`, normally 0), and the first pass's tile status words.
__global__ __launch_bounds__(WG) void k_os_clear(uint32_t* __restrict__ hist,
                                                 uint32_t* __restrict__ tickets,
                                                 uint32_t* __restrict__ abort_word,
                                                 uint32_t preset,
                                                 uint64_t* __restrict__ status0,
                                                 int64_t status_words) {
  const int64_t i0 = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (blockIdx.x == 0) {
#pragma unroll
    for (int p = 0; p < HCOPIES * MAX_PASSES; ++p) hist[p * RADIX + threadIdx.x] = 0;
    if (threadIdx.x < CHAINS + MAX_PASSES) tickets[threadIdx.x] = 0;
    if (threadIdx.x == 0) *abort_word = preset;
  }
  for (int64_t i = i0; i < status_words; i += (int64_t)gridDim.x * WG) status0[i] = 0;
}

// Digit totals of every pass: per-wave counts in LDS over per_group tiles
// (pairs of waves share a set of counters), summed per workgroup, then one
// global atomic add per digit into the copy of the group's range.  From the queries,
// a whole tile of 16-byte aligned L and R is read four queries per load.
template <int MODE, int ROUNDS>
__global__ __launch_bounds__(WG) void k_os_hist(const uint64_t* __restrict__ items_in,
                                                const int32_t* __restrict__ L,
                                                const int32_t* __restrict__ R, int64_t N,
                                                int64_t n, Digits dg, int per_group,
                                                int64_t range_tiles,
                                                uint32_t* __restrict__ hist) {
  constexpr int TILE = WG * ROUNDS;
  constexpr int HSETS = 4;  // counter sets, one per pair of waves
  __shared__ uint32_t h[HSETS][MAX_PASSES][RADIX];
  const int lane = lane_id(), wave = threadIdx.x >> 6, hs = wave & (HSETS - 1);
#pragma unroll
  for (int w = 0; w < HSETS; ++w)
#pragma unroll
    for (int p = 0; p < MAX_PASSES; ++p) h[w][p][threadIdx.x] = 0;
  __syncthreads();
  auto count = [&](uint64_t item) {
#pragma unroll
    for (int p = 0; p < MAX_PASSES; ++p)
      if (p < dg.passes) atomicAdd(&h[hs][p][digit_bits(item, dg.shift[p], dg.bits[p])], 1u);
  };
  const bool vec = MODE == QUERIES && ROUNDS % 8 == 0 && (((uintptr_t)L | (uintptr_t)R) & 15) == 0;
  for (int t = 0; t < per_group; ++t) {
    const int64_t tile0 = ((int64_t)blockIdx.x * per_group + t) * TILE;
    if (tile0 >= N) break;
    if constexpr (MODE == QUERIES && ROUNDS % 8 == 0) {
      if (vec && tile0 + TILE <= N) {
        // queries tile0/2 .. (tile0 + TILE)/2 - 1, four per thread and step
        constexpr int STEPS = ROUNDS / 8;
        const int64_t q0 = tile0 >> 1;
        v4i32 l[STEPS], r[STEPS];
#pragma unroll
        for (int st = 0; st < STEPS; ++st) {
          const int64_t qi = q0 + (int64_t)st * (WG * 4) + threadIdx.x * 4;
          l[st] = *reinterpret_cast<const v4i32*>(L + qi);
          r[st] = *reinterpret_cast<const v4i32*>(R + qi);
        }
#pragma unroll
        for (int st = 0; st < STEPS; ++st)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int32_t lo = l[st][k], hi = r[st][k];
            const bool ok = 0 <= lo && lo <= hi && (int64_t)hi < n;  // as finish_item
            count((uint64_t)(ok ? (uint32_t)lo : 0u) << 32);
            count((uint64_t)(ok ? (uint32_t)hi : 0u) << 32);
          }
        continue;
      }
    }
    uint64_t it[ROUNDS];
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd)
      it[rd] = load_raw<MODE>(items_in, L, R, N, item_index<ROUNDS>(tile0, wave, rd, lane));
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd)
      it[rd] = finish_item<MODE>(it[rd], n, item_index<ROUNDS>(tile0, wave, rd, lane));
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) {
      if (item_index<ROUNDS>(tile0, wave, rd, lane) < N) count(it[rd]);
    }
  }
  __syncthreads();
  // the copy of the range holding this group's tiles
  uint32_t* mine = hist + (((int64_t)blockIdx.x * per_group) / range_tiles) * HSTRIDE;
  for (int p = 0; p < dg.passes; ++p) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < HSETS; ++w) c += h[w][p][threadIdx.x];
    if (c) atomicAdd(&mine[p * RADIX + threadIdx.x], c);
  }
}

// Exclusive scan of WG values held one per thread; returns the total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp,
                                                         uint32_t& excl) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t x = wave_inclusive_add_u32(v);
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  uint32_t off = 0, total = 0;
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) {
    if (w < wave) off += tmp[w];
    total += tmp[w];
  }
  __syncthreads();
  excl = off + x - v;
  return total;
}

// Decoupled look-back for digit d of `tile`: the number of digit-d items in
// the earlier tiles of its range (`first` .. tile - 1; tile `first`
// publishes an inclusive word at once).  Reads LOOKBACK predecessors' words
// at once, newest first, and takes values up to the first inclusive one, or
// stops at an unpublished one and reads again.  A tile only waits on tiles that took
// their ticket earlier; the wait is bounded, and an exceeded bound (or an
// abort word already set) ends it with a partial count and sets the abort
// word, which ends every other wait at once.
__device__ __forceinline__ uint64_t look_back(const uint64_t* status, int64_t tile,
                                              int64_t first, int d, uint32_t* abort_word) {
  uint64_t before = 0;
  int64_t j = tile - 1;
  uint32_t spins = 0;
  for (;;) {
    uint64_t w[LOOKBACK];
#pragma unroll
    for (int i = 0; i < LOOKBACK; ++i)
      w[i] = j - i >= first ? load_status(status + (j - i) * RADIX + d) : 0;
    bool done = false;
    int used = 0;
#pragma unroll
    for (int i = 0; i < LOOKBACK; ++i) {
      if (done || used != i || (w[i] & ~ST_VAL) == 0) continue;
      before += w[i] & ST_VAL;
      done = (w[i] & ST_INC) != 0;
      used = i + 1;
    }
    if (done) break;
    j -= used;
    if (used == 0) {  // the nearest unread predecessor has not published yet
      if (++spins > SPIN_LIMIT ||
          __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return before;
}

// Stable rank of each lane's digit among the lanes of the wave holding the
// same digit: the lanes whose every one of the BITS digit bits equals this
// lane's are those outside the OR over the bits of (ballot of the bit) XOR
// (own bit spread over the word).  Returns the mask of those lanes.
template <int BITS>
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, uint64_t valid_mask) {
  uint32_t xlo = 0, xhi = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);  // bit b, spread
    const uint64_t m = ballot(x != 0);
    xlo |= (uint32_t)m ^ x;
    xhi |= (uint32_t)(m >> 32) ^ x;
  }
  return valid_mask & ~(((uint64_t)xhi << 32) | xlo);
}

// The remap through LR windows (the last pass of long endpoint sorts): tags
// fall into windows of 2^win_shift consecutive tags (at most 2^15, 128 KiB
// of LR); the last pass writes each tile's (tag << 32 | slot) pairs grouped
// by window into the tile's own range of a pair buffer, with the window
// offsets in a row of `pre`, and k_remap_windows then builds each window of
// LR in LDS and writes it out whole.  The window is the largest that still
// gives 256 windows (one workgroup each), down to 2^12 tags.
constexpr int WIN_SHIFT = 15;  // the largest window
constexpr int WIN = 1 << WIN_SHIFT;
constexpr int MIN_WIN_SHIFT = 12;
constexpr int MAX_WINDOWS = 1024;       // windows of one sort (LDS counters of the pass)
constexpr int WIN_MAX_TILES = 6144;     // tiles whose runs a window workgroup keeps in LDS
// Shorter lists keep the scattered stores (their LR stays in the L2s).
constexpr int64_t WIN_MIN_N = 1 << 20;

// One pass over a tile (see the top of this file).  WINDOWS: the last pass
// of a long endpoint sort, which also writes the tile's remap pairs.
template <int MODE, int ROUNDS, bool WINDOWS, int BITS>
__device__ __forceinline__ void os_pass(const uint64_t* __restrict__ items_in,
                                        const int32_t* __restrict__ L,
                                        const int32_t* __restrict__ R, int64_t N, int64_t n,
                                        int shift, int bits, const uint32_t* __restrict__ hist,
                                        uint64_t* status, uint64_t* status_next,
                                        Chains ch, uint32_t* abort_word,
                                        uint64_t* __restrict__ items_out,
                                        int32_t* __restrict__ LR, uint64_t* __restrict__ pairs,
                                        uint16_t* __restrict__ pre, int nwin, int win_shift) {
  constexpr int TILE = WG * ROUNDS;
  // per wave and digit: the wave's count, then the tile-local slot of its
  // first item of that digit
  // (16 bits: a tile has fewer than 2^16 items, so that a workgroup over a
  // large tile takes under half of a CU's LDS and two share a CU)
  __shared__ uint16_t wave_cnt[WG / 64][RADIX];
  // per digit: global slot minus tile-local slot of the digit's items
  __shared__ uint32_t shift_to_global[RADIX];
  __shared__ uint32_t tmp[WG / 64];
  __shared__ uint64_t s_item[TILE];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wcnt[WINDOWS ? MAX_WINDOWS : 1];  // pairs per window, then offsets

  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int chain = (int)(blockIdx.x % (unsigned)ch.nchains);
  if (threadIdx.x == 0) s_tile = atomicAdd(ch.tickets + chain, 1u);
  // the digit's total, and its items in the earlier ranges
  uint32_t total = 0, below = 0;
#pragma unroll
  for (int c = 0; c < HCOPIES; ++c) {
    const uint32_t h = hist[c * HSTRIDE + threadIdx.x];
    total += h;
    below += c < chain ? h : 0u;
  }
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) wave_cnt[w][threadIdx.x] = 0;
  if (WINDOWS) {
#pragma unroll
    for (int i = 0; i < MAX_WINDOWS / WG; ++i) s_wcnt[i * WG + threadIdx.x] = 0;
  }
  // digit offsets of this pass: exclusive scan of the digit totals, plus
  // the digit's items in the earlier ranges
  uint32_t digit_base;
  block_exclusive_scan(total, tmp, digit_base);
  digit_base += below;
  // tiles of a range in the order its workgroups started
  const int64_t first = (int64_t)chain * ch.range_tiles;
  const int64_t tile = first + (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_tile);
  const int64_t range_end = first + ch.range_tiles < ch.num_tiles ? first + ch.range_tiles
                                                                   : ch.num_tiles;
  if (tile >= range_end) return;  // the whole workgroup: a padding ticket
  const int64_t tile0 = tile * TILE;
  const uint32_t mask = (1u << bits) - 1u;
  if (status_next) status_next[tile * RADIX + threadIdx.x] = 0;  // for the next pass

  // this wave's items: tile0 + wave * 64 * ROUNDS + round * 64 + lane, the
  // first nval of them inside the list (all of them but in the last tile)
  const int64_t wbase = tile0 + (int64_t)wave * (64 * ROUNDS);
  const bool full = tile0 + TILE <= N;  // workgroup-uniform
  const int nval = full ? 64 * ROUNDS
                        : (N - wbase <= 0 ? 0
                                          : (N - wbase >= 64 * ROUNDS ? 64 * ROUNDS
                                                                      : (int)(N - wbase)));
  // the items (position << 32 | tag) as positions in registers and tags:
  // from the queries or a list's tags the tag is the item's own index; the
  // tags of general items wait in the first half of s_item while the tile
  // is ranked (in registers they pushed the kernel past its register
  // budget) and come back before it is staged
  constexpr bool OWN_TAG = MODE != ITEMS;
  uint32_t qpos[ROUNDS];
  uint32_t tag[OWN_TAG ? 1 : ROUNDS];
  uint32_t* const s_tag = reinterpret_cast<uint32_t*>(s_item) + wave * (64 * ROUNDS) + lane;
  auto key_hi = [&](int rd) -> uint32_t { return qpos[rd]; };
  auto item_at = [&](int rd) -> uint64_t {
    if constexpr (OWN_TAG)
      return ((uint64_t)qpos[rd] << 32) | (uint32_t)(wbase + rd * 64 + lane);
    else return ((uint64_t)qpos[rd] << 32) | tag[rd];
  };
  // each item's rank among the wave's items of its digit so far (below
  // 2^16: two to a register, so that the items stay in registers)
  uint32_t rank2[(ROUNDS + 1) / 2];
  // all loads of the tile first, so they are in flight together (a full
  // tile reads at fixed offsets from one base, no index clamping)
  if constexpr (MODE == QUERIES) {
    if (full) {
      // item j = wbase + 64 rd + lane is an end of query j / 2 (wbase even)
      const int32_t* src = ((lane & 1) ? R : L) + (wbase >> 1) + (lane >> 1);
#pragma unroll
      for (int rd = 0; rd < ROUNDS; ++rd) qpos[rd] = (uint32_t)src[rd * 32];
    } else {
#pragma unroll
      for (int rd = 0; rd < ROUNDS; ++rd)
        qpos[rd] = (uint32_t)load_raw<MODE>(items_in, L, R, N, wbase + rd * 64 + lane);
    }
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd)
      qpos[rd] = (uint32_t)(finish_item<MODE>(qpos[rd], n, wbase + rd * 64 + lane) >> 32);
  } else {
    // the wave's items through one buffer resource over its part of the
    // list: reads past the list's end return zero, so full and partial
    // tiles take the same loads, each a lane offset plus a constant from one
    // scalar base (per-load 64-bit addresses pushed the kernel past its
    // register budget)
    const int64_t wuni = tile0 + (int64_t)__builtin_amdgcn_readfirstlane(wave) * (64 * ROUNDS);
    const int64_t wlen = N - wuni;
    const int bytes = wlen <= 0 ? 0 : (wlen >= 64 * ROUNDS ? 64 * ROUNDS * 8 : (int)wlen * 8);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint64_t*>(items_in + (wlen > 0 ? wuni : 0)), (short)0, bytes, 0x00020000);
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, rd * 512, 0);
      if constexpr (MODE == E_TAGS) {
        qpos[rd] = v[0];  // the list's low half becomes the key
      } else {
        qpos[rd] = v[1];
        s_tag[rd * 64] = v[0];
      }
    }
  }
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const uint32_t d = __builtin_amdgcn_ubfe(key_hi(rd), (uint32_t)shift, (uint32_t)bits);
    // lanes holding digit d: those whose every digit bit equals this lane's,
    // i.e. outside the OR over the bits of (ballot of the bit) XOR (own bit
    // spread over the word); bits above `bits` are zero in every lane and
    // add nothing
    const uint64_t match =
        same_digit_lanes<BITS>(d, full ? ~0ull : ballot(rd * 64 + lane < nval));
    const uint32_t before = wave_cnt[wave][d];
    // + this lane's predecessors in the group (set bits of match below it)
    const uint32_t r = before + __builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(match >> 32),
                                    __builtin_amdgcn_mbcnt_lo((uint32_t)match, 0u));
    rank2[rd >> 1] = (rd & 1) ? (rank2[rd >> 1] | (r << 16)) : r;
    // every lane of a digit group stores the same new count (an invalid
    // lane's group holds the valid lanes of its digit, or none)
    wave_cnt[wave][d] = (uint16_t)(before + (uint32_t)__popcll(match));
  }
  __syncthreads();

  // thread d: this tile's count of digit d, published at once so that later
  // tiles can go on; then the tile is staged in LDS in digit order while
  // earlier tiles publish theirs
  const int d = threadIdx.x;
  uint32_t run = 0;  // items of digit d in this tile; waves' offsets in place
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) {
    const uint32_t c = wave_cnt[w][d];
    wave_cnt[w][d] = (uint16_t)run;
    run += c;
  }
  // this tile's row of status words (a wave-uniform base; digit d's word
  // is row[d], a 32-bit offset, so that no 64-bit address stays live)
  uint64_t* const row = status + tile * RADIX;
  // digits at or above 2^bits occur in no item: their threads neither
  // publish nor look back (no tile ever reads those words)
  const bool used_digit = d <= (int)mask;
  if (used_digit) store_status(row + d, (tile == first ? ST_INC : ST_AGG) | run);
  uint32_t local_start;  // tile-local slot of digit d's first item
  block_exclusive_scan(run, tmp, local_start);
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) wave_cnt[w][d] = (uint16_t)(wave_cnt[w][d] + local_start);
  if constexpr (!OWN_TAG) {
    // back from LDS; the barrier below separates these reads from the
    // staging stores into s_item
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) tag[rd] = s_tag[rd * 64];
  }
  __syncthreads();
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    if (full || rd * 64 + lane < nval) {
      const uint32_t dd = __builtin_amdgcn_ubfe(key_hi(rd), (uint32_t)shift, (uint32_t)bits);
      const uint32_t lp = wave_cnt[wave][dd] + ((rank2[rd >> 1] >> ((rd & 1) * 16)) & 0xFFFFu);
      if (lp < (uint32_t)TILE) s_item[lp] = item_at(rd);  // always true for consistent ranks
    }
  }

  // digit d's count in all earlier tiles
  const uint64_t before =
      tile > first && used_digit ? look_back(status, tile, first, d, abort_word) : 0;
  if (tile > first && used_digit) store_status(row + d, ST_INC | (before + run));
  shift_to_global[d] = digit_base + (uint32_t)before - local_start;
  __syncthreads();

  const int64_t tile_n = N - tile0 < TILE ? N - tile0 : TILE;
  int32_t* pos_out = reinterpret_cast<int32_t*>(items_out);
  if (!WINDOWS) {
    for (int t = threadIdx.x; t < tile_n; t += WG) {
      const uint64_t x = s_item[t];
      const uint32_t dst = shift_to_global[digit_bits(x, shift, bits)] + (uint32_t)t;
      if ((int64_t)dst < N) {  // always true for consistent counts
        if (LR) {
          // last pass of the endpoint sort: the remap, LR[tag] = slot
          // (minus one for a right end), written here directly, and the
          // position alone (the tag is used up)
          pos_out[dst] = (int32_t)(x >> 32);
          const uint32_t g = (uint32_t)x;
          if ((int64_t)g < N) LR[g] = (g & 1u) ? (int32_t)dst - 1 : (int32_t)dst;
        } else {
          items_out[dst] = x;
        }
      }
    }
    return;
  }
  // ---- WINDOWS: the items as above, and each item's (tag, slot) pair
  // ranked inside its window by an LDS counter ----
  uint64_t pr[ROUNDS];     // (tag << 32) | slot
  // window << 16 | rank inside the window (both found once: a second
  // shift by the run-time window width pushed the kernel into scratch);
  // ~0 = not placed
  uint32_t pr_at[ROUNDS];
#pragma unroll
  for (int i = 0; i < ROUNDS; ++i) {
    const int t = i * WG + threadIdx.x;
    pr[i] = 0;
    pr_at[i] = ~0u;
    if (t >= tile_n) continue;
    const uint64_t x = s_item[t];
    const uint32_t dst = shift_to_global[digit_bits(x, shift, bits)] + (uint32_t)t;
    if ((int64_t)dst >= N) continue;  // never, for consistent counts
    pos_out[dst] = (int32_t)(x >> 32);  // the position alone (the tag is used up)
    const uint32_t g = (uint32_t)x;
    const uint32_t w = min(g >> win_shift, (uint32_t)nwin - 1u);
    pr[i] = ((uint64_t)g << 32) | dst;
    pr_at[i] = (w << 16) | atomicAdd(&s_wcnt[w], 1u);
  }
  __syncthreads();  // counts final; s_item free again
  // window offsets inside the tile: thread u scans windows 4u .. 4u + 3
  constexpr int WPT = MAX_WINDOWS / WG;
  uint32_t c[WPT], sum = 0;
#pragma unroll
  for (int k = 0; k < WPT; ++k) {
    c[k] = s_wcnt[threadIdx.x * WPT + k];
    sum += c[k];
  }
  uint32_t off;
  block_exclusive_scan(sum, tmp, off);
  // start of window w's run in this tile: pre[w * num_tiles + tile], window
  // by window, so that a window's workgroup reads one contiguous column
  // (column nwin: the end of the last run)
  const int64_t num_tiles = (N + TILE - 1) / TILE;
#pragma unroll
  for (int k = 0; k < WPT; ++k) {
    const int w = threadIdx.x * WPT + k;
    if (w <= nwin) pre[w * num_tiles + tile] = (uint16_t)off;
    s_wcnt[w] = off;
    off += c[k];
  }
  if (threadIdx.x == WG - 1 && nwin == MAX_WINDOWS) pre[nwin * num_tiles + tile] = (uint16_t)off;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ROUNDS; ++i) {
    if (pr_at[i] == ~0u) continue;
    const uint32_t at = s_wcnt[pr_at[i] >> 16] + (pr_at[i] & 0xFFFFu);
    if (at < (uint32_t)TILE) s_item[at] = pr[i];  // always true
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ROUNDS; ++i) {
    const int t = i * WG + threadIdx.x;
    if (t < tile_n) pairs[tile0 + t] = s_item[t];
  }
}

// (at most 128 VGPRs: two 8-wave workgroups share a CU, with their LDS)
template <int MODE, int ROUNDS, int BITS>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void k_os_pass(const uint64_t* __restrict__ items_in,
                                                const int32_t* __restrict__ L,
                                                const int32_t* __restrict__ R, int64_t N,
                                                int64_t n, int shift, int bits,
                                                const uint32_t* __restrict__ hist,
                                                uint64_t* status, uint64_t* status_next,
                                                Chains ch, uint32_t* abort_word,
                                                uint64_t* __restrict__ items_out,
                                                int32_t* __restrict__ LR) {
  os_pass<MODE, ROUNDS, false, BITS>(items_in, L, R, N, n, shift, bits, hist, status,
                                     status_next, ch, abort_word, items_out, LR, nullptr,
                                     nullptr, 1, WIN_SHIFT);
}

// Launch of a pass whose digits have `bits` bits: the ranking takes one
// ballot per digit bit, unrolled for the widths digit splits produce (the
// others rank all RADIX_BITS bits, those above the digit zero everywhere).
template <int MODE, int ROUNDS>
hipError_t launch_pass(dim3 grid, hipStream_t stream, int bits, const uint64_t* in,
                       const int32_t* L, const int32_t* R, int64_t N, int64_t n, int shift,
                       const uint32_t* hist, uint64_t* st, uint64_t* st_next, Chains ch,
                       uint32_t* abort_word, uint64_t* dst, int32_t* lr) {
  switch (bits) {
    case RADIX_BITS - 2:
      return launch(k_os_pass<MODE, ROUNDS, RADIX_BITS - 2>, grid, dim3(WG), 0, stream, in, L, R,
                    N, n, shift, bits, hist, st, st_next, ch, abort_word, dst, lr);
    case RADIX_BITS - 1:
      return launch(k_os_pass<MODE, ROUNDS, RADIX_BITS - 1>, grid, dim3(WG), 0, stream, in, L, R,
                    N, n, shift, bits, hist, st, st_next, ch, abort_word, dst, lr);
    default:
      return launch(k_os_pass<MODE, ROUNDS, RADIX_BITS>, grid, dim3(WG), 0, stream, in, L, R, N,
                    n, shift, bits, hist, st, st_next, ch, abort_word, dst, lr);
  }
}

// The last pass of a long endpoint sort (4096-item tiles), remap through
// LR windows.  Its own kernel, so that the registers the pairs take do not
// lower the occupancy of the other passes.
template <int MODE, int BITS>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void k_os_pass_windows(
    const uint64_t* __restrict__ items_in, const int32_t* __restrict__ L,
    const int32_t* __restrict__ R, int64_t N, int64_t n, int shift, int bits,
    const uint32_t* __restrict__ hist, uint64_t* status, Chains ch, uint32_t* abort_word,
    uint64_t* __restrict__ items_out, uint64_t* __restrict__ pairs, uint16_t* __restrict__ pre,
    int nwin, int win_shift) {
  os_pass<MODE, BIG_ROUNDS, true, BITS>(items_in, L, R, N, n, shift, bits, hist, status, nullptr,
                                        ch, abort_word, items_out, nullptr, pairs, pre, nwin,
                                        win_shift);
}

template <int MODE>
hipError_t launch_win_pass(dim3 grid, hipStream_t stream, const uint64_t* in, const int32_t* L,
                           const int32_t* R, int64_t N, int64_t n, int shift, int bits,
                           const uint32_t* hist, uint64_t* st, Chains ch,
                           uint32_t* abort_word, uint64_t* dst, uint64_t* pairs, uint16_t* pre,
                           int nwin, int win_shift) {
  switch (bits) {
    case RADIX_BITS - 2:
      return launch(k_os_pass_windows<MODE, RADIX_BITS - 2>, grid, dim3(WG), 0, stream, in, L, R,
                    N, n, shift, bits, hist, st, ch, abort_word, dst, pairs, pre, nwin, win_shift);
    case RADIX_BITS - 1:
      return launch(k_os_pass_windows<MODE, RADIX_BITS - 1>, grid, dim3(WG), 0, stream, in, L, R,
                    N, n, shift, bits, hist, st, ch, abort_word, dst, pairs, pre, nwin, win_shift);
    default:
      return launch(k_os_pass_windows<MODE, RADIX_BITS>, grid, dim3(WG), 0, stream, in, L, R, N,
                    n, shift, bits, hist, st, ch, abort_word, dst, pairs, pre, nwin, win_shift);
  }
}

// LR window w (tags [w << win_shift, (w + 1) << win_shift)) from the pairs
// of every tile: tile j's run for the window is pairs[j * T + pre[w][j] ..
// j * T + pre[w + 1][j]) (T items per tile).  The runs' bounds (two contiguous columns of pre) go to
// LDS first; then each wave takes 64 / lpt tiles per load, lpt lanes per
// tile (lpt: a power of two near the mean run length), U such loads in
// flight per lane, and writes the entries into the LDS image of the window;
// the image is written to LR with coalesced stores.  Every tag of the
// window occurs in exactly one pair, so the image is complete.
// (At 2q = 2e7 it fetches 1.25x the pair bytes from HBM; with the windows
// spread over the XCDs it fetched 3.6x.)
constexpr int AWG = 1024;  // threads of a window workgroup
constexpr int WIN_TILE = BIG_TILE;
__global__ __launch_bounds__(AWG) void k_remap_windows(const uint64_t* __restrict__ pairs,
                                                       const uint16_t* __restrict__ pre,
                                                       int64_t num_tiles, int nwin, int win_shift,
                                                       int lpt_shift,
                                                       int64_t N, int32_t* __restrict__ LR) {
  __shared__ int32_t win[WIN];
  __shared__ uint32_t runs[WIN_MAX_TILES];  // start | end << 16
  // XCD x takes the x-th contiguous range of windows: neighbouring windows
  // run together on one XCD and share, in its L2, the cache lines where
  // their runs meet
  const int64_t wx = xcd_tile(nwin);
  if (wx < 0) return;  // whole workgroup
  const int w = (int)wx;
  const int64_t wbase = (int64_t)w << win_shift;
  const int wsize = 1 << win_shift;
  {
    constexpr int PER = (WIN_MAX_TILES + AWG - 1) / AWG;
    const uint16_t* c0 = pre + (int64_t)w * num_tiles;
    const uint16_t* c1 = c0 + num_tiles;
    uint32_t r[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t j = threadIdx.x + (int64_t)k * AWG;
      r[k] = j < num_tiles ? (uint32_t)c0[j] | ((uint32_t)c1[j] << 16) : 0u;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t j = threadIdx.x + (int64_t)k * AWG;
      if (j < num_tiles) runs[j] = r[k];
    }
  }
  __syncthreads();
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int lpt = 1 << lpt_shift;                   // lanes per tile
  const int sub = lane & (lpt - 1), tj = lane >> lpt_shift;
  const int64_t per_load = 64 >> lpt_shift;         // tiles per wave load
  auto put = [&](uint64_t x) {
    const uint32_t t = (uint32_t)(x >> 32), slot = (uint32_t)x;
    const int64_t at = (int64_t)t - wbase;
    if (at >= 0 && at < wsize) win[at] = (t & 1u) ? (int32_t)slot - 1 : (int32_t)slot;
  };
  constexpr int U = 8;
  const int64_t stride = (AWG / 64) * per_load;     // tiles per round of the block's waves
  for (int64_t j0 = wave * per_load; j0 < num_tiles; j0 += stride * U) {
    uint64_t v[U];
    uint32_t se[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * stride + tj;
      se[u] = j < num_tiles ? runs[j] : 0u;
      const uint32_t s0 = se[u] & 0xFFFFu, e0 = se[u] >> 16;
      v[u] = s0 + sub < e0 ? pairs[j * WIN_TILE + s0 + sub] : ~0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (v[u] != ~0ull) put(v[u]);
    // runs longer than lpt (about a quarter of them): their next lpt
    // entries, all of the round's loads at once
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * stride + tj;
      const uint32_t s0 = se[u] & 0xFFFFu, e0 = se[u] >> 16;
      v[u] = s0 + lpt + sub < e0 ? pairs[j * WIN_TILE + s0 + lpt + sub] : ~0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (v[u] != ~0ull) put(v[u]);
    // runs longer than 2 lpt (rare)
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * stride + tj;
      const uint32_t s0 = se[u] & 0xFFFFu, e0 = se[u] >> 16;
      for (uint32_t i = s0 + 2 * lpt + sub; i < e0; i += lpt) put(pairs[j * WIN_TILE + i]);
    }
  }
  __syncthreads();
  const int64_t len = N - wbase < wsize ? N - wbase : wsize;
  for (int64_t i = threadIdx.x; i < len; i += AWG) LR[wbase + i] = win[i];
}

// Remap writes from (tag, slot) items ordered by the top bits of the tag.
// If the bucketing sweep gave up (abort word set), every entry of LR is -1.
__global__ __launch_bounds__(WG) void k_remap_apply(const uint64_t* __restrict__ items,
                                                    int64_t N, int32_t* __restrict__ LR,
                                                    int64_t num_chunks,
                                                    const uint32_t* __restrict__ abort_word) {
  const int64_t chunk = xcd_tile(num_chunks);
  if (chunk < 0) return;
  const bool failed = *abort_word != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t j = chunk * (4 * WG) + i * WG + threadIdx.x;
    if (j < N) {
      if (failed) {
        LR[j] = -1;
        continue;
      }
      const uint64_t x = items[j];
      const uint32_t t = (uint32_t)(x >> 32), s = (uint32_t)x;
      if ((int64_t)t < N) LR[t] = (t & 1u) ? (int32_t)s - 1 : (int32_t)s;
    }
  }
}

// Split / join of the packed sorted list (for the single-stage entry points).
// If the sort gave up (abort word set), every position and tag is -1.
__global__ __launch_bounds__(WG) void k_unpack(const uint64_t* __restrict__ E, int64_t N,
                                               int32_t* __restrict__ pos,
                                               int32_t* __restrict__ tag,
                                               const uint32_t* __restrict__ abort_word) {
  const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (j < N) {
    const bool failed = *abort_word != 0;
    pos[j] = failed ? -1 : (int32_t)(E[j] >> 32);
    tag[j] = failed ? -1 : (int32_t)(uint32_t)E[j];
  }
}
__global__ __launch_bounds__(WG) void k_pack(const int32_t* __restrict__ pos,
                                             const int32_t* __restrict__ tag, int64_t N,
                                             uint64_t* __restrict__ E) {
  const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (j < N) E[j] = ((uint64_t)(uint32_t)pos[j] << 32) | (uint32_t)tag[j];
}

int bit_length(uint64_t x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

struct SortLayout {
  int64_t N, num_tiles, hist_groups;
  int64_t range_tiles;  // tiles per chain's range; a pass launches CHAINS * range_tiles groups
  int hist_per_group;
  int rounds;  // items per thread of a tile
  int nwin;    // LR windows of the remap, 0 = scattered remap stores
  int win_shift;  // log2 of the tags per window
  size_t off_items, off_status0, off_status1, off_hist, off_tickets, off_abort, off_pre, bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout for N items (the endpoint sort has N = 2q).
SortLayout sort_layout_items(int64_t N) {
  SortLayout s{};
  s.N = N;
  s.rounds = rounds_for(N);
  const int64_t tile = (int64_t)WG * s.rounds;
  s.num_tiles = (s.N + tile - 1) / tile;
  s.hist_per_group = hist_tiles(s.num_tiles);
  s.hist_groups = (s.num_tiles + s.hist_per_group - 1) / s.hist_per_group;
  // ranges of whole histogram groups, so that a group counts into one copy
  const int64_t groups_per_range = (s.hist_groups + CHAINS - 1) / CHAINS;
  s.range_tiles = groups_per_range * s.hist_per_group;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  s.off_items = take(sizeof(uint64_t) * (size_t)s.N);
  s.off_status0 = take(sizeof(uint64_t) * (size_t)RADIX * (size_t)s.num_tiles);
  s.off_status1 = take(sizeof(uint64_t) * (size_t)RADIX * (size_t)s.num_tiles);
  s.off_hist = take(sizeof(uint32_t) * (size_t)HCOPIES * HSTRIDE);
  s.off_tickets = take(sizeof(uint32_t) * (CHAINS + MAX_PASSES));
  s.off_abort = take(sizeof(uint32_t));
  s.win_shift = WIN_SHIFT;
  while (s.win_shift > MIN_WIN_SHIFT && (N >> s.win_shift) < 256) --s.win_shift;
  const int64_t nwin = (N + ((int64_t)1 << s.win_shift) - 1) >> s.win_shift;
  s.nwin = N >= WIN_MIN_N && s.rounds == BIG_ROUNDS && s.num_tiles <= WIN_MAX_TILES &&
                   nwin <= MAX_WINDOWS
               ? (int)nwin
               : 0;
  s.off_pre = take(sizeof(uint16_t) * (size_t)(s.nwin + 1) * (size_t)s.num_tiles);
  s.bytes = o;
  return s;
}

struct SortBufs {
  uint64_t* items;
  uint64_t* status[2];
  uint32_t *hist, *tickets, *abort_word;
  uint16_t* pre;
};

SortBufs sort_bufs(const SortLayout& lay, void* ws) {
  char* base = static_cast<char*>(ws);
  SortBufs b;
  b.items = reinterpret_cast<uint64_t*>(base + lay.off_items);
  b.status[0] = reinterpret_cast<uint64_t*>(base + lay.off_status0);
  b.status[1] = reinterpret_cast<uint64_t*>(base + lay.off_status1);
  b.hist = reinterpret_cast<uint32_t*>(base + lay.off_hist);
  b.tickets = reinterpret_cast<uint32_t*>(base + lay.off_tickets);
  b.abort_word = reinterpret_cast<uint32_t*>(base + lay.off_abort);
  b.pre = reinterpret_cast<uint16_t*>(base + lay.off_pre);
  return b;
}

hipError_t clear(const SortLayout& lay, const SortBufs& b, hipStream_t stream) {
  const int64_t status_words = lay.num_tiles * RADIX;
  const int64_t grid = status_words / (4 * WG) + 1;
  return launch(k_os_clear, dim3((unsigned)(grid < 1024 ? grid : 1024)), dim3(WG), 0, stream,
                b.hist, b.tickets, b.abort_word, g_abort_preset.load(), b.status[0],
                status_words);
}

// A whole sort: clear, histograms of every pass, then the passes.  Passes
// alternate between the scratch buffer and `out` so the last lands in `out`.
template <int MODE, int ROUNDS>
hipError_t onesweep_r(const uint64_t* src, const int32_t* L, const int32_t* R, int64_t N,
                      int64_t n, const Digits& dg, const SortLayout& lay, const SortBufs& b,
                      uint64_t* out, int32_t* LR, uint64_t* pairs, hipStream_t stream) {
  // the remap through LR windows: a long list, 4096-item tiles, and pair scratch
  const bool windows = LR && pairs && lay.nwin > 0 && ROUNDS == BIG_ROUNDS;
  RMQ_TRY(clear(lay, b, stream));
  RMQ_TRY(launch(k_os_hist<MODE, ROUNDS>, dim3((unsigned)lay.hist_groups), dim3(WG), 0, stream,
                 src, L, R, N, n, dg, lay.hist_per_group, lay.range_tiles, b.hist));
  const uint64_t* in = src;
  for (int p = 0; p < dg.passes; ++p) {
    const bool to_out = ((dg.passes - 1 - p) % 2) == 0;
    uint64_t* dst = to_out ? out : b.items;
    uint64_t* st = b.status[p & 1];
    uint64_t* st_next = p + 1 < dg.passes ? b.status[(p + 1) & 1] : nullptr;
    int32_t* lr = p + 1 < dg.passes ? nullptr : LR;
    const Chains ch = p == 0 ? first_pass_chains(b.tickets, lay.range_tiles, lay.num_tiles)
                             : one_chain(b.tickets + CHAINS + p, lay.num_tiles);
    const dim3 grid((unsigned)(ch.nchains * ch.range_tiles)), block(WG);
    if (windows && p + 1 == dg.passes) {
      if (p == 0)
        RMQ_TRY((launch_win_pass<MODE>)(grid, stream, in, L, R, N, n, dg.shift[p], dg.bits[p],
                                        b.hist + p * RADIX, st, ch, b.abort_word,
                                        dst, pairs, b.pre, lay.nwin, lay.win_shift));
      else
        RMQ_TRY((launch_win_pass<ITEMS>)(grid, stream, in, L, R, N, n, dg.shift[p], dg.bits[p],
                                         b.hist + p * RADIX, st, ch, b.abort_word,
                                         dst, pairs, b.pre, lay.nwin, lay.win_shift));
      // lanes per tile: the power of two at or above the mean run length
      // (tile items * window tags / N pairs), between 4 and 64
      const double mean_run = (double)WIN_TILE * (double)(1 << lay.win_shift) / (double)N;
      int lpt_shift = 2;
      while (lpt_shift < 6 && (double)(1 << lpt_shift) < mean_run) ++lpt_shift;
      RMQ_TRY(launch(k_remap_windows, dim3((unsigned)xcd_grid(lay.nwin)), dim3(AWG), 0, stream,
                     static_cast<const uint64_t*>(pairs), static_cast<const uint16_t*>(b.pre),
                     lay.num_tiles, lay.nwin, lay.win_shift, lpt_shift, N, LR));
    } else if (p == 0)
      RMQ_TRY((launch_pass<MODE, ROUNDS>)(grid, stream, dg.bits[p], in, L, R, N, n, dg.shift[p],
                                        b.hist + p * RADIX, st, st_next, ch,
                                        b.abort_word, dst, lr));
    else
      RMQ_TRY((launch_pass<ITEMS, ROUNDS>)(grid, stream, dg.bits[p], in, L, R, N, n, dg.shift[p],
                                         b.hist + p * RADIX, st, st_next, ch,
                                         b.abort_word, dst, lr));
    in = dst;
  }
  return hipSuccess;
}

template <int MODE>
hipError_t onesweep(const uint64_t* src, const int32_t* L, const int32_t* R, int64_t N, int64_t n,
                    const Digits& dg, const SortLayout& lay, const SortBufs& b, uint64_t* out,
                    int32_t* LR, uint64_t* pairs, hipStream_t stream) {
  switch (lay.rounds) {
    case R1K: return onesweep_r<MODE, R1K>(src, L, R, N, n, dg, lay, b, out, LR, pairs, stream);
    case R2K: return onesweep_r<MODE, R2K>(src, L, R, N, n, dg, lay, b, out, LR, pairs, stream);
    default:
      return onesweep_r<MODE, BIG_ROUNDS>(src, L, R, N, n, dg, lay, b, out, LR, pairs, stream);
  }
}

// One sweep on the top bits of the tag (the stand-alone remap's bucketing).
template <int ROUNDS>
hipError_t tag_sweep(const uint64_t* E, const SortLayout& lay, const SortBufs& b,
                     const Digits& dg, uint64_t* sorted, hipStream_t stream) {
  RMQ_TRY(clear(lay, b, stream));
  RMQ_TRY(launch(k_os_hist<E_TAGS, ROUNDS>, dim3((unsigned)lay.hist_groups), dim3(WG), 0, stream,
                 E, static_cast<const int32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                 lay.N, (int64_t)0, dg, lay.hist_per_group, lay.range_tiles, b.hist));
  const Chains ch = first_pass_chains(b.tickets, lay.range_tiles, lay.num_tiles);
  RMQ_TRY((launch_pass<E_TAGS, ROUNDS>)(dim3((unsigned)(CHAINS * lay.range_tiles)), stream,
                                       dg.bits[0], E, nullptr, nullptr, lay.N, 0, dg.shift[0],
                                       b.hist, b.status[0], nullptr, ch, b.abort_word, sorted,
                                       nullptr));
  return hipSuccess;
}

SortLayout sort_layout(int64_t q) { return sort_layout_items(2 * q); }

}  // namespace

size_t sort_workspace_bytes(int64_t q) { return q > 0 ? sort_layout(q).bytes : 0; }

size_t sort_pairs_workspace_bytes(int64_t N) { return N > 0 ? sort_layout_items(N).bytes : 0; }

hipError_t launch_sort_pairs(const uint64_t* items, int64_t N, int key_bits, uint64_t* out,
                             void* ws, size_t ws_bytes, hipStream_t stream) {
  if (N <= 0) return hipSuccess;
  const SortLayout lay = sort_layout_items(N);
  if (ws_bytes < lay.bytes || key_bits < 1 || key_bits > 32) return hipErrorInvalidValue;
  const SortBufs b = sort_bufs(lay, ws);
  return onesweep<ITEMS>(items, nullptr, nullptr, N, 0, split_digits(0, key_bits), lay, b, out,
                         nullptr, nullptr, stream);
}

hipError_t launch_sort_endpoints(const int32_t* L, const int32_t* R, int64_t q, int64_t n,
                                 uint64_t* E, int32_t* LR, uint64_t* pair_scratch, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const SortLayout lay = sort_layout(q);
  if (ws_bytes < lay.bytes) return hipErrorInvalidValue;
  const SortBufs b = sort_bufs(lay, ws);
  const int nbits = n > 1 ? bit_length((uint64_t)(n - 1)) : 1;
  return onesweep<QUERIES>(nullptr, L, R, lay.N, n, split_digits(0, nbits), lay, b, E, LR,
                           pair_scratch, stream);
}

hipError_t launch_remap(const uint64_t* E, int64_t q, int32_t* LR, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const SortLayout lay = sort_layout(q);
  if (ws_bytes < lay.bytes) return hipErrorInvalidValue;
  const SortBufs b = sort_bufs(lay, ws);
  // one sweep on the top (at most 8) bits of the tag; its output goes to the
  // scratch item buffer (E itself is still needed by the contraction)
  const int tbits = lay.N > 1 ? bit_length((uint64_t)(lay.N - 1)) : 1;
  const int top = tbits > RADIX_BITS ? RADIX_BITS : tbits;
  Digits dg{};
  dg.passes = 1;
  dg.shift[0] = tbits - top;
  dg.bits[0] = top;
  uint64_t* sorted = b.items;
  switch (lay.rounds) {
    case R1K: RMQ_TRY(tag_sweep<R1K>(E, lay, b, dg, sorted, stream)); break;
    case R2K: RMQ_TRY(tag_sweep<R2K>(E, lay, b, dg, sorted, stream)); break;
    default: RMQ_TRY(tag_sweep<BIG_ROUNDS>(E, lay, b, dg, sorted, stream)); break;
  }
  const int64_t chunks = (lay.N + 4 * WG - 1) / (4 * WG);
  RMQ_TRY(launch(k_remap_apply, dim3((unsigned)xcd_grid(chunks)), dim3(WG), 0, stream, sorted,
                 lay.N, LR, chunks, static_cast<const uint32_t*>(b.abort_word)));
  return hipSuccess;
}

const uint32_t* sort_abort_word(const void* ws, int64_t q) {
  return sort_pairs_abort_word(ws, 2 * q);
}

const uint32_t* sort_pairs_abort_word(const void* ws, int64_t N) {
  if (!ws || N <= 0) return nullptr;
  return reinterpret_cast<const uint32_t*>(static_cast<const char*>(ws) +
                                           sort_layout_items(N).off_abort);
}

hipError_t launch_unpack_endpoints(const uint64_t* E, int64_t q, int32_t* pos, int32_t* tag,
                                   const uint32_t* abort_word, hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t N = 2 * q;
  RMQ_TRY(launch(k_unpack, dim3((unsigned)((N + WG - 1) / WG)), dim3(WG), 0, stream, E, N, pos,
                 tag, abort_word));
  return hipSuccess;
}

hipError_t launch_pack_endpoints(const int32_t* pos, const int32_t* tag, int64_t q, uint64_t* E,
                                 hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t N = 2 * q;
  RMQ_TRY(launch(k_pack, dim3((unsigned)((N + WG - 1) / WG)), dim3(WG), 0, stream, pos, tag, N,
                 E));
  return hipSuccess;
}

}  // namespace rmq
