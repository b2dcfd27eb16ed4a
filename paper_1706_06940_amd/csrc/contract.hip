// Contraction (Section 3.1 step 2).
//
// With the M = 2q endpoints sorted (E_0 <= ... <= E_{M-1}), A_Q[s] is the min
// key over the CLOSED area A[E_s .. E_{s+1}], s = 0 .. M-2.  Split each area
// into its half-open part [E_s, E_{s+1}) and its closing element E_{s+1}:
//   A_Q[s] = min(min over [E_s, E_{s+1}), key(E_{s+1})),
// where the half-open parts of consecutive areas tile [E_0, E_{M-1}) and are
// empty for repeated endpoints (then A_Q[s] = key(E_s)).
//
// A is cut into tiles of T = 1024 elements.
// k_tiles_search / k_tiles_scatter: tile_start[t] = first slot whose
//   endpoint is >= t * T (by binary search per tile for sparse lists, by
//   streaming the list for dense ones); and A_Q[j - 1] = +inf for every slot
//   j that is the first in its tile -- that area reaches into the tile from
//   an earlier one, so it may be finished by atomicMin from several waves.
// k_contract (one streaming pass over A): each wave walks a run of up to 63
//   consecutive tiles, the next tile's values and first endpoints in flight
//   while it works on the current one, and carries the area that is still
//   open at a tile's end into the next tile (no barrier: waves share nothing).
//   * a tile without endpoints lies inside the open area: each lane keeps
//     its min over a run of such tiles (32-bit compares, leftmost on ties),
//     and the wave's min over the run joins the carried value when the run
//     ends;
//   * otherwise the tile is staged in LDS, its endpoints set head bits, and
//     lane l takes elements 16l .. 16l+15 with a running min that restarts
//     at heads; a segmented min-scan over the lanes' last runs gives each
//     lane the min of the run coming in from the lanes before it.  Then one
//     lane per endpoint slot j reads off area j-1: the key at E_j, the
//     running min just before E_j, and the incoming run when E_{j-1} lies in
//     an earlier lane.  Areas inside the tile are stored; the area entering
//     the tile is stored too when it opened in an earlier tile of the same
//     wave, and the run after the last endpoint becomes the open area.
//   Only areas open at the wave's first tile or still open after its last
//   tile take atomicMin (at most two per wave).
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int TSHIFT = 10;
constexpr int T = 1 << TSHIFT;  // contraction tile (elements of A per wave)
constexpr int EPL = T / 64;     // elements per lane in the lane-consecutive layout

// Where each tile's endpoints start: tile_start[t] = first slot whose
// endpoint is >= t * T (t = 0 .. num_tiles, the last entry M), and
// A_Q[j - 1] = +inf for every slot j that is the first of its tile (that
// area reaches into the tile from an earlier one).
//
// Sparse lists (fewer than 8 endpoints per tile on average): one thread per
// tile, binary search over the sorted list (it stays in cache).
__global__ __launch_bounds__(WG) void k_tiles_search(const int32_t* __restrict__ E, int64_t M,
                                                     uint64_t* __restrict__ aq,
                                                     int32_t* __restrict__ tile_start,
                                                     int64_t num_tiles,
                                                     const uint32_t* __restrict__ fail) {
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t > num_tiles || (fail && *fail)) return;
  const int64_t target = t << TSHIFT;
  int64_t lo = 0, hi = M;  // first j in [lo, hi] with E_j >= target
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)E[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  tile_start[t] = (int32_t)lo;
  if (lo >= 1 && lo <= M - 1) aq[lo - 1] = KEY_NONE;
}

// Dense lists: four slots per thread, streaming the list.  Slot j is the
// first of its tile p when slot j - 1 lies in an earlier tile pp; it then
// starts every tile of (pp, p] (a short run when endpoints are dense), and
// the last slot starts every tile after its own.  Tile indices are clamped
// to the tiles of A, so a list that is not sorted positions of A (a caller's
// buffer) cannot send a write out of bounds.
__device__ __forceinline__ int64_t tile_of(int32_t e, int64_t num_tiles) {
  const int64_t p = (int64_t)(uint32_t)e >> TSHIFT;
  return p < num_tiles ? p : num_tiles - 1;
}
__global__ __launch_bounds__(WG) void k_tiles_scatter(const int32_t* __restrict__ E, int64_t M,
                                                      uint64_t* __restrict__ aq,
                                                      int32_t* __restrict__ tile_start,
                                                      int64_t num_tiles,
                                                      const uint32_t* __restrict__ fail) {
  const int64_t j0 = ((int64_t)blockIdx.x * WG + threadIdx.x) * 4;
  if (j0 >= M || (fail && *fail)) return;
  int32_t e[5];  // E[j0 - 1 .. j0 + 3]
  if (j0 + 4 <= M && (((uintptr_t)(E + j0)) & 15) == 0) {
    const v4i32 v = *reinterpret_cast<const v4i32*>(E + j0);
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i + 1] = v[i];
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i + 1] = j0 + i < M ? E[j0 + i] : 0;
  }
  e[0] = j0 > 0 ? E[j0 - 1] : 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t j = j0 + i;
    if (j >= M) break;
    const int64_t p = tile_of(e[i + 1], num_tiles);
    const int64_t pp = j > 0 ? tile_of(e[i], num_tiles) : -1;
    if (p > pp) {
      if (j >= 1) aq[j - 1] = KEY_NONE;
      for (int64_t t = pp + 1; t <= p; ++t) tile_start[t] = (int32_t)j;
    }
    if (j == M - 1)
      for (int64_t t = p + 1; t <= num_tiles; ++t) tile_start[t] = (int32_t)M;
  }
}

// LDS staging of a tile's values: the 16 elements of lane l (block l) at
// words 16 l .. 16 l + 15, their four 4-word groups in the order g ^ s(l),
// s(l) = ((l >> 1) ^ (l >> 2)) & 3.  A 16-byte LDS access serves 8 lanes a
// cycle over 32 banks (16 over 64): the lanes reading one group of their
// own blocks then hit different banks (s differs among blocks that share
// banks), and the lanes storing 4-element pieces of the coalesced load fill
// whole blocks, which share no banks.  (A 20-word row per lane kept the
// reads apart but made those stores wrap onto the same banks.)
constexpr int BLOCK_WORDS = 16;
constexpr int XWORDS = 64 * BLOCK_WORDS;
__device__ __forceinline__ int group_swizzle(int block) { return ((block >> 1) ^ (block >> 2)) & 3; }
__device__ __forceinline__ int stage_index(int e) {
  const int b = e >> 4;
  return b * BLOCK_WORDS + ((((e >> 2) & 3) ^ group_swizzle(b)) << 2) + (e & 3);
}

// Completes this wave's LDS operations before the next ones (the waves of a
// workgroup never share LDS here, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tiles per wave: about 8 where less than one round of waves covers A (2 or
// 4 were slower at every density), at most 63 (a lane per tile of the wave
// holds its table entry); in between, whole rounds of waves share the tiles
// evenly.
constexpr int TPW_MIN = 8, TPW_MAX = 63, WAVES_PER_SIMD = 5;
constexpr int KREG = 4;  // endpoint slots per lane of a tile held in registers (256 a tile)

// The tile's values, coalesced: lane l holds elements 256 c + 4 l + (0..3);
// INT32_MAX past the end of A (never part of an area).
__device__ __forceinline__ void load_tile(const int32_t* __restrict__ A, int64_t n, int64_t t0,
                                          bool aligned, int lane, v4i32 (&xv)[4]) {
  if (aligned && t0 + T <= n) {
#pragma unroll
    for (int c = 0; c < 4; ++c) xv[c] = load_stream(A + t0 + c * 256 + lane * 4);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t p = t0 + c * 256 + lane * 4 + i;
        xv[c][i] = p < n ? A[p] : INT32_MAX;
      }
  }
}

// Positions of the endpoint slots j = jlo + lane + 64 k (k < KREG) of the
// tile starting at t0, t0 + T for slots past jend; only the rounds the tile
// has are loaded.  The values are used as loaded (the tile offset is taken
// where the tile is processed), so that no wait for these loads -- and with
// it for the next tile's values, loaded just before -- comes here.
__device__ __forceinline__ void load_ends(const int32_t* __restrict__ E, uint32_t jlo,
                                          uint32_t jend, uint32_t t0, int lane,
                                          uint32_t (&ep)[KREG]) {
  const uint32_t rounds = (jend - jlo + 63u) >> 6;  // wave-uniform
#pragma unroll
  for (int k = 0; k < KREG; ++k) {
    uint32_t v = t0 + (uint32_t)T;
    if ((uint32_t)k < rounds) {
      const uint32_t j = jlo + (uint32_t)lane + 64u * k;
      if (j < jend) v = (uint32_t)E[j];
    }
    ep[k] = v;
  }
}

// (at most 96 VGPRs: 5 waves per SIMD; the LDS of 5 workgroups fits a CU)
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WAVES_PER_SIMD))) void
k_contract(const int32_t* __restrict__ A, int64_t n, const int32_t* __restrict__ E, int64_t M,
           const int32_t* __restrict__ tile_start, int64_t num_tiles, int64_t nwaves,
           uint64_t* __restrict__ aq, const uint32_t* __restrict__ fail) {
  __shared__ __align__(16) int32_t s_x[WAVES][XWORDS];  // the tile, lane-consecutive
  __shared__ uint32_t s_off[WAVES][EPL / 2][64];         // run-min offsets, 2 x 16 bits
  __shared__ uint32_t s_head[WAVES][T / 32];             // endpoint bits
  __shared__ uint64_t s_carry[WAVES][64];                // run entering each lane
  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // wave g of the launch's nwaves: tiles [g T_n / nwaves, (g + 1) T_n / nwaves)
  // of the T_n tiles, at most 63 (nwaves is chosen so)
  const int64_t gw = (int64_t)blockIdx.x * WAVES + wave;
  if (gw >= nwaves) return;  // the whole wave
  const int64_t tb = gw * num_tiles / nwaves;
  const int cnt = (int)((gw + 1) * num_tiles / nwaves - tb);
  if (cnt <= 0) return;
  const bool aligned = ((uintptr_t)A & 15) == 0;
  // the first tile's values go out before anything else is read: they are
  // in flight while the wave reads the abort word and its table entries
  v4i32 xv[4];
  load_tile(A, n, tb << TSHIFT, aligned, lane, xv);
  if (fail && *fail) return;
  // slots and areas as 32-bit unsigned (M <= 2^31); area j - 1 of slot 0
  // wraps above the last area, M - 2
  const uint32_t Mu = (uint32_t)M;
  const uint32_t last_area = Mu - 2u;
  // tile_start of the wave's tiles and of the tile after them, one per lane
  // (made non-decreasing and at most M, whatever the table holds)
  uint32_t ts_lane = lane <= cnt ? (uint32_t)tile_start[tb + lane] : 0u;
  ts_lane = ts_lane < Mu ? ts_lane : Mu;
#pragma unroll
  for (int dlt = 1; dlt < 64; dlt <<= 1) {  // running max over lanes 0 .. cnt (<= 63)
    const uint32_t up = (uint32_t)__shfl_up((int)ts_lane, dlt);
    if (lane >= dlt && up > ts_lane) ts_lane = up;
  }
  auto ts = [&](int i) { return (uint32_t)__builtin_amdgcn_readlane((int)ts_lane, i); };
  // a wave without endpoints outside the areas (before E_0 or after
  // E_{M-1}) has nothing to do
  if (ts(0) == ts(cnt) && (ts(0) == 0u || ts(0) >= Mu)) return;
  int32_t* xs = s_x[wave];

  uint32_t en[KREG];  // the next tile's endpoint positions (load_ends)
  load_ends(E, ts(0), ts(1), (uint32_t)(tb << TSHIFT), lane, en);
  // the area open at the current tile's start: its index, its min over the
  // part already seen in this wave, and whether it opened before the wave
  // (then other waves add to it too)
  uint32_t open_area = ts(0) - 1u;
  uint64_t acc = KEY_NONE;
  bool shared = true;
  // endpoint-free tiles in a row: each lane's own min over them (value and
  // position, leftmost on ties), folded across the wave into acc only when
  // the run ends (an endpoint tile, or the wave's last tile), so that such a
  // tile costs the lane's compares alone
  int32_t rv = INT32_MAX;
  uint32_t ro = ~0u;  // none yet (positions are below 2^31)
  bool pend = false;  // wave-uniform: the lanes hold values not yet in acc
  auto flush = [&]() {
    if (pend) {
      const uint64_t m = group_min_u64<64>(ro != ~0u ? make_key(rv, ro) : KEY_NONE);
      acc = umin64(acc, (uint64_t)readlane64((int64_t)m, 63));
      rv = INT32_MAX;
      ro = ~0u;
      pend = false;
    }
  };

  for (int i = 0; i < cnt; ++i) {
    const int64_t t0l = (tb + i) << TSHIFT;
    const uint32_t t0 = (uint32_t)t0l;
    const uint32_t jlo = ts(i), jend = ts(i + 1);  // endpoints in [t0, t0 + T)
    const int tile_n = (int)(n - t0l < T ? n - t0l : T);
    const bool more = i + 1 < cnt;
    int32_t ep[KREG];
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      ep[k] = (int32_t)(en[k] - t0);  // tile offsets
      // taken here, while the only loads in flight are this tile's: moved
      // down to their use, the subtraction would wait for the next tile's
      // loads as well
      __asm__ volatile("" : "+v"(ep[k]));
    }

    if (jlo == jend) {
      // no endpoint inside: the tile lies in the open area (none before E_0
      // or after E_{M-1})
      // the next tile's loads go out first, so that they are in flight
      // while this tile is compared
      v4i32 cur[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) cur[c] = xv[c];
      if (more) {
        load_tile(A, n, t0l + T, aligned, lane, xv);
        load_ends(E, jend, ts(i + 2), t0 + T, lane, en);
      }
      if (jlo != 0 && jlo < Mu) {
        pend = true;
        // the lane's elements in increasing position: < keeps the leftmost
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int a = c * 256 + lane * 4 + k;
            const bool take = tile_n == T ? (cur[c][k] < rv || (c == 0 && k == 0 && ro == ~0u))
                                          : (a < tile_n && (cur[c][k] < rv || ro == ~0u));
            rv = take ? cur[c][k] : rv;
            ro = take ? t0 + (uint32_t)a : ro;
          }
      }
      continue;
    }

    // ---- a tile with endpoints: staged in LDS, then the registers take
    // the next tile's loads ----
    flush();  // the area entering the tile has all its earlier values in acc
#pragma unroll
    for (int c = 0; c < 4; ++c)
      *reinterpret_cast<v4i32*>(xs + stage_index(c * 256 + lane * 4)) = xv[c];
    if (lane < T / 32) s_head[wave][lane] = 0;
    if (more) {
      load_tile(A, n, t0l + T, aligned, lane, xv);
      load_ends(E, jend, ts(i + 2), t0 + T, lane, en);
    }
    // the slot before each of this lane's slots (-1: before the tile)
    const uint32_t rounds = (jend - jlo + 63u) >> 6;
    int32_t epv[KREG];
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      const int32_t up = (int32_t)dpp_u32_id<DPP_WAVE_SHR1>((uint32_t)ep[k], 0u);
      const int32_t wrap = k == 0 ? -1 : __builtin_amdgcn_readlane(ep[k - 1], 63);
      epv[k] = lane == 0 ? wrap : up;
    }
    wave_lds_sync();  // head words cleared
#pragma unroll
    for (int k = 0; k < KREG; ++k)
      if ((uint32_t)k < rounds && (uint32_t)ep[k] < (uint32_t)T)
        atomicOr(&s_head[wave][ep[k] >> 5], 1u << (ep[k] & 31));
    for (uint32_t j = jlo + 64u * KREG + (uint32_t)lane; j < jend; j += 64u) {
      const uint32_t e = (uint32_t)E[j] - t0;
      if (e < (uint32_t)T) atomicOr(&s_head[wave][e >> 5], 1u << (e & 31));
    }
    // the tile's last endpoint
    const uint32_t lastj = jend - 1u - jlo;
    int last;
    if (lastj < 64u * KREG) {
      const uint32_t k = lastj >> 6;
      const int32_t v = k == 0 ? ep[0] : (k == 1 ? ep[1] : (k == 2 ? ep[2] : ep[3]));
      last = __builtin_amdgcn_readlane(v, (int)(lastj & 63u));
    } else {
      last = (int)((uint32_t)E[jend - 1u] - t0);
    }
    wave_lds_sync();  // tile staged, heads set

    // lane l: elements 16 l .. 16 l + 15, a running min restarting at heads
    // (and at the lane's first element); < keeps the leftmost
    const uint32_t hb = (s_head[wave][lane >> 1] >> ((lane & 1) * 16)) & 0xFFFFu;
    int32_t cv = 0;
    uint32_t co = 0;
#pragma unroll
    for (int c = 0; c < EPL; c += 4) {
      const v4i32 v = *reinterpret_cast<const v4i32*>(xs + stage_index(lane * EPL + c));
      uint32_t pair = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int cc = c + k;
        const bool take = cc == 0 || ((hb >> cc) & 1u) || v[k] < cv;
        cv = take ? v[k] : cv;
        co = take ? (uint32_t)(lane * EPL + cc) : co;
        if (k & 1)
          s_off[wave][cc >> 1][lane] = pair | (co << 16);
        else
          pair = co;
      }
    }
    // the run entering lane l: min over the lanes' last runs back to the
    // nearest lane with a head (its run from that head on)
    const uint64_t incl = seg_scan_min_u64(make_key(cv, t0 + co), hb != 0);
    s_carry[wave][lane] = dpp_u64_id<DPP_WAVE_SHR1>(incl, KEY_NONE);  // lane 0: none comes in
    wave_lds_sync();

    // min over the half-open part of an area up to tile offset r
    // (inclusive), whose last head is at tile offset h <= r (h = -1: none in
    // this tile)
    auto run_min = [&](int r, int h) {
      const uint32_t o = (s_off[wave][(r & 15) >> 1][r >> 4] >> ((r & 1) * 16)) & 0xFFFFu;
      uint64_t v = make_key(xs[stage_index((int)o)], t0 + o);
      if ((h >> 4) < (r >> 4)) v = umin64(v, s_carry[wave][r >> 4]);  // h >> 4 = -1 for h = -1
      return v;
    };
    // area j - 1, closed by slot j at tile offset e, the slot before at
    // tile offset eprev (-1: before the tile; the area is the open one)
    auto finish = [&](uint32_t j, int e, int eprev) {
      const uint32_t area = j - 1u;
      if (area > last_area || (uint32_t)e >= (uint32_t)tile_n) return;  // e: never, if sorted
      uint64_t val = make_key(xs[stage_index(e)], t0 + (uint32_t)e);  // key(E_j)
      if (eprev < e && e > 0) val = umin64(val, run_min(e - 1, eprev));
      if (eprev < 0) {
        val = umin64(val, acc);
        if (shared)
          atomicMin((unsigned long long*)&aq[area], (unsigned long long)val);
        else
          aq[area] = val;
      } else {
        aq[area] = val;
      }
    };
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      if ((uint32_t)k >= rounds) break;
      const uint32_t j = jlo + (uint32_t)lane + 64u * k;
      if (j < jend) finish(j, ep[k], epv[k]);
    }
    for (uint32_t j = jlo + 64u * KREG + (uint32_t)lane; j < jend; j += 64u)
      finish(j, (int)((uint32_t)E[j] - t0), (int)((uint32_t)E[j - 1u] - t0));
    // the area after the last endpoint stays open
    acc = run_min(tile_n - 1, last);
    open_area = jend - 1u;
    shared = false;
  }
  // the area still open after the wave's last tile continues in later waves
  flush();
  if (lane == 0 && open_area <= last_area && acc != KEY_NONE)
    atomicMin((unsigned long long*)&aq[open_area], (unsigned long long)acc);
}

}  // namespace

hipError_t launch_contract(const int32_t* A, int64_t n, const int32_t* E, int64_t q,
                           uint64_t* aq, int32_t* tile_start, hipStream_t stream,
                           const uint32_t* fail) {
  if (q <= 0) return hipSuccess;
  const int64_t M = 2 * q;
  const int64_t num_tiles = (n + T - 1) / T;
  if (M >= 8 * num_tiles)
    RMQ_TRY(launch(k_tiles_scatter, dim3((unsigned)((M + 4 * WG - 1) / (4 * WG))), dim3(WG), 0,
                   stream, E, M, aq, tile_start, num_tiles, fail));
  else
    RMQ_TRY(launch(k_tiles_search, dim3((unsigned)((num_tiles + 1 + WG - 1) / WG)), dim3(WG), 0,
                   stream, E, M, aq, tile_start, num_tiles, fail));
  // 8 tiles per wave (7 or 8, shared evenly) while that takes less than one
  // round of waves, else the fewest whole rounds with at most 63 tiles per
  // wave, the tiles shared evenly so that every SIMD of a round has the same
  // load.  A round is 5 waves per SIMD, or 4 where the list has at most one
  // endpoint per tile (n = 1e8: 64.3 against 66.8 us at 2e3 endpoints, while
  // 4e7 endpoints took 224 against 204 us)
  const int round_waves = M <= num_tiles ? 4 : WAVES_PER_SIMD;
  const int64_t slots = (int64_t)device_cu_count() * 4 * round_waves;
  const int64_t waves = num_tiles <= slots * TPW_MIN
                            ? (num_tiles + TPW_MIN - 1) / TPW_MIN
                            : slots * ((num_tiles + slots * TPW_MAX - 1) / (slots * TPW_MAX));
  const int64_t grid = (waves + WAVES - 1) / WAVES;
  RMQ_TRY(launch(k_contract, dim3((unsigned)grid), dim3(WG), 0, stream, A, n, E, M, tile_start,
                 num_tiles, waves, aq, fail));
  return hipSuccess;
}

// The comparison system ST-RMQ_CON (Section 2) marks the positions of A
// that end a query and keeps, in A_Q, each marked element and, between two
// marked positions, one entry for the region that separates them.  With
// every sorted endpoint listed twice, the closed areas between neighbouring
// entries of the list alternate between a marked element ([p, p]) and the
// region up to the next marked position ([p, p'], which holds both marked
// ends: that changes no answer, since every query that covers the region's
// entry also covers the two element entries beside it), so the contraction
// above builds that A_Q, 4q - 1 entries, from the doubled list.
namespace {
typedef int32_t v2i32 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(WG) void k_double_ends(const int32_t* __restrict__ E, int64_t M,
                                                    int32_t* __restrict__ E2) {
  const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (j >= M) return;
  const int32_t p = E[j];
  reinterpret_cast<v2i32*>(E2)[j] = v2i32{p, p};
}
}  // namespace

hipError_t launch_double_ends(const int32_t* E, int64_t M, int32_t* E2, hipStream_t stream) {
  if (M <= 0) return hipSuccess;
  RMQ_TRY(launch(k_double_ends, dim3((unsigned)((M + WG - 1) / WG)), dim3(WG), 0, stream, E, M,
                 E2));
  return hipSuccess;
}

size_t contract_tile_start_bytes(int64_t n) {
  return sizeof(int32_t) * (size_t)((n + T - 1) / T + 1);
}

}  // namespace rmq
