// Remap and contraction (Section 3.1 steps 1-2).
//
// With the M = 2q endpoints sorted (E_0 <= ... <= E_{M-1}), A_Q[s] is the min
// key over the CLOSED area A[E_s .. E_{s+1}], s = 0 .. M-2.  Split each area
// into its half-open part [E_s, E_{s+1}) and its closing element E_{s+1}:
//   A_Q[s] = min(min over [E_s, E_{s+1}), key(E_{s+1})),
// where the half-open parts of consecutive areas tile [E_0, E_{M-1}) and are
// empty for repeated endpoints (then A_Q[s] = key(E_s)).
//
// k_tiles (one thread per contraction tile of T = 1024 elements, plus one):
//   * tile_start[t] = first slot whose endpoint is >= t * T (binary search
//     over the sorted list);
//   * A_Q[tile_start[t] - 1] = +inf: that area holds t * T and spans two or
//     more tiles, so several waves finish it with atomicMin.
// k_contract (one wave per tile, one streaming pass over A):
//   * a tile without endpoints lies inside one area: wave min, atomicMin;
//   * otherwise the tile's endpoints set head bits in LDS; lane l walks its
//     16 consecutive elements with a running min that restarts at heads; a
//     segmented min-scan over the lanes carries runs across lanes, and the
//     1024 running minima go to LDS.  Then one lane per endpoint slot j in
//     the tile reads off area j-1: the running min just before E_j (the
//     half-open part, or its piece inside this tile) and the key at E_j.
//     Areas inside the tile get plain coalesced stores; the area entering
//     the tile and the one leaving it get atomicMin.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;
constexpr int TSHIFT = 10;
constexpr int T = 1 << TSHIFT;  // contraction tile (elements of A per wave)
constexpr int EPL = T / 64;     // elements per lane

// Position of sorted endpoint j (P: the sorted endpoint positions).
__device__ __forceinline__ int64_t epos(const int32_t* __restrict__ P, int64_t j) {
  return (int64_t)P[j];
}

__global__ __launch_bounds__(WG) void k_tiles(const int32_t* __restrict__ E, int64_t M,
                                              uint64_t* __restrict__ aq,
                                              int32_t* __restrict__ tile_start,
                                              int64_t num_tiles) {
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t > num_tiles) return;
  const int64_t target = t << TSHIFT;
  int64_t lo = 0, hi = M;  // first j in [lo, hi] with E_j >= target
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (epos(E, mid) < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  tile_start[t] = (int32_t)lo;
  if (lo >= 1 && lo <= M - 1) aq[lo - 1] = KEY_NONE;
}

// LDS staging of a tile's values: 16-element block b at word 20 b, so lane l
// reading block l (16 bytes at a time) and lanes writing 4-element pieces of
// the coalesced load stay spread over the banks.
constexpr int BLOCK_WORDS = 20;
__device__ __forceinline__ int stage_index(int e) { return (e >> 4) * BLOCK_WORDS + (e & 15); }

constexpr int KREG = 8;  // endpoint slots per lane held in registers (512 per tile)

__global__ __launch_bounds__(WG) void k_contract(const int32_t* __restrict__ A, int64_t n,
                                                 const int32_t* __restrict__ E, int64_t M,
                                                 const int32_t* __restrict__ tile_start,
                                                 int64_t num_tiles, uint64_t* __restrict__ aq) {
  __shared__ __align__(16) int32_t vals[WG / 64][(T / 16) * BLOCK_WORDS];
  __shared__ uint32_t offs[WG / 64][EPL / 2][64];  // argmin offsets of the runs
  __shared__ uint32_t heads[WG / 64][T / 32];       // endpoint bits
  __shared__ uint64_t wmin[WG / 64];                // tiles without endpoints:
  __shared__ int64_t warea[WG / 64];                //   their min and area
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * (WG / 64) + wave;
  const bool tile_ok = tile < num_tiles;
  const int64_t tc = tile_ok ? tile : num_tiles - 1;  // loads below stay in bounds
  const int64_t t0 = tile << TSHIFT;
  const int64_t tile_n = n - t0 < T ? n - t0 : T;

  // every load that does not depend on another is issued at once: the
  // tile's endpoint range, then its 1024 elements (coalesced 16-byte loads:
  // lane l holds elements 256c + 4l + (0..3))
  int64_t jlo = tile_start[tc];
  int64_t jend = tile_start[tc + 1];  // endpoints in [t0, t0+T)
  v4i32 xv[4];
  if (((uintptr_t)A & 15) == 0 && (tc << TSHIFT) + T <= n) {
#pragma unroll
    for (int c = 0; c < 4; ++c) xv[c] = load_stream(A + (tc << TSHIFT) + c * 256 + lane * 4);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t p = (tc << TSHIFT) + c * 256 + lane * 4 + i;
        xv[c][i] = p < n ? A[p] : INT32_MAX;  // never part of an area
      }
  }
  if (!tile_ok) jlo = jend = M;
  jlo = jlo < 0 ? 0 : (jlo > M ? M : jlo);
  jend = jend < jlo ? jlo : (jend > M ? M : jend);
  // tiles wholly before E_0 (jend == 0) or after E_{M-1} (jlo == M) hold no area
  const bool active = tile_ok && jend > 0 && jlo < M;
  const bool marked = active && jend > jlo;  // the tile holds endpoints
  const int64_t last_area = M - 2;           // valid areas are 0 .. M-2

  // tile offsets of this lane's endpoint slots j = jlo + lane + 64k (first
  // KREG rounds), and of the slot before each; loads clamped to the list
  // (rounds with no slot are skipped as a whole: the test is uniform)
  const int rounds = marked ? (int)((jend - jlo + 63) >> 6) : 0;
  int32_t ep[KREG], epv[KREG];
  if (marked) {
    int32_t raw[KREG];
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      const int64_t j = jlo + lane + 64 * k;
      raw[k] = k < rounds ? E[j < M ? j : M - 1] : 0;
    }
    const int32_t raw_lo = E[jlo > 0 ? jlo - 1 : 0];
#pragma unroll
    for (int k = 0; k < KREG; ++k)
      ep[k] = jlo + lane + 64 * k < jend ? (int32_t)(raw[k] - t0) : T;
    const int32_t before_lo = jlo > 0 ? (int32_t)(raw_lo - t0) : -1;
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      if (k >= rounds) break;
      const int32_t up = (int32_t)dpp_u32_id<DPP_WAVE_SHR1>((uint32_t)ep[k], 0u);
      const int32_t wrap = k == 0 ? before_lo : __builtin_amdgcn_readlane(ep[k - 1], 63);
      epv[k] = lane == 0 ? wrap : up;
    }
  }

  uint64_t m = KEY_NONE;
  if (active && !marked) {
    // no endpoint inside: the whole tile lies in area jlo - 1
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t p = t0 + c * 256 + lane * 4 + i;
        if (p < n) m = umin64(m, make_key(xv[c][i], (uint32_t)p));
      }
    m = group_min_u64<64>(m);  // the wave's min lands in lane 63
  }
  if (lane == 63) {
    wmin[wave] = m;
    warea[wave] = active && !marked ? jlo - 1 : -1;
  }

  int32_t* xs = vals[wave];
  if (marked) {
    if (lane < T / 32) heads[wave][lane] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      *reinterpret_cast<v4i32*>(xs + stage_index(c * 256 + lane * 4)) = xv[c];
  }
  __syncthreads();
  if (active && !marked && lane == 63) {
    // consecutive endpoint-free tiles of this workgroup in the same area
    // make one atomic, issued by the first of them
    const int64_t area = jlo - 1;
    if ((wave == 0 || warea[wave - 1] != area) && area >= 0 && area <= last_area) {
      uint64_t r = m;
      for (int w = wave + 1; w < WG / 64 && warea[w] == area; ++w) r = umin64(r, wmin[w]);
      atomicMin((unsigned long long*)&aq[area], (unsigned long long)r);
    }
  }
  if (marked) {
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
      if (k >= rounds) break;
      if (ep[k] >= 0 && ep[k] < T) atomicOr(&heads[wave][ep[k] >> 5], 1u << (ep[k] & 31));
    }
    for (int64_t j = jlo + 64 * KREG + lane; j < jend; j += 64) {
      const int64_t e = epos(E, j) - t0;
      if (e >= 0 && e < T) atomicOr(&heads[wave][e >> 5], 1u << (e & 31));
    }
  }
  __syncthreads();
  if (marked) {
    // ---- lane l: elements 16l .. 16l+15, a running min restarting at heads;
    // values compared with < keep the leftmost of equal values ----
    const uint32_t hb = (heads[wave][lane >> 1] >> ((lane & 1) * 16)) & 0xFFFFu;
    int32_t rv[EPL];
    uint32_t ro[EPL];
#pragma unroll
    for (int c = 0; c < EPL; c += 4) {
      const v4i32 v = *reinterpret_cast<const v4i32*>(xs + lane * BLOCK_WORDS + c);
#pragma unroll
      for (int i = 0; i < 4; ++i) rv[c + i] = v[i];
    }
    int32_t cv = INT32_MAX;
    uint32_t co = 0;
#pragma unroll
    for (int c = 0; c < EPL; ++c) {
      const uint32_t o = (uint32_t)(lane * EPL + c);
      const bool take = ((hb >> c) & 1u) || rv[c] < cv || c == 0;
      cv = take ? rv[c] : cv;
      co = take ? o : co;
      rv[c] = cv;
      ro[c] = co;
    }
    // ---- runs across lanes: segmented inclusive min-scan of lane totals
    // (keys of value and offset, so equal values keep the leftmost) ----
    const uint64_t v = seg_scan_min_u64(make_key(cv, co), hb != 0);
    const uint64_t carry = dpp_u64_id<DPP_WAVE_SHR1>(v, KEY_NONE);  // lane 0: no run comes in
    const int first = hb ? __builtin_ctz(hb) : EPL;
    const int32_t kv = (int32_t)((uint32_t)(carry >> 32) ^ 0x80000000u);
    const uint32_t ko = (uint32_t)carry;
#pragma unroll
    for (int c = 0; c < EPL; ++c)
      if (lane > 0 && c < first && kv <= rv[c]) ro[c] = ko;  // the run coming in
#pragma unroll
    for (int c = 0; c < EPL; c += 2) offs[wave][c >> 1][lane] = ro[c] | (ro[c + 1] << 16);
  }
  __syncthreads();
  if (!marked) return;  // whole wave leaves together; no barrier follows

  // key of the run minimum ending at tile offset e
  auto run_key = [&](int e) {
    const uint32_t o = (offs[wave][(e & 15) >> 1][e >> 4] >> ((e & 1) * 16)) & 0xFFFFu;
    return make_key(xs[stage_index((int)o)], (uint32_t)(t0 + o));
  };
  // area j - 1 from endpoint slot j at tile offset e (previous endpoint at eprev)
  auto finish = [&](int64_t j, int64_t e, int64_t eprev) {
    const int64_t area = j - 1;
    if (area < 0 || area > last_area || e < 0 || e >= tile_n) return;  // e: never, if sorted
    uint64_t val = make_key(xs[stage_index((int)e)], (uint32_t)(t0 + e));  // key(E_j)
    if (eprev < e && e > 0) val = umin64(val, run_key((int)e - 1));
    if (eprev < 0)
      atomicMin((unsigned long long*)&aq[area], (unsigned long long)val);  // entering area
    else
      aq[area] = val;
  };
#pragma unroll
  for (int k = 0; k < KREG; ++k) {
    if (k >= rounds) break;
    const int64_t j = jlo + lane + 64 * k;
    if (j < jend) finish(j, ep[k], epv[k]);
  }
  for (int64_t j = jlo + 64 * KREG + lane; j < jend; j += 64)
    finish(j, epos(E, j) - t0, epos(E, j - 1) - t0);
  // the area leaving the tile: from the last head to the tile's end
  if (lane == 0) {
    const int64_t area = jend - 1;
    if (area <= last_area)
      atomicMin((unsigned long long*)&aq[area], (unsigned long long)run_key((int)tile_n - 1));
  }
}

}  // namespace

hipError_t launch_contract(const int32_t* A, int64_t n, const int32_t* E, int64_t q,
                           uint64_t* aq, int32_t* tile_start, hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t M = 2 * q;
  const int64_t num_tiles = (n + T - 1) / T;
  RMQ_TRY(launch(k_tiles, dim3((unsigned)((num_tiles + 1 + WG - 1) / WG)), dim3(WG), 0, stream, E,
                 M, aq, tile_start, num_tiles));
  const int64_t grid = (num_tiles + (WG / 64) - 1) / (WG / 64);
  RMQ_TRY(launch(k_contract, dim3((unsigned)grid), dim3(WG), 0, stream, A, n, E, M, tile_start,
                 num_tiles, aq));
  return hipSuccess;
}

size_t contract_tile_start_bytes(int64_t n) {
  return sizeof(int32_t) * (size_t)((n + T - 1) / T + 1);
}

}  // namespace rmq
