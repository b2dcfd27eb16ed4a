// Remap and contraction (Section 3.1 steps 1-2).
//
// With the M = 2q endpoints sorted (E_0 <= ... <= E_{M-1}), A_Q[s] is the min
// key over the CLOSED area A[E_s .. E_{s+1}], s = 0 .. M-2.  Each element p
// in [E_0, E_{M-1}] contributes to the area whose half-open part [E_s,
// E_{s+1}) holds it, and, when p is an endpoint, also closes the area(s)
// ending at p (several, when endpoints repeat: the repeated ones span the
// single element p).
//
// k_tiles (one thread per sorted slot s):
//   * A_Q[s] = +inf for each area that spans two or more contraction tiles
//     (those are finished with atomicMin by several waves);
//   * tile_start[t] = index of the first endpoint >= t * T (written by the
//     thread whose endpoint gap holds t * T).
// k_contract (one wave per tile of T = 1024 elements of A, one streaming
// pass over A between the first and last endpoint):
//   1. the tile's endpoints mark, in LDS, the last slot of every endpoint
//      position inside the tile;
//   2. lane l walks elements 16l .. 16l+15 in order, closing and opening
//      areas at endpoint positions; an area that opens and closes inside the
//      lane is stored directly;
//   3. areas crossing lanes are finished by a segmented min-scan over the 64
//      lanes; areas crossing tiles get atomicMin on their slot.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;
constexpr int TSHIFT = 10;
constexpr int T = 1 << TSHIFT;  // contraction tile (elements of A per wave)
constexpr int EPL = T / 64;     // elements per lane

// One thread per 4 consecutive slots s = 4i .. 4i+3 (and the past-the-end
// slot M, which closes the tile table).
// Position of sorted endpoint j: the list holds (position << 32) | tag.
__device__ __forceinline__ int32_t epos(const uint64_t* __restrict__ E, int64_t j) {
  return (int32_t)(E[j] >> 32);
}

__global__ __launch_bounds__(WG) void k_tiles(const uint64_t* __restrict__ E, int64_t M,
                                              uint64_t* __restrict__ aq,
                                              int32_t* __restrict__ tile_start,
                                              int64_t num_tiles) {
  const int64_t s0 = ((int64_t)blockIdx.x * WG + threadIdx.x) * 4;
  if (s0 > M) return;
  // positions of a sorted list lie in [0, n); clamping only guards the
  // writes below against a malformed list
  const int64_t last = num_tiles * T - 1;
  auto clampp = [last](int64_t e) { return e < 0 ? 0 : (e > last ? last : e); };
  int64_t e[6];  // positions of slots s0-1 .. s0+4
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int64_t s = s0 - 1 + i;
    e[i] = (s >= 0 && s < M) ? clampp(epos(E, s)) : -1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t s = s0 + i;
    if (s > M) break;
    const int64_t e_prev = e[i], e_cur = e[i + 1];
    if (s + 1 < M && (e_cur >> TSHIFT) != (e[i + 2] >> TSHIFT)) aq[s] = KEY_NONE;
    // tiles t with e_prev < t*T <= e_cur get tile_start[t] = s
    const int64_t t_lo = s == 0 ? 0 : (e_prev >> TSHIFT) + 1;
    const int64_t t_hi = s == M ? num_tiles : (e_cur >> TSHIFT);
    for (int64_t t = t_lo; t <= t_hi; ++t) tile_start[t] = (int32_t)s;
  }
}

// A[p..p+3], elements past n read as INT32_MAX (never part of an area).
__device__ __forceinline__ v4i32 load4(const int32_t* __restrict__ A, int64_t p, int64_t n,
                                       bool aligned) {
  if (aligned && p + 3 < n) return load_stream(A + p);
  v4i32 x;
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = p + i < n ? A[p + i] : INT32_MAX;
  return x;
}

__global__ __launch_bounds__(WG) void k_contract(const int32_t* __restrict__ A, int64_t n,
                                                 const uint64_t* __restrict__ E, int64_t M,
                                                 const int32_t* __restrict__ tile_start,
                                                 int64_t num_tiles, uint64_t* __restrict__ aq) {
  __shared__ __align__(16) int32_t head_last[WG / 64][T];
  __shared__ __align__(16) int32_t vals[WG / 64][T];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * (WG / 64) + wave;
  const bool tile_ok = tile < num_tiles;
  const int64_t t0 = tile << TSHIFT;
  int64_t jlo = tile_ok ? tile_start[tile] : M;
  int64_t jend = tile_ok ? tile_start[tile + 1] : M;  // endpoints in [t0, t0+T)
  jlo = jlo < 0 ? 0 : (jlo > M ? M : jlo);
  jend = jend < jlo ? jlo : (jend > M ? M : jend);
  // tiles wholly before E_0 (jend == 0) or after E_{M-1} (jlo == M) hold no area
  const bool active = tile_ok && jend > 0 && jlo < M;
  const bool marked = active && jend > jlo;  // the tile holds endpoints
  const int64_t last_area = M - 2;           // valid areas are 0 .. M-2
  int32_t* hl = head_last[wave];
  int32_t* xs = vals[wave];

  // coalesced 16-byte loads: lane l holds elements 4l + 256c + (0..3)
  const bool aligned = ((uintptr_t)A & 15) == 0;
  v4i32 xv[4];
  if (tile_ok) {  // issued before the tile's endpoint range is known
#pragma unroll
    for (int c = 0; c < 4; ++c) xv[c] = load4(A, t0 + c * 256 + lane * 4, n, aligned);
  }

  if (active && !marked) {
    // no endpoint inside: the whole tile lies in area jlo - 1
    uint64_t m = KEY_NONE;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t p = t0 + c * 256 + lane * 4 + i;
        if (p < n) m = umin64(m, make_key(xv[c][i], (uint32_t)p));
      }
    m = group_min_u64<64>(m);
    const int64_t area = jlo - 1;
    if (lane == 63 && area >= 0 && area <= last_area)
      atomicMin((unsigned long long*)&aq[area], (unsigned long long)m);
  }

  if (marked) {
    for (int c = lane; c < T; c += 64) hl[c] = -1;
#pragma unroll
    for (int c = 0; c < 4; ++c) *reinterpret_cast<v4i32*>(xs + c * 256 + lane * 4) = xv[c];
  }
  __syncthreads();
  if (marked) {
    for (int64_t j = jlo + lane; j < jend; j += 64) {
      const int32_t e = epos(E, j);
      const bool last_dup = (j + 1 == M) || (epos(E, j + 1) != e);
      if (last_dup && e >= t0 && e < t0 + T) hl[e - t0] = (int32_t)j;
    }
  }
  __syncthreads();
  if (!marked) return;  // whole wave leaves together; no barrier follows

  // ---- per lane: 16 consecutive elements and their endpoint slots ----
  const int64_t p0 = t0 + (int64_t)lane * EPL;
  int32_t h[EPL], x[EPL];
#pragma unroll
  for (int c = 0; c < EPL; c += 4) {
    const v4i32 hv = *reinterpret_cast<const v4i32*>(hl + lane * EPL + c);
    const v4i32 v = *reinterpret_cast<const v4i32*>(xs + lane * EPL + c);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h[c + i] = hv[i];
      x[c + i] = v[i];
    }
  }
  int32_t last_head = -1;
  bool has_head = false;
#pragma unroll
  for (int c = 0; c < EPL; ++c) {
    if (h[c] >= 0) {
      last_head = h[c];
      has_head = true;
    }
  }

  // area open when this lane starts: the last slot marked in an earlier lane,
  // else the area open at the tile start (slot jlo - 1; -1 before E_0)
  const uint64_t heads = ballot(has_head);
  const uint64_t below = heads & ((1ull << lane) - 1ull);
  const int src = below ? 63 - __clzll(below) : lane;
  const int32_t from_below = __shfl(last_head, src);
  const int64_t in_area = below ? (int64_t)from_below : jlo - 1;

  // ---- walk the lane's elements ----
  uint64_t in_key = KEY_NONE, out_key = KEY_NONE;
  int64_t cur = in_area;
  bool seen = false;
#pragma unroll
  for (int c = 0; c < EPL; ++c) {
    const int64_t p = p0 + c;
    const uint64_t key = make_key(x[c], (uint32_t)p);
    if (h[c] >= 0) {
      // p closes area `cur` and the repeated-endpoint areas cur+1 .. h-1
      if (!seen) {
        in_key = umin64(in_key, key);
      } else if (cur >= 0 && cur <= last_area) {
        aq[cur] = umin64(out_key, key);  // opened and closed in this lane
      }
      for (int64_t s = cur + 1; s < h[c]; ++s)
        if (s >= 0 && s <= last_area) aq[s] = key;
      cur = h[c];
      out_key = key;
      seen = true;
    } else if (seen) {
      out_key = umin64(out_key, key);
    } else {
      in_key = umin64(in_key, key);
    }
  }

  // ---- areas that cross lanes: segmented inclusive min-scan ----
  // carry-out of lane i: the partial of the area open at its end
  uint64_t v = has_head ? out_key : in_key;
  bool f = has_head;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t vu = __shfl_up(v, d);
    const int fu = __shfl_up((int)f, d);
    if (lane >= d) {
      if (!f) v = umin64(v, vu);
      f = f || fu;
    }
  }
  uint64_t carry_in = __shfl_up(v, 1);
  if (lane == 0) carry_in = KEY_NONE;

  if (has_head && in_area >= 0 && in_area <= last_area) {
    const uint64_t val = umin64(carry_in, in_key);
    if (below)
      aq[in_area] = val;  // opened earlier in this tile: single writer
    else
      atomicMin((unsigned long long*)&aq[in_area], (unsigned long long)val);
  }
  if (lane == 63) {
    const int64_t tail_area = has_head ? cur : in_area;
    if (tail_area >= 0 && tail_area <= last_area)
      atomicMin((unsigned long long*)&aq[tail_area], (unsigned long long)v);
  }
}

}  // namespace

hipError_t launch_contract(const int32_t* A, int64_t n, const uint64_t* E, int64_t q,
                           uint64_t* aq, int32_t* tile_start, hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t M = 2 * q;
  const int64_t num_tiles = (n + T - 1) / T;
  const int64_t threads = M / 4 + 1;  // slots 0 .. M, four per thread
  RMQ_TRY(launch(k_tiles, dim3((unsigned)((threads + WG - 1) / WG)), dim3(WG), 0, stream, E, M,
                 aq, tile_start, num_tiles));
  const int64_t grid = (num_tiles + (WG / 64) - 1) / (WG / 64);
  RMQ_TRY(launch(k_contract, dim3((unsigned)grid), dim3(WG), 0, stream, A, n, E, M, tile_start,
                 num_tiles, aq));
  return hipSuccess;
}

size_t contract_tile_start_bytes(int64_t n) {
  return sizeof(int32_t) * (size_t)((n + T - 1) / T + 1);
}

}  // namespace rmq
