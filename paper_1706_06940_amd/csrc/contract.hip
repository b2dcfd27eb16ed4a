// Remap and contraction (Section 3.1 steps 1-2).
//
// With the M = 2q endpoints sorted (E_0 <= ... <= E_{M-1}), A_Q[s] is the min
// key over the CLOSED area A[E_s .. E_{s+1}], s = 0 .. M-2.  Each element p
// in [E_0, E_{M-1}] contributes to the area whose half-open part [E_s,
// E_{s+1}) holds it, and, when p is an endpoint, also closes the area(s)
// ending at p (several, when endpoints repeat: the repeated ones span the
// single element p).
//
// k_remap (one thread per sorted slot s):
//   * Lc[i] = s for the left end of query i, Rc[i] = s - 1 for its right end;
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

__global__ __launch_bounds__(WG) void k_remap(const int32_t* __restrict__ pos,
                                              const int32_t* __restrict__ tag, int64_t M,
                                              int32_t* __restrict__ Lc, int32_t* __restrict__ Rc,
                                              uint64_t* __restrict__ aq,
                                              int32_t* __restrict__ tile_start,
                                              int64_t num_tiles) {
  const int64_t s = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (s > M) return;
  if (s < M) {
    const int32_t t = tag[s];
    if (t >= 0 && t < M) {  // a sorted list holds every tag once
      if (t & 1)
        Rc[t >> 1] = (int32_t)(s - 1);
      else
        Lc[t >> 1] = (int32_t)s;
    }
  }
  // positions of a sorted list lie in [0, n); clamping only guards the
  // writes below against a malformed list
  const int64_t last = num_tiles * T - 1;
  auto clampp = [last](int64_t e) { return e < 0 ? 0 : (e > last ? last : e); };
  const int64_t e_prev = s > 0 ? clampp(pos[s - 1]) : -1;
  const int64_t e_cur = s < M ? clampp(pos[s]) : -1;
  if (s + 1 < M) {
    const int64_t e_next = clampp(pos[s + 1]);
    if ((e_cur >> TSHIFT) != (e_next >> TSHIFT)) aq[s] = KEY_NONE;
  }
  // tiles t with e_prev < t*T <= e_cur get tile_start[t] = s
  const int64_t t_lo = s == 0 ? 0 : (e_prev >> TSHIFT) + 1;
  const int64_t t_hi = s == M ? num_tiles : (e_cur >> TSHIFT);
  for (int64_t t = t_lo; t <= t_hi; ++t) tile_start[t] = (int32_t)s;
}

__device__ __forceinline__ int32_t load_elem(const int32_t* __restrict__ A, int64_t p, int64_t n) {
  return p < n ? A[p] : INT32_MAX;
}

__global__ __launch_bounds__(WG) void k_contract(const int32_t* __restrict__ A, int64_t n,
                                                 const int32_t* __restrict__ E, int64_t M,
                                                 const int32_t* __restrict__ tile_start,
                                                 int64_t num_tiles, uint64_t* __restrict__ aq) {
  __shared__ __align__(16) int32_t head_last[WG / 64][T];
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
  int32_t* hl = head_last[wave];

  for (int c = lane; c < T; c += 64) hl[c] = -1;
  __syncthreads();
  if (active) {
    for (int64_t j = jlo + lane; j < jend; j += 64) {
      const int32_t e = E[j];
      const bool last_dup = (j + 1 == M) || (E[j + 1] != e);
      if (last_dup && e >= t0 && e < t0 + T) hl[e - t0] = (int32_t)j;
    }
  }
  __syncthreads();
  if (!active) return;  // whole wave leaves together; no barrier follows

  // ---- per lane: its endpoint slots and elements ----
  const int64_t p0 = t0 + (int64_t)lane * EPL;
  int32_t h[EPL];
#pragma unroll
  for (int c = 0; c < EPL; c += 4) {
    const int4 v = *reinterpret_cast<const int4*>(hl + lane * EPL + c);
    h[c] = v.x;
    h[c + 1] = v.y;
    h[c + 2] = v.z;
    h[c + 3] = v.w;
  }
  int32_t x[EPL];
  if (((uintptr_t)A & 15) == 0 && p0 + EPL <= n) {
#pragma unroll
    for (int c = 0; c < EPL; c += 4) {
      const v4i32 v = load_stream(A + p0 + c);
      x[c] = v[0];
      x[c + 1] = v[1];
      x[c + 2] = v[2];
      x[c + 3] = v[3];
    }
  } else {
#pragma unroll
    for (int c = 0; c < EPL; ++c) x[c] = load_elem(A, p0 + c, n);
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
  const int64_t last_area = M - 2;  // valid areas are 0 .. M-2
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

hipError_t launch_contract(const int32_t* A, int64_t n, const int32_t* pos, const int32_t* tag,
                           int64_t q, int32_t* Lc, int32_t* Rc, uint64_t* aq, int32_t* tile_start,
                           hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const int64_t M = 2 * q;
  const int64_t num_tiles = (n + T - 1) / T;
  hipLaunchKernelGGL(k_remap, dim3((unsigned)((M + 1 + WG - 1) / WG)), dim3(WG), 0, stream, pos,
                     tag, M, Lc, Rc, aq, tile_start, num_tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = (num_tiles + (WG / 64) - 1) / (WG / 64);
  hipLaunchKernelGGL(k_contract, dim3((unsigned)grid), dim3(WG), 0, stream, A, n, pos, M,
                     tile_start, num_tiles, aq);
  return hipGetLastError();
}

size_t contract_tile_start_bytes(int64_t n) {
  return sizeof(int32_t) * (size_t)((n + T - 1) / T + 1);
}

}  // namespace rmq
