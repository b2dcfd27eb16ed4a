// Block minima (Section 3.2, first stage; Section 3.1 step 3 on A_Q):
// keys[j] = min key over block j of k consecutive elements.
//
// One streaming pass over the input with 16-byte loads.  A workgroup of 4
// waves owns a chunk of C elements -- one whole block when k > 4 wave loads,
// else 16 wave loads -- and wave w owns the w-th quarter of it.  Inside a wave:
//   * k <= 4 wave loads   -> the wave's four loads go out together; a block
//     is then k / (one wave load) of them (a per-lane running (value,
//     position) minimum, then a full-wave DPP min), or k / V lanes of one
//     load (a DPP group min);
//   * k >  4 wave loads   -> the four waves hold quarters of one block, four
//     loads in flight per step, and combine their minima through LDS.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;

// ---------------------------------------------------------------- int32 input
// Per-lane running minimum over 4 consecutive int32 at positions p..p+3.
// Elements are met in increasing position, so a strict < keeps the leftmost.
struct LaneMin {
  int32_t v;
  int64_t p;
};

__device__ __forceinline__ void lane_update(LaneMin& m, v4i32 x, int64_t p) {
  if (x.x < m.v) { m.v = x.x; m.p = p; }
  if (x.y < m.v) { m.v = x.y; m.p = p + 1; }
  if (x.z < m.v) { m.v = x.z; m.p = p + 2; }
  if (x.w < m.v) { m.v = x.w; m.p = p + 3; }
}

template <bool ALIGNED>
__device__ __forceinline__ v4i32 load4_i32(const int32_t* __restrict__ A, int64_t p, int64_t n) {
  if (ALIGNED && p + 3 < n) return load_stream(A + p);
  v4i32 x;
  x.x = p + 0 < n ? A[p + 0] : INT32_MAX;
  x.y = p + 1 < n ? A[p + 1] : INT32_MAX;
  x.z = p + 2 < n ? A[p + 2] : INT32_MAX;
  x.w = p + 3 < n ? A[p + 3] : INT32_MAX;
  return x;
}

// Key of a lane's running minimum.  The minimum starts as (INT32_MAX, first
// position of the lane): correct even when that element is INT32_MAX, since
// a strict < never replaces an equal value.  A lane whose first position is
// past n contributes nothing.
__device__ __forceinline__ uint64_t lane_key(const LaneMin& m, int64_t first, int64_t n) {
  return first < n ? make_key(m.v, (uint32_t)m.p) : KEY_NONE;
}

// The work of workgroup `wg` (chunk wg of C elements) of one array.
template <bool ALIGNED>
__device__ __forceinline__ void blockmin_i32_wg(const int32_t* __restrict__ A, int64_t n,
                                                int kshift, uint64_t* __restrict__ keys,
                                                int64_t wg, uint64_t* part) {
  constexpr int V = 4, WL = 64 * V;  // elements per lane load / per wave load
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t k = 1ll << kshift;
  const int64_t C = k > 4 * WL ? k : 16 * WL;
  const int64_t WS = C / 4;  // elements per wave, >= 4 * WL
  const int64_t w0 = wg * C + wave * WS;

  if (k <= 4 * WL) {
    // the wave's four loads (WS = 4 WL) go out together, then its blocks
    // are reduced: k / WL loads per block, or k / V lanes of one load
    v4i32 x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = load4_i32<ALIGNED>(A, w0 + c * WL + lane * V, n);
    if (k >= WL) {
      const int per = (int)(k / WL);  // 1, 2 or 4
#pragma unroll
      for (int b0 = 0; b0 < 4; ++b0) {
        if (b0 % per) continue;
        const int64_t first = w0 + b0 * WL + lane * V;
        LaneMin m{INT32_MAX, first};
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (c >= b0 && c < b0 + per) lane_update(m, x[c], w0 + c * WL + lane * V);
        const uint64_t key = group_min_u64<64>(lane_key(m, first, n));
        const int64_t s0 = w0 + b0 * WL;
        if (lane == 63 && s0 < n) keys[s0 >> kshift] = key;
      }
    } else {
      // several blocks per wave load: groups of g = k / V lanes
      const int g = (int)(k / V);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t first = w0 + c * WL + lane * V;
        LaneMin m{INT32_MAX, first};
        lane_update(m, x[c], first);
        const uint64_t key = group_min_u64_rt(lane_key(m, first, n), g);
        const int64_t blk_start = first - (int64_t)(lane % g) * V;
        if ((lane % g) == g - 1 && blk_start < n) keys[blk_start >> kshift] = key;
      }
    }
    return;
  }

  // one block spans more than 4 wave loads: the workgroup holds one block,
  // each wave a quarter of it, with four loads in flight per step
  const int64_t first = w0 + lane * V;
  LaneMin m{INT32_MAX, first};
  const v4i32 none = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  for (int64_t it = 0; it < WS; it += 4 * WL) {  // WS = 2, 4, 8, ... wave loads
    v4i32 x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      x[c] = it + c * WL < WS ? load4_i32<ALIGNED>(A, first + it + c * WL, n) : none;
#pragma unroll
    for (int c = 0; c < 4; ++c) lane_update(m, x[c], first + it + c * WL);
  }
  const uint64_t key = group_min_u64<64>(lane_key(m, first, n));
  if (lane == 63) part[wave] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t b = umin64(umin64(part[0], part[1]), umin64(part[2], part[3]));
    if (wg * C < n) keys[wg] = b;
  }
}

template <bool ALIGNED>
__global__ __launch_bounds__(WG) void k_blockmin_i32(const int32_t* __restrict__ A, int64_t n,
                                                     int kshift, uint64_t* __restrict__ keys) {
  __shared__ uint64_t part[4];
  blockmin_i32_wg<ALIGNED>(A, n, kshift, keys, blockIdx.x, part);
}

// Block minima of every array of a batch in one launch: workgroup w does
// jobs 2w and 2w + 1, one chunk of one array each.  Both job records are
// read at once, so a workgroup waits for one record read per two chunks
// (one job per workgroup: 0.81 of the HBM peak on the batched workload,
// against 0.85 for one array's pass, whose workgroups find their chunk from
// their index).
constexpr int MULTI_JOBS = 2;
__global__ __launch_bounds__(WG) void k_blockmin_multi(const ChunkJob* __restrict__ jobs,
                                                       int64_t count) {
  __shared__ uint64_t part[MULTI_JOBS][4];  // one set per job: no barrier between them
  ChunkJob jb[MULTI_JOBS];
#pragma unroll
  for (int u = 0; u < MULTI_JOBS; ++u) {
    const int64_t j = (int64_t)blockIdx.x * MULTI_JOBS + u;
    jb[u] = jobs[j < count ? j : count - 1];
  }
#pragma unroll
  for (int u = 0; u < MULTI_JOBS; ++u) {
    if ((int64_t)blockIdx.x * MULTI_JOBS + u >= count) break;  // uniform
    const int32_t* A = static_cast<const int32_t*>(jb[u].src);
    if (((uintptr_t)A & 15) == 0)
      blockmin_i32_wg<true>(A, jb[u].len, jb[u].shift, jb[u].keys, jb[u].chunk, part[u]);
    else
      blockmin_i32_wg<false>(A, jb[u].len, jb[u].shift, jb[u].keys, jb[u].chunk, part[u]);
  }
}

// ---------------------------------------------------------------- uint64 keys
template <bool ALIGNED>
__device__ __forceinline__ void load2_key(const uint64_t* __restrict__ S, int64_t p, int64_t m,
                                          uint64_t& a, uint64_t& b) {
  if (ALIGNED && p + 1 < m) {
    v2u64 x = load_stream(S + p);
    a = x.x;
    b = x.y;
    return;
  }
  a = p < m ? S[p] : KEY_NONE;
  b = p + 1 < m ? S[p + 1] : KEY_NONE;
}

template <bool ALIGNED>
__device__ __forceinline__ void blockmin_keys_wg(const uint64_t* __restrict__ S, int64_t m,
                                                 int kshift, uint64_t* __restrict__ keys,
                                                 int64_t wg, uint64_t* part) {
  constexpr int V = 2, WL = 64 * V;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t k = 1ll << kshift;
  const int64_t C = k > 4 * WL ? k : 16 * WL;
  const int64_t WS = C / 4;
  const int64_t w0 = wg * C + wave * WS;

  if (k >= WL) {
    const int64_t span = k < WS ? k : WS;
    for (int64_t s0 = w0; s0 < w0 + WS; s0 += span) {
      const int64_t first = s0 + lane * V;
      uint64_t best = KEY_NONE;
      int64_t it = 0;
      for (; it + 4 * WL <= span; it += 4 * WL) {
        uint64_t a0, b0, a1, b1, a2, b2, a3, b3;
        load2_key<ALIGNED>(S, first + it, m, a0, b0);
        load2_key<ALIGNED>(S, first + it + WL, m, a1, b1);
        load2_key<ALIGNED>(S, first + it + 2 * WL, m, a2, b2);
        load2_key<ALIGNED>(S, first + it + 3 * WL, m, a3, b3);
        best = umin64(best, umin64(umin64(a0, b0), umin64(a1, b1)));
        best = umin64(best, umin64(umin64(a2, b2), umin64(a3, b3)));
      }
      for (; it < span; it += WL) {
        uint64_t a, b;
        load2_key<ALIGNED>(S, first + it, m, a, b);
        best = umin64(best, umin64(a, b));
      }
      uint64_t key = group_min_u64<64>(best);
      if (k > WS) {
        if (lane == 63) part[wave] = key;
      } else if (lane == 63 && s0 < m) {
        keys[s0 >> kshift] = key;
      }
    }
    if (k > WS) {
      __syncthreads();
      if (threadIdx.x == 0) {
        uint64_t b = umin64(umin64(part[0], part[1]), umin64(part[2], part[3]));
        if (wg * C < m) keys[wg] = b;
      }
    }
  } else {
    const int g = (int)(k / V);
    for (int64_t it = 0; it < WS; it += WL) {
      const int64_t first = w0 + it + lane * V;
      uint64_t a, b;
      load2_key<ALIGNED>(S, first, m, a, b);
      uint64_t key = group_min_u64_rt(umin64(a, b), g);
      const int64_t blk_start = first - (int64_t)(lane % g) * V;
      if ((lane % g) == g - 1 && blk_start < m) keys[blk_start >> kshift] = key;
    }
  }
}

template <bool ALIGNED>
__global__ __launch_bounds__(WG) void k_blockmin_keys(const uint64_t* __restrict__ S, int64_t m,
                                                      int kshift, uint64_t* __restrict__ keys) {
  __shared__ uint64_t part[4];
  blockmin_keys_wg<ALIGNED>(S, m, kshift, keys, blockIdx.x, part);
}

// Two block levels in a batch: the k-block minima of each such array from
// its k1-block minima; workgroup w does job w.
__global__ __launch_bounds__(WG) void k_blockmin_keys_multi(const ChunkJob* __restrict__ jobs) {
  __shared__ uint64_t part[4];
  const ChunkJob jb = jobs[blockIdx.x];
  blockmin_keys_wg<true>(static_cast<const uint64_t*>(jb.src), jb.len, jb.shift, jb.keys,
                         jb.chunk, part);
}

}  // namespace

int64_t blockmin_grid(int64_t n, int kshift, int elems_per_lane_load) {
  const int64_t k = 1ll << kshift;
  const int64_t WL = 64ll * elems_per_lane_load;
  const int64_t C = k > 4 * WL ? k : 16 * WL;
  return (n + C - 1) / C;
}

hipError_t launch_blockmin_i32(const int32_t* A, int64_t n, int kshift, uint64_t* keys,
                               hipStream_t stream) {
  const int64_t grid = blockmin_grid(n, kshift, 4);
  if (grid <= 0) return hipSuccess;
  if (((uintptr_t)A & 15) == 0)
    RMQ_TRY(launch(k_blockmin_i32<true>, dim3((unsigned)grid), dim3(WG), 0, stream, A, n,
                       kshift, keys));
  else
    RMQ_TRY(launch(k_blockmin_i32<false>, dim3((unsigned)grid), dim3(WG), 0, stream, A, n,
                       kshift, keys));
  return hipGetLastError();
}

hipError_t launch_blockmin_multi(const ChunkJob* jobs, int64_t count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int64_t grid = (count + MULTI_JOBS - 1) / MULTI_JOBS;
  RMQ_TRY(launch(k_blockmin_multi, dim3((unsigned)grid), dim3(WG), 0, stream, jobs, count));
  return hipSuccess;
}

hipError_t launch_blockmin_keys_multi(const ChunkJob* jobs, int64_t count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  RMQ_TRY(launch(k_blockmin_keys_multi, dim3((unsigned)count), dim3(WG), 0, stream, jobs));
  return hipSuccess;
}

int64_t blockmin_keys_grid(int64_t m, int kshift) { return blockmin_grid(m, kshift, 2); }

hipError_t launch_blockmin_keys(const uint64_t* S, int64_t m, int kshift, uint64_t* keys,
                                hipStream_t stream) {
  const int64_t grid = blockmin_grid(m, kshift, 2);
  if (grid <= 0) return hipSuccess;
  if (((uintptr_t)S & 15) == 0)
    RMQ_TRY(launch(k_blockmin_keys<true>, dim3((unsigned)grid), dim3(WG), 0, stream, S, m,
                       kshift, keys));
  else
    RMQ_TRY(launch(k_blockmin_keys<false>, dim3((unsigned)grid), dim3(WG), 0, stream, S, m,
                       kshift, keys));
  return hipGetLastError();
}

}  // namespace rmq
