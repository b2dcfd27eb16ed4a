// Device-side building blocks shared by the kernels: the (value, position)
// key encoding, wave64 min reductions over DPP, and vector loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmq {

constexpr uint64_t KEY_NONE = ~0ull;  // identity of min over keys

// key(p) = ((uint32(v) ^ 0x80000000) << 32) | p: unsigned order of keys is the
// lexicographic order of (v, p), so min over keys = leftmost minimum.
__device__ __forceinline__ uint64_t make_key(int32_t v, uint32_t p) {
  return ((uint64_t)((uint32_t)v ^ 0x80000000u) << 32) | (uint64_t)p;
}
__device__ __forceinline__ uint32_t key_pos(uint64_t k) { return (uint32_t)k; }

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Where block b's entry sits in a level of the table over powers of l whose
// windows span s = 2^sh blocks: levels are stored by residue class (b mod s
// first, then b / s), so the windows b, b + s, b + 2s, ... that a query or the
// next level's build reads are adjacent.  Classes r < nb mod s hold one more
// entry than the others; the map is a permutation of [0, nb).  sh = 0 is the
// identity (level 0, the block minima).
__host__ __device__ __forceinline__ int64_t lary_addr(int64_t b, int64_t nb, int sh) {
  const int64_t m = (1ll << sh) - 1;
  const int64_t r = b & m, rem = nb & m;
  return r * (nb >> sh) + (r < rem ? r : rem) + (b >> sh);
}

// ---- DPP moves of a 64-bit value (gfx9 DPP control codes) ------------------
enum : int {
  DPP_QUAD_XOR1 = 0xB1,        // quad_perm [1,0,3,2]
  DPP_QUAD_XOR2 = 0x4E,        // quad_perm [2,3,0,1]
  DPP_ROW_HALF_MIRROR = 0x141,  // lane i <-> 7-i within 8
  DPP_ROW_MIRROR = 0x140,       // lane i <-> 15-i within 16
  DPP_ROW_BCAST15 = 0x142,      // lane 15 of each row -> next row
  DPP_ROW_BCAST31 = 0x143,      // lane 31 -> rows 2 and 3
};

// Lanes whose DPP source is disabled keep their own value (old = src), so a
// following min() is a no-op for them.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// DPP move whose lanes without a source (outside the row for row shifts,
// lane 0 for the wave shift, rows masked off) read `ident` instead.
enum : int {
  DPP_ROW_SHR1 = 0x111,  // lane i <- i-1 within each row of 16
  DPP_ROW_SHR2 = 0x112,
  DPP_ROW_SHR4 = 0x114,
  DPP_ROW_SHR8 = 0x118,
  DPP_WAVE_SHR1 = 0x138,  // lane i <- i-1 across the wave
};
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32_id(uint32_t v, uint32_t ident) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64_id(uint64_t v, uint64_t ident) {
  const uint32_t lo = dpp_u32_id<CTRL, ROW_MASK>((uint32_t)v, (uint32_t)ident);
  const uint32_t hi = dpp_u32_id<CTRL, ROW_MASK>((uint32_t)(v >> 32), (uint32_t)(ident >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive segmented min-scan over the wave: lane l ends with the min of v
// over lanes s..l, s the last lane <= l with a set flag (lane 0 if none).
// Row shifts 1, 2, 4, 8 scan each row of 16; broadcasts of lanes 15 and 31
// join the rows.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_min_step(uint64_t& v, uint32_t& f) {
  const uint64_t vu = dpp_u64_id<CTRL, ROW_MASK>(v, KEY_NONE);
  const uint32_t fu = dpp_u32_id<CTRL, ROW_MASK>(f, 0u);
  v = f ? v : umin64(v, vu);
  f |= fu;
}
__device__ __forceinline__ uint64_t seg_scan_min_u64(uint64_t v, bool head) {
  uint32_t f = head ? 1u : 0u;
  seg_min_step<DPP_ROW_SHR1, 0xF>(v, f);
  seg_min_step<DPP_ROW_SHR2, 0xF>(v, f);
  seg_min_step<DPP_ROW_SHR4, 0xF>(v, f);
  seg_min_step<DPP_ROW_SHR8, 0xF>(v, f);
  seg_min_step<DPP_ROW_BCAST15, 0xA>(v, f);
  seg_min_step<DPP_ROW_BCAST31, 0xC>(v, f);
  return v;
}

// Inclusive prefix sum over the wave (same DPP pattern).
__device__ __forceinline__ uint32_t wave_inclusive_add_u32(uint32_t x) {
  x += dpp_u32_id<DPP_ROW_SHR1, 0xF>(x, 0u);
  x += dpp_u32_id<DPP_ROW_SHR2, 0xF>(x, 0u);
  x += dpp_u32_id<DPP_ROW_SHR4, 0xF>(x, 0u);
  x += dpp_u32_id<DPP_ROW_SHR8, 0xF>(x, 0u);
  x += dpp_u32_id<DPP_ROW_BCAST15, 0xA>(x, 0u);
  x += dpp_u32_id<DPP_ROW_BCAST31, 0xC>(x, 0u);
  return x;
}

// Min over aligned groups of G lanes (G = 1..64, power of two).  Afterwards
// the LAST lane of each group (lane % G == G-1) holds the group's minimum
// (for G <= 16 every lane of the group does).
template <int G>
__device__ __forceinline__ uint64_t group_min_u64(uint64_t v) {
  if constexpr (G >= 2) v = umin64(v, dpp_u64<DPP_QUAD_XOR1>(v));
  if constexpr (G >= 4) v = umin64(v, dpp_u64<DPP_QUAD_XOR2>(v));
  if constexpr (G >= 8) v = umin64(v, dpp_u64<DPP_ROW_HALF_MIRROR>(v));
  if constexpr (G >= 16) v = umin64(v, dpp_u64<DPP_ROW_MIRROR>(v));
  if constexpr (G >= 32) v = umin64(v, dpp_u64<DPP_ROW_BCAST15, 0xA>(v));
  if constexpr (G >= 64) v = umin64(v, dpp_u64<DPP_ROW_BCAST31, 0xC>(v));
  return v;
}

// Runtime group size dispatch (uniform across the wave).
__device__ __forceinline__ uint64_t group_min_u64_rt(uint64_t v, int g) {
  switch (g) {
    case 1: return v;
    case 2: return group_min_u64<2>(v);
    case 4: return group_min_u64<4>(v);
    case 8: return group_min_u64<8>(v);
    case 16: return group_min_u64<16>(v);
    case 32: return group_min_u64<32>(v);
    default: return group_min_u64<64>(v);
  }
}

// Full-wave minimum, broadcast to every lane.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  v = group_min_u64<64>(v);
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Wave-uniform broadcast of a 64-bit register from lane `src` (src uniform).
__device__ __forceinline__ int64_t readlane64(int64_t v, int src) {
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, src);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));

// Streaming 16-byte loads with the non-temporal hint (each byte of the input
// is read once per pass).
__device__ __forceinline__ v4i32 load_stream(const int32_t* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(p));
}
__device__ __forceinline__ v2u64 load_stream(const uint64_t* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const v2u64*>(p));
}

// Largest j in [0, count) with prefix[j] <= x, for a non-decreasing prefix
// table with prefix[0] = 0 (binary search; the table stays in cache).
__device__ __forceinline__ int find_item(const int64_t* __restrict__ prefix, int count,
                                         int64_t x) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// find_item for every lane of a wave whose lanes hold consecutive x (a
// wave's share of a concatenated list): one search for the wave's first x
// with wave-uniform values (scalar loads), then each lane steps forward past
// the few boundaries inside the wave.  x_first: the wave's first x, clamped to
// [0, prefix[count]).
__device__ __forceinline__ int find_item_wave(const int64_t* __restrict__ prefix, int count,
                                              int64_t x_first, int64_t x) {
  const uint64_t u = (uint64_t)x_first;
  const int64_t xf = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(
                                    (int)(uint32_t)(u >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
  int j = find_item(prefix, count, xf);
  while (j + 1 < count && prefix[j + 1] <= x) ++j;
  return j;
}

// Floor log2 for x >= 1.
__device__ __forceinline__ int ilog2_u64(uint64_t x) { return 63 - __clzll(x); }

}  // namespace rmq
