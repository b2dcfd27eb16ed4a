// Block Sparse Table (Section 3.1 step 3; Section 2, the doubling of Bender
// and Farach): st[j][b] = min(st[0][b .. min(b + 2^j, nb) - 1]), level-major.
// The table over powers of l (Section 3.1's generalisation) is at the end.
//
// A round computes t consecutive levels j0+1 .. j0+t from level j0 inside
// LDS.  With stride s = 2^j0, level j0+m at block b is the min of level j0 at
// b, b+s, ..., b+(2^m - 1)s, so the work splits into the s residue classes
// b mod s.  A workgroup takes R adjacent residues (one contiguous row of R
// keys per class index i, so global accesses stay coalesced) and TI rows
// i0 .. i0+TI-1, plus a halo of 2^t - 1 rows below; it then doubles t times
// in LDS (ping-pong buffers) and writes each level's TI rows.  Keys past the
// last block read as the min identity, which gives exactly the truncated
// spans at the end of the table.  Round r starts at the same j0 for every
// table (0, 10, 16, 22, ...), so the rounds of many tables batch into one
// launch each.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;
// The doubling rounds' workgroups: 16 waves, so that a small table's one or
// two tiles still spread their per-level LDS work over every SIMD of a CU.
constexpr int STWG = 1024;
constexpr int TILE = 1024;  // outputs per workgroup per level (R * TI)

struct RoundShape {
  int j0, R, TI, tmax;
};

// Largest t such that the halo fits: rows TI + 2^t - 1 <= 2 * TI.
int levels_per_round(int TI) {
  int t = 0;
  while ((2 << t) - 1 <= TI) ++t;
  return t;
}

RoundShape round_shape(int r) {
  RoundShape s{0, 1, TILE, 0};
  for (int i = 0;; ++i) {
    const int64_t stride = 1ll << s.j0;
    s.R = (int)(stride < 16 ? stride : 16);
    s.TI = TILE / s.R;
    s.tmax = levels_per_round(s.TI);
    if (i == r) return s;
    s.j0 += s.tmax;
  }
}

__device__ __forceinline__ void st_tile(uint64_t* __restrict__ st, int64_t nb, int j0, int t,
                                        int R, int64_t col_tiles, int64_t tile_idx,
                                        uint64_t* lds) {
  const int64_t s = 1ll << j0;
  const int TI = TILE / R;
  const int H = (1 << t) - 1;
  const int rows = TI + H;
  uint64_t* buf0 = lds;
  uint64_t* buf1 = lds + (size_t)rows * R;

  const int64_t tile_c = tile_idx % col_tiles;
  const int64_t tile_r = tile_idx / col_tiles;
  const int64_t r0 = tile_c * R;
  // R is a power of two (min(stride, 16)): rows and columns of an LDS index
  // by shift and mask (a run-time division per entry and level was most of
  // a small table's build time)
  const int rs = __builtin_ctz((unsigned)R);
  const int64_t i0 = tile_r * TI;
  const uint64_t* src = st + (size_t)j0 * nb;

  // all loads first (rows * R <= 2 * TILE entries, at most LOADS per
  // thread), so that they are in flight together
  constexpr int LOADS = 2 * TILE / STWG;
  uint64_t v[LOADS];
#pragma unroll
  for (int u = 0; u < LOADS; ++u) {
    const int idx = threadIdx.x + u * STWG;
    const int row = idx >> rs, c = idx & (R - 1);
    const int64_t r = r0 + c;
    const int64_t b = ((i0 + row) << j0) + r;
    const bool ok = idx < rows * R && r < s && b < nb;
    v[u] = src[ok ? b : 0];
    if (!ok) v[u] = KEY_NONE;
  }
#pragma unroll
  for (int u = 0; u < LOADS; ++u) {
    const int idx = threadIdx.x + u * STWG;
    if (idx < rows * R) buf0[idx] = v[u];
  }
  __syncthreads();

  uint64_t* cur = buf0;
  uint64_t* nxt = buf1;
  for (int m = 1; m <= t; ++m) {
    const int half = 1 << (m - 1);
    const int rows_m = TI + H - ((1 << m) - 1);  // rows still needed by later levels
    uint64_t* dst = st + (size_t)(j0 + m) * nb;
    // unrolled, so the LDS reads of all of a thread's entries overlap
    uint64_t w[LOADS];
#pragma unroll
    for (int u = 0; u < LOADS; ++u) {
      const int idx = threadIdx.x + u * STWG;
      if (idx < rows_m * R) w[u] = umin64(cur[idx], cur[idx + half * R]);
    }
#pragma unroll
    for (int u = 0; u < LOADS; ++u) {
      const int idx = threadIdx.x + u * STWG;
      if (idx < rows_m * R) {
        nxt[idx] = w[u];
        const int row = idx >> rs, c = idx & (R - 1);
        if (row < TI) {
          const int64_t r = r0 + c;
          const int64_t b = ((i0 + row) << j0) + r;
          if (r < s && b < nb) dst[b] = w[u];
        }
      }
    }
    __syncthreads();
    uint64_t* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

__global__ __launch_bounds__(STWG) void k_st_levels(uint64_t* __restrict__ st, int64_t nb, int j0,
                                                  int t, int R, int64_t col_tiles) {
  extern __shared__ uint64_t lds[];
  st_tile(st, nb, j0, t, R, col_tiles, blockIdx.x, lds);
}

// Round `round` of every table of a batch: workgroup w does job w, one
// tile of one table.
__global__ __launch_bounds__(STWG) void k_st_multi(const TileJob* __restrict__ jobs, int j0, int R,
                                                 int tmax) {
  extern __shared__ uint64_t lds[];
  const TileJob jb = jobs[blockIdx.x];
  const int t = jb.levels - 1 - j0 < tmax ? jb.levels - 1 - j0 : tmax;
  const int64_t s = 1ll << j0;
  const int64_t col_tiles = (s + R - 1) / R;
  st_tile(jb.st, jb.nb, j0, t, R, col_tiles, jb.tile, lds);
}

// Division of a < 2^31 by a divisor fixed for the launch, d >= 1: with
// e = ceil(log2 d) and m = ceil(2^(31+e) / d) < 2^32, floor(a / d) =
// (a * m) >> (31 + e) (the round-up method of Granlund and Montgomery).
struct Divisor {
  uint32_t d, m;
  int shift;
};
Divisor make_divisor(uint32_t d) {
  int e = 0;
  while ((1ull << e) < d) ++e;
  const unsigned __int128 num = (unsigned __int128)1 << (31 + e);
  return Divisor{d, (uint32_t)((num + d - 1) / d), 31 + e};
}
__device__ __forceinline__ uint32_t div_by(uint32_t a, const Divisor& v) {
  return (uint32_t)(((uint64_t)a * v.m) >> v.shift);
}

// Block b of the a-th stored entry of a level whose windows span 2^sh blocks:
// b = p * 2^sh + r for the p-th entry of class r; the first nb mod 2^sh
// classes (`long_cls.d` = base + 1 entries each) come before the others
// (`short_cls.d` = base entries each).  Also the class length.
__device__ __forceinline__ int64_t lary_block(uint32_t a, uint32_t nb, int sh,
                                              const Divisor& long_cls, const Divisor& short_cls,
                                              uint32_t* p_out = nullptr,
                                              uint32_t* len_out = nullptr) {
  const uint32_t rem = nb & ((1u << sh) - 1), big = rem * long_cls.d;
  uint32_t r, p, len;
  if (a < big) {
    r = div_by(a, long_cls);
    p = a - r * long_cls.d;
    len = long_cls.d;
  } else {
    const uint32_t c = div_by(a - big, short_cls);
    r = rem + c;
    p = a - big - c * short_cls.d;
    len = short_cls.d;
  }
  if (p_out) *p_out = p;
  if (len_out) *len_out = len;
  return ((int64_t)p << sh) + r;
}

constexpr int LARY_TILE = 1024;  // entries of level i-1 per workgroup

// One level of the table over powers of l = 2^lg (Section 3.1): level i at
// block b is the min of level i-1 at b, b + s', ..., b + (l-1)s' with
// s' = l^(i-1), entries past the last block left out (truncated spans, as in
// the doubling table).  Level i-1 is stored by residue class mod s'
// (lary_addr), so these terms are l adjacent entries of one class: a window
// of width l sliding along the class, cut at the class's end.  A workgroup
// stages LARY_TILE consecutive entries of level i-1 plus the l - 1 after
// them in LDS (each entry read once from HBM) and makes the window minimum
// starting at each of its entries, written to block b's place in level i
// (within a wave: l classes of level i, adjacent positions in each).
__global__ __launch_bounds__(WG) void k_st_lary(const uint64_t* __restrict__ prev,
                                                uint64_t* __restrict__ cur, uint32_t nb, int sh,
                                                int lg, Divisor long_cls, Divisor short_cls) {
  __shared__ uint64_t tile[LARY_TILE + 32];
  constexpr int LOADS = (LARY_TILE + 32 + WG - 1) / WG;
  const int l = 1 << lg;
  const int psh = sh - lg;
  const int64_t x0 = (int64_t)blockIdx.x * LARY_TILE;
  uint64_t v[LOADS];
#pragma unroll
  for (int u = 0; u < LOADS; ++u) {
    const int64_t x = x0 + u * WG + threadIdx.x;
    v[u] = prev[x < (int64_t)nb ? x : 0];
    if (x >= (int64_t)nb) v[u] = KEY_NONE;
  }
#pragma unroll
  for (int u = 0; u < LOADS; ++u) {
    const int idx = u * WG + threadIdx.x;
    if (idx < LARY_TILE + l - 1) tile[idx] = v[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < LARY_TILE / WG; ++u) {
    const int idx = u * WG + threadIdx.x;
    const int64_t x = x0 + idx;
    if (x >= (int64_t)nb) break;
    // entry x of level i-1: block b, p-th of its class, class length len
    uint32_t p, len;
    const int64_t b = lary_block((uint32_t)x, nb, psh, long_cls, short_cls, &p, &len);
    const int cnt = (int)(len - p) < l ? (int)(len - p) : l;  // terms inside the class
    uint64_t m = tile[idx];
#pragma unroll 8
    for (int j = 1; j < cnt; ++j) m = umin64(m, tile[idx + j]);
    cur[lary_addr(b, nb, sh)] = m;
  }
}

// Query records: one thread per key, in record order (coalesced writes);
// the table reads are gathers from a table small enough for L2.
// (Records are built only while they take at most 8 MiB, so pair indices
// stay below 2^31 and divide by the level count through a Divisor.)
__global__ __launch_bounds__(WG) void k_records(const uint64_t* __restrict__ st, int64_t nb,
                                                int levels, Divisor lv,
                                                uint64_t* __restrict__ rec) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= 4 * nb * levels) return;
  const int64_t pair = e >> 1;
  // record: forward 0 .. nb-1, backward nb .. 2nb-1
  const int64_t rb = div_by((uint32_t)pair, lv);
  const int t = (int)(pair - rb * levels);
  const bool fwd = rb < nb;
  const int64_t b = fwd ? rb : rb - nb;
  uint64_t v = KEY_NONE;
  if ((e & 1) == 0) {
    v = st[b];
  } else {
    const int64_t x = fwd ? b + 1 : b - (1ll << t);  // window start
    if (fwd ? x < nb : x >= 0) v = st[(size_t)t * nb + x];
  }
  rec[e] = v;
}

}  // namespace

hipError_t launch_records(const uint64_t* st, int64_t nb, int levels, uint64_t* rec,
                          hipStream_t stream) {
  const int64_t total = 4 * nb * levels;
  if (total / 2 >= (1ll << 31)) return hipErrorInvalidValue;  // never: records are at most 8 MiB
  RMQ_TRY(launch(k_records, dim3((unsigned)((total + WG - 1) / WG)), dim3(WG), 0, stream, st, nb,
                 levels, make_divisor((uint32_t)levels), rec));
  return hipSuccess;
}

int lary_levels(int64_t nb, int lg) {
  if (nb <= 3) return 1;
  int t = 0;  // floor(log2(nb - 2)): the largest inner span is nb - 2 blocks
  while ((int64_t)2 << t <= nb - 2) ++t;
  return t / lg + 1;
}

hipError_t launch_sparse_table_lary(uint64_t* st, int64_t nb, int lg, hipStream_t stream) {
  const int levels = lary_levels(nb, lg);
  if (nb >= ((int64_t)1 << 31)) return hipErrorInvalidValue;  // 32-bit index math
  const int64_t grid = (nb + LARY_TILE - 1) / LARY_TILE;
  for (int i = 1; i < levels; ++i) {
    // classes of level i-1 (mod l^(i-1)): base or base + 1 entries, base >= 1
    const uint32_t base = (uint32_t)(nb >> ((i - 1) * lg));
    RMQ_TRY(launch(k_st_lary, dim3((unsigned)grid), dim3(WG), 0, stream,
                   static_cast<const uint64_t*>(st + (size_t)(i - 1) * nb),
                   st + (size_t)i * nb, (uint32_t)nb, i * lg, lg, make_divisor(base + 1),
                   make_divisor(base)));
  }
  return hipSuccess;
}

int st_round_j0(int r) { return round_shape(r).j0; }

int st_rounds(int levels) {
  int r = 0;
  while (round_shape(r).j0 + 1 < levels) ++r;
  return r;
}

int64_t st_round_tiles(int64_t nb, int levels, int r) {
  const RoundShape sh = round_shape(r);
  if (sh.j0 + 1 >= levels) return 0;
  const int64_t s = 1ll << sh.j0;
  const int64_t col_tiles = (s + sh.R - 1) / sh.R;
  const int64_t rows_total = (nb + s - 1) / s;  // largest class length
  return col_tiles * ((rows_total + sh.TI - 1) / sh.TI);
}

size_t st_round_lds(int r) {
  const RoundShape sh = round_shape(r);
  return 2ull * (size_t)(sh.TI + (1 << sh.tmax) - 1) * sh.R * sizeof(uint64_t);
}

hipError_t launch_sparse_table(uint64_t* st, int64_t nb, int levels, hipStream_t stream) {
  for (int r = 0; r < st_rounds(levels); ++r) {
    const RoundShape sh = round_shape(r);
    const int t = sh.j0 + sh.tmax > levels - 1 ? levels - 1 - sh.j0 : sh.tmax;
    const int64_t s = 1ll << sh.j0;
    const int64_t col_tiles = (s + sh.R - 1) / sh.R;
    const int64_t grid = st_round_tiles(nb, levels, r);
    const size_t lds = 2ull * (size_t)(sh.TI + (1 << t) - 1) * sh.R * sizeof(uint64_t);
    RMQ_TRY(launch(k_st_levels, dim3((unsigned)grid), dim3(STWG), (uint32_t)lds, stream, st, nb,
                   sh.j0, t, sh.R, col_tiles));
  }
  return hipSuccess;
}

hipError_t launch_sparse_table_multi(const TileJob* jobs, int round, int64_t count,
                                     hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const RoundShape sh = round_shape(round);
  RMQ_TRY(launch(k_st_multi, dim3((unsigned)count), dim3(STWG), (uint32_t)st_round_lds(round),
                 stream, jobs, sh.j0, sh.R, sh.tmax));
  return hipSuccess;
}

}  // namespace rmq
