// Device LSD radix sort of the 2q query endpoints, and the remap that follows
// it (Section 3.1 step 1).
//
// Item j of the endpoint list is (position, tag j): the left end of query i
// is item 2i and its right end item 2i+1.  Sorting by position with a STABLE
// sort keeps equal positions in tag order, so the result is ordered by
// (position, tag) -- the same order any sort on the pair gives.
//
// Each pass handles 8 bits of the position (ceil(log2 n) bits in all) with
// three kernels and no inter-workgroup waiting:
//   count   -- per-tile digit histogram (LDS atomics), stored digit-major;
//   rowscan -- one workgroup per digit turns its row of tile counts into
//              exclusive offsets and a digit total;
//   scatter -- recomputes stable ranks inside the tile (8 wave ballots give
//              the lanes that share a digit), stages the tile in LDS in
//              digit order and writes runs of equal digits contiguously.
// Tiles are 4096 items: 4 waves x 16 rounds x 64 lanes, each wave owning a
// contiguous quarter so that (wave, round, lane) order is item order.
// Workgroups are dealt round-robin over the 8 XCDs; tiles are numbered so that
// each XCD gets a contiguous range of them, so the runs that neighbouring
// tiles write for one digit meet in the same L2 and leave it as whole lines.
//
// Remap: slot s of the sorted list holding tag t gives Lc[t/2] = s (t even)
// or Rc[t/2] = s - 1 (t odd).  Written directly these are 2q scattered 4-byte
// stores; instead one more radix pass orders the (tag, slot) pairs by the top
// bits of the tag, and the stores then go out window by window, each window
// of the interleaved LR array written while it sits in one XCD's L2.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;
constexpr int ROUNDS = 16;
constexpr int TILE = WG * ROUNDS;  // items per tile
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int NXCD = 8;

// where a pass takes its items from
enum Mode : int {
  ARRAYS = 0,   // keys_in[j], vals_in[j]
  QUERIES = 1,  // item j = (L[j/2] or R[j/2], j)
  KEY_IDX = 2,  // keys_in[j], value j
};

// Tile handled by this workgroup: XCD x = blockIdx % 8 takes the x-th
// contiguous range of tiles.  Returns -1 for the padding workgroups.
__device__ __forceinline__ int64_t xcd_tile(int64_t num_tiles) {
  const int64_t per = (num_tiles + NXCD - 1) / NXCD;
  const int64_t t = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  return t < num_tiles ? t : -1;
}
int64_t xcd_grid(int64_t num_tiles) { return ((num_tiles + NXCD - 1) / NXCD) * NXCD; }

__device__ __forceinline__ int64_t item_index(int64_t tile0, int wave, int round, int lane) {
  return tile0 + (int64_t)wave * (64 * ROUNDS) + round * 64 + lane;
}

// Item j read straight from the queries.  Lanes 2i and 2i+1 of a round hold
// the two ends of one query, so validity is shared through a lane swap.
__device__ __forceinline__ void load_from_queries(const int32_t* __restrict__ L,
                                                  const int32_t* __restrict__ R, int64_t N,
                                                  int64_t n, int64_t j, uint32_t& key,
                                                  uint32_t& val) {
  int32_t x = 0;
  if (j < N) x = (j & 1) ? R[j >> 1] : L[j >> 1];
  const int32_t other = __shfl_xor(x, 1);
  const int32_t l = (j & 1) ? other : x, r = (j & 1) ? x : other;
  const bool ok = 0 <= l && l <= r && (int64_t)r < n;
  key = ok ? (uint32_t)x : 0u;
  val = (uint32_t)j;
}

template <int MODE>
__device__ __forceinline__ void load_item(const uint32_t* __restrict__ keys_in,
                                          const uint32_t* __restrict__ vals_in,
                                          const int32_t* __restrict__ L,
                                          const int32_t* __restrict__ R, int64_t N, int64_t n,
                                          int64_t j, uint32_t& key, uint32_t& val) {
  if (MODE == QUERIES) {
    load_from_queries(L, R, N, n, j, key, val);
  } else {
    const bool valid = j < N;
    key = valid ? keys_in[j] : 0u;
    val = MODE == KEY_IDX ? (uint32_t)j : (valid ? vals_in[j] : 0u);
  }
}

template <int MODE>
__global__ __launch_bounds__(WG) void k_radix_count(const uint32_t* __restrict__ keys_in,
                                                    const int32_t* __restrict__ L,
                                                    const int32_t* __restrict__ R, int64_t N,
                                                    int64_t n, int shift, int bits,
                                                    uint32_t* __restrict__ counts,
                                                    int64_t num_tiles) {
  __shared__ uint32_t hist[RADIX];
  const int64_t tile = xcd_tile(num_tiles);
  if (tile < 0) return;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t tile0 = tile * TILE;
  const uint32_t mask = (1u << bits) - 1u;
  hist[threadIdx.x] = 0;
  __syncthreads();
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int64_t j = item_index(tile0, wave, rd, lane);
    uint32_t key, val;
    load_item<MODE == QUERIES ? QUERIES : KEY_IDX>(keys_in, nullptr, L, R, N, n, j, key, val);
    if (j < N) atomicAdd(&hist[(key >> shift) & mask], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * num_tiles + tile] = hist[threadIdx.x];
}

// Exclusive scan of 256 values held one per thread; returns the total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp,
                                                         uint32_t& excl) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
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

__global__ __launch_bounds__(WG) void k_radix_rowscan(uint32_t* __restrict__ counts,
                                                      int64_t num_tiles,
                                                      uint32_t* __restrict__ row_total) {
  __shared__ uint32_t tmp[WG / 64];
  uint32_t* row = counts + (int64_t)blockIdx.x * num_tiles;
  uint32_t carry = 0;
  for (int64_t base = 0; base < num_tiles; base += 4 * WG) {
    uint32_t v[4], s = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t t = base + threadIdx.x * 4 + c;
      v[c] = t < num_tiles ? row[t] : 0u;
      s += v[c];
    }
    uint32_t excl;
    const uint32_t total = block_exclusive_scan(s, tmp, excl);
    uint32_t run = carry + excl;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t t = base + threadIdx.x * 4 + c;
      if (t < num_tiles) row[t] = run;
      run += v[c];
    }
    carry += total;
  }
  if (threadIdx.x == 0) row_total[blockIdx.x] = carry;
}

template <int MODE>
__global__ __launch_bounds__(WG) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const int32_t* __restrict__ L, const int32_t* __restrict__ R, int64_t N, int64_t n, int shift,
    int bits, const uint32_t* __restrict__ counts, const uint32_t* __restrict__ row_total,
    int64_t num_tiles, uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t wave_cnt[WG / 64][RADIX];
  __shared__ uint32_t local_start[RADIX];
  __shared__ uint32_t global_start[RADIX];
  __shared__ uint32_t tmp[WG / 64];
  __shared__ uint32_t s_key[TILE];
  __shared__ uint32_t s_val[TILE];

  const int64_t tile = xcd_tile(num_tiles);
  if (tile < 0) return;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t tile0 = tile * TILE;
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t lt = (1ull << lane) - 1ull;

#pragma unroll
  for (int w = 0; w < WG / 64; ++w) wave_cnt[w][threadIdx.x] = 0;
  __syncthreads();

  uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int64_t j = item_index(tile0, wave, rd, lane);
    const bool valid = j < N;
    load_item<MODE>(keys_in, vals_in, L, R, N, n, j, key[rd], val[rd]);
    const uint32_t d = (key[rd] >> shift) & mask;
    uint64_t match = ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = ballot(bit);
      match &= bit ? m : ~m;
    }
    const uint32_t before = wave_cnt[wave][d];
    rank[rd] = before + (uint32_t)__popcll(match & lt);
    const bool leader = (match >> lane) == 1ull;  // highest lane of its digit group
    if (valid && leader) wave_cnt[wave][d] = before + (uint32_t)__popcll(match);
  }
  __syncthreads();

  // per digit: offsets of the waves inside the tile, then digit order in the tile
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < WG / 64; ++w) {
      const uint32_t c = wave_cnt[w][d];
      wave_cnt[w][d] = run;
      run += c;
    }
    uint32_t excl;
    block_exclusive_scan(run, tmp, excl);
    local_start[d] = excl;
    uint32_t base_excl;
    block_exclusive_scan(row_total[d], tmp, base_excl);
    global_start[d] = base_excl + counts[(int64_t)d * num_tiles + tile];
  }
  __syncthreads();

#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int64_t j = item_index(tile0, wave, rd, lane);
    if (j < N) {
      const uint32_t d = (key[rd] >> shift) & mask;
      const uint32_t lp = local_start[d] + wave_cnt[wave][d] + rank[rd];
      if (lp < (uint32_t)TILE) {  // always true for consistent ranks
        s_key[lp] = key[rd];
        s_val[lp] = val[rd];
      }
    }
  }
  __syncthreads();

  const int64_t tile_n = N - tile0 < TILE ? N - tile0 : TILE;
  for (int t = threadIdx.x; t < tile_n; t += WG) {
    const uint32_t k = s_key[t];
    const uint32_t d = (k >> shift) & mask;
    const uint32_t dst = global_start[d] + (uint32_t)t - local_start[d];
    if ((int64_t)dst < N) {  // always true for consistent counts
      keys_out[dst] = k;
      vals_out[dst] = s_val[t];
    }
  }
}

// Remap writes from (tag, slot) pairs ordered by the top bits of the tag.
__global__ __launch_bounds__(WG) void k_remap_apply(const uint32_t* __restrict__ tags,
                                                    const uint32_t* __restrict__ slots,
                                                    int64_t N, int32_t* __restrict__ LR,
                                                    int64_t num_chunks) {
  const int64_t chunk = xcd_tile(num_chunks);
  if (chunk < 0) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t j = chunk * (4 * WG) + i * WG + threadIdx.x;
    if (j < N) {
      const uint32_t t = tags[j], s = slots[j];
      if ((int64_t)t < N) LR[t] = (t & 1u) ? (int32_t)s - 1 : (int32_t)s;
    }
  }
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
  int64_t N, num_tiles;
  size_t off_key, off_val, off_counts, off_total, bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SortLayout sort_layout(int64_t q) {
  SortLayout s{};
  s.N = 2 * q;
  s.num_tiles = (s.N + TILE - 1) / TILE;
  size_t o = 0;
  s.off_key = o;
  o = align256(o + sizeof(uint32_t) * (size_t)s.N);
  s.off_val = o;
  o = align256(o + sizeof(uint32_t) * (size_t)s.N);
  s.off_counts = o;
  o = align256(o + sizeof(uint32_t) * (size_t)RADIX * (size_t)s.num_tiles);
  s.off_total = o;
  o = align256(o + sizeof(uint32_t) * RADIX);
  s.bytes = o;
  return s;
}

struct SortBufs {
  uint32_t *tkey, *tval, *counts, *total;
};

SortBufs sort_bufs(const SortLayout& lay, void* ws) {
  char* base = static_cast<char*>(ws);
  return {reinterpret_cast<uint32_t*>(base + lay.off_key),
          reinterpret_cast<uint32_t*>(base + lay.off_val),
          reinterpret_cast<uint32_t*>(base + lay.off_counts),
          reinterpret_cast<uint32_t*>(base + lay.off_total)};
}

// One stable pass: count, scan, scatter.
template <int MODE>
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, const int32_t* L, const int32_t* R,
                      int64_t N, int64_t n, int shift, int bits, const SortLayout& lay,
                      const SortBufs& b, uint32_t* kout, uint32_t* vout, hipStream_t stream) {
  const dim3 grid((unsigned)xcd_grid(lay.num_tiles)), block(WG);
  RMQ_TRY(launch(k_radix_count<MODE>, grid, block, 0, stream, kin, L, R, N, n, shift, bits,
                 b.counts, lay.num_tiles));
  // all RADIX rows, so that digits unused by a short pass get total 0
  RMQ_TRY(launch(k_radix_rowscan, dim3(RADIX), block, 0, stream, b.counts, lay.num_tiles,
                 b.total));
  RMQ_TRY(launch(k_radix_scatter<MODE>, grid, block, 0, stream, kin, vin, L, R, N, n, shift,
                 bits, b.counts, b.total, lay.num_tiles, kout, vout));
  return hipSuccess;
}

}  // namespace

size_t sort_workspace_bytes(int64_t q) { return q > 0 ? sort_layout(q).bytes : 0; }

hipError_t launch_sort_endpoints(const int32_t* L, const int32_t* R, int64_t q, int64_t n,
                                 int32_t* pos, int32_t* tag, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const SortLayout lay = sort_layout(q);
  if (ws_bytes < lay.bytes) return hipErrorInvalidValue;
  const SortBufs b = sort_bufs(lay, ws);
  uint32_t* okey = reinterpret_cast<uint32_t*>(pos);
  uint32_t* oval = reinterpret_cast<uint32_t*>(tag);

  const int nbits = n > 1 ? bit_length((uint64_t)(n - 1)) : 1;
  const int passes = (nbits + RADIX_BITS - 1) / RADIX_BITS;
  const uint32_t* src_k = nullptr;
  const uint32_t* src_v = nullptr;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RADIX_BITS;
    const int bits = nbits - shift < RADIX_BITS ? nbits - shift : RADIX_BITS;
    // passes alternate between the scratch pair and the output pair so that
    // the last one lands in the output
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t* dk = to_out ? okey : b.tkey;
    uint32_t* dv = to_out ? oval : b.tval;
    if (p == 0)
      RMQ_TRY(radix_pass<QUERIES>(nullptr, nullptr, L, R, lay.N, n, shift, bits, lay, b, dk, dv,
                                  stream));
    else
      RMQ_TRY(radix_pass<ARRAYS>(src_k, src_v, nullptr, nullptr, lay.N, n, shift, bits, lay, b,
                                 dk, dv, stream));
    src_k = dk;
    src_v = dv;
  }
  return hipSuccess;
}

hipError_t launch_remap(const int32_t* tag, int64_t q, int32_t* LR, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  if (q <= 0) return hipSuccess;
  const SortLayout lay = sort_layout(q);
  if (ws_bytes < lay.bytes) return hipErrorInvalidValue;
  const SortBufs b = sort_bufs(lay, ws);
  const int tbits = lay.N > 1 ? bit_length((uint64_t)(lay.N - 1)) : 1;
  const int shift = tbits > RADIX_BITS ? tbits - RADIX_BITS : 0;
  RMQ_TRY(radix_pass<KEY_IDX>(reinterpret_cast<const uint32_t*>(tag), nullptr, nullptr, nullptr,
                              lay.N, 0, shift, tbits - shift, lay, b, b.tkey, b.tval, stream));
  const int64_t chunks = (lay.N + 4 * WG - 1) / (4 * WG);
  RMQ_TRY(launch(k_remap_apply, dim3((unsigned)xcd_grid(chunks)), dim3(WG), 0, stream, b.tkey,
                 b.tval, lay.N, LR, chunks));
  return hipSuccess;
}

}  // namespace rmq
