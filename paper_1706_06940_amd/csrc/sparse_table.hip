// Block Sparse Table (Section 3.1 step 3; Section 2, the doubling of Bender
// and Farach): st[j][b] = min(st[0][b .. min(b + 2^j, nb) - 1]), level-major.
//
// A launch computes t consecutive levels j0+1 .. j0+t from level j0 inside
// LDS.  With stride s = 2^j0, level j0+m at block b is the min of level j0 at
// b, b+s, ..., b+(2^m - 1)s, so the work splits into the s residue classes
// b mod s.  A workgroup takes R adjacent residues (one contiguous row of R
// keys per class index i, so global accesses stay coalesced) and TI rows
// i0 .. i0+TI-1, plus a halo of 2^t - 1 rows below; it then doubles t times
// in LDS (ping-pong buffers) and writes each level's TI rows.  Keys past the
// last block read as the min identity, which gives exactly the truncated
// spans at the end of the table.
#include "device.h"
#include "kernels.h"

namespace rmq {

namespace {

constexpr int WG = 256;
constexpr int TILE = 1024;  // outputs per workgroup per level (R * TI)

__global__ __launch_bounds__(WG) void k_st_levels(uint64_t* __restrict__ st, int64_t nb, int j0,
                                                  int t, int R, int col_tiles) {
  extern __shared__ uint64_t lds[];
  const int64_t s = 1ll << j0;
  const int TI = TILE / R;
  const int H = (1 << t) - 1;
  const int rows = TI + H;
  uint64_t* buf0 = lds;
  uint64_t* buf1 = lds + (size_t)rows * R;

  const int64_t tile_c = blockIdx.x % col_tiles;
  const int64_t tile_r = blockIdx.x / col_tiles;
  const int64_t r0 = tile_c * R;
  const int64_t i0 = tile_r * TI;
  const uint64_t* src = st + (size_t)j0 * nb;

  for (int idx = threadIdx.x; idx < rows * R; idx += WG) {
    const int row = idx / R, c = idx % R;
    const int64_t r = r0 + c;
    const int64_t b = (i0 + row) * s + r;
    buf0[idx] = (r < s && b < nb) ? src[b] : KEY_NONE;
  }
  __syncthreads();

  uint64_t* cur = buf0;
  uint64_t* nxt = buf1;
  for (int m = 1; m <= t; ++m) {
    const int half = 1 << (m - 1);
    const int rows_m = TI + H - ((1 << m) - 1);  // rows still needed by later levels
    uint64_t* dst = st + (size_t)(j0 + m) * nb;
    for (int idx = threadIdx.x; idx < rows_m * R; idx += WG) {
      const uint64_t v = umin64(cur[idx], cur[idx + half * R]);
      nxt[idx] = v;
      const int row = idx / R, c = idx % R;
      if (row < TI) {
        const int64_t r = r0 + c;
        const int64_t b = (i0 + row) * s + r;
        if (r < s && b < nb) dst[b] = v;
      }
    }
    __syncthreads();
    uint64_t* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

}  // namespace

// Largest t such that the halo fits: rows TI + 2^t - 1 <= 2 * TI.
static int levels_per_launch(int TI) {
  int t = 0;
  while ((2 << t) - 1 <= TI) ++t;
  return t;
}

hipError_t launch_sparse_table(uint64_t* st, int64_t nb, int levels, hipStream_t stream) {
  int j0 = 0;
  while (j0 + 1 < levels) {
    const int64_t s = 1ll << j0;
    const int R = (int)(s < 16 ? s : 16);
    const int TI = TILE / R;
    int t = levels_per_launch(TI);
    if (j0 + t > levels - 1) t = levels - 1 - j0;
    const int64_t col_tiles = (s + R - 1) / R;
    const int64_t rows_total = (nb + s - 1) / s;  // largest class length
    const int64_t row_tiles = (rows_total + TI - 1) / TI;
    const int64_t grid = col_tiles * row_tiles;
    const size_t lds = 2ull * (size_t)(TI + (1 << t) - 1) * R * sizeof(uint64_t);
    hipLaunchKernelGGL(k_st_levels, dim3((unsigned)grid), dim3(WG), lds, stream, st, nb, j0, t, R,
                       (int)col_tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    j0 += t;
  }
  return hipSuccess;
}

}  // namespace rmq
