// A measurement aid, not a step of the method: the achievable streaming-read
// rate of this part for the block-minima pass.
#include "device.h"
#include "kernels.h"

namespace rmq {

constexpr int WG = 256;

// The achievable streaming-read rate of this part, to set block minima
// against: the same 16-byte non-temporal loads and per-wave span as the
// block-minima pass (four 1 KB wave loads per wave), with only a fold of
// the data kept (written only if it hits an impossible value, so that the
// loads stay live).
namespace {
__global__ __launch_bounds__(WG) void k_read_probe(const int32_t* __restrict__ A, int64_t n4,
                                                   uint32_t* __restrict__ sink) {
  const int64_t wave = ((int64_t)blockIdx.x * WG + threadIdx.x) >> 6;
  const int64_t base = wave * 256 + lane_id();
  uint32_t acc = 0;
  v4i32 x[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = base + u * 64;
    x[u] = load_stream(A + 4 * (i < n4 ? i : n4 - 1));
  }
  __builtin_amdgcn_sched_barrier(0);  // all four loads in flight before any use
#pragma unroll
  for (int u = 0; u < 4; ++u) acc += (uint32_t)(x[u].x ^ x[u].y ^ x[u].z ^ x[u].w);
  if (acc == 0x9E3779B9u && base < n4) sink[0] = acc;
}
}  // namespace

hipError_t launch_read_probe(const int32_t* A, int64_t n, uint32_t* sink, hipStream_t stream) {
  const int64_t n4 = n / 4;
  if (n4 < 1) return hipSuccess;
  const int64_t waves = (n4 + 255) / 256;
  RMQ_TRY(launch(k_read_probe, dim3((unsigned)((waves * 64 + WG - 1) / WG)), dim3(WG), 0, stream, A,
                 n4, sink));
  return hipSuccess;
}

}  // namespace rmq
