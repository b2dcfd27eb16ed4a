// Allocation-free form of rmq_query_batch_ex, for callers that may not
// allocate device memory (code under stream capture, tight serving loops).
//
// The per-call scratch of both methods (block minima and table, or the
// endpoint sort's buffers, LR, A_Q and its table) lives in one fixed device
// array of this library instead of the stream-ordered pool.  Every kernel of
// the two methods writes each scratch word it later reads within the same
// call (the sort clears its counters and status words with a kernel, the
// contraction sets the areas it finishes by atomics to +inf first), so the
// contents a previous call left behind never matter.
#include <mutex>

#include "device.h"
#include "rmq.h"

namespace {

// One array per device, alive until the process ends.  In host code its
// name is only a handle for the symbol lookup below; kernels get the device
// address that lookup returns.
static __device__ __align__(256) unsigned char scratch[RMQ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices];  // the array's address on each device, once looked up

// Address of `scratch` on the current device, looked up on the first call
// made with that device current.
rmq_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RMQ_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RMQ_ERR_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RMQ_OK;
}

}  // namespace

extern "C" rmq_status rmq_query_batch_noalloc(const int32_t* A, int64_t n, const int32_t* L,
                                              const int32_t* R, int64_t q, int32_t* out,
                                              void* stream, const rmq_options* opt) {
  rmq_options o{};
  if (opt) o = *opt;
  if (o.workspace || o.workspace_bytes) return RMQ_ERR_INVALID_ARG;  // the scratch is fixed
  if (n < 1 || n > RMQ_MAX_N || q < 0 || q > RMQ_MAX_Q || !A) return RMQ_ERR_INVALID_ARG;
  if (q == 0) return rmq_query_batch_ex(A, n, L, R, q, out, stream, &o);  // checks, no-op
  const size_t need = rmq_workspace_bytes(n, q, &o);
  if (need == 0) return RMQ_ERR_INVALID_ARG;  // options the planner rejects
  if (need > (size_t)RMQ_NOALLOC_SCRATCH_BYTES) return RMQ_ERR_SCRATCH_LIMIT;
  void* ws = nullptr;
  const rmq_status st = scratch_address(&ws);
  if (st != RMQ_OK) return st;
  o.workspace = ws;
  o.workspace_bytes = RMQ_NOALLOC_SCRATCH_BYTES;
  return rmq_query_batch_ex(A, n, L, R, q, out, stream, &o);
}
