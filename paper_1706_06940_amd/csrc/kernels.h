// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rmq {

// ---- non-contracted path (Section 3.2) ----
hipError_t launch_blockmin_i32(const int32_t* A, int64_t n, int kshift, uint64_t* keys,
                               hipStream_t stream);
hipError_t launch_blockmin_keys(const uint64_t* S, int64_t m, int kshift, uint64_t* keys,
                                hipStream_t stream);
hipError_t launch_sparse_table(uint64_t* st, int64_t nb, int levels, hipStream_t stream);
hipError_t launch_query_full(const int32_t* A, int64_t n, int kshift, const uint64_t* st,
                             int64_t nb, const int32_t* L, const int32_t* R, int64_t q,
                             int32_t* out, int64_t* bad_count, uint64_t* stats,
                             hipStream_t stream);

// ---- contracted path (Section 3.1) ----
// Device LSD radix sort of the 2q endpoints by (position, tag).
size_t sort_workspace_bytes(int64_t q);
hipError_t launch_sort_endpoints(const int32_t* L, const int32_t* R, int64_t q, int64_t n,
                                 int32_t* pos, int32_t* tag, void* ws, size_t ws_bytes,
                                 hipStream_t stream);
// Remap + contraction: Lc/Rc, A_Q over closed areas between endpoints.
// tile_start: scratch of contract_tile_start_bytes(n).
size_t contract_tile_start_bytes(int64_t n);
hipError_t launch_contract(const int32_t* A, int64_t n, const int32_t* pos, const int32_t* tag,
                           int64_t q, int32_t* Lc, int32_t* Rc, uint64_t* aq, int32_t* tile_start,
                           hipStream_t stream);
hipError_t launch_query_contracted(const uint64_t* aq, int64_t m, int64_t n, int kshift,
                                   const uint64_t* st, int64_t nb, const int32_t* L,
                                   const int32_t* R, const int32_t* Lc, const int32_t* Rc,
                                   int64_t q, int32_t* out, int64_t* bad_count, uint64_t* stats,
                                   hipStream_t stream);

}  // namespace rmq
