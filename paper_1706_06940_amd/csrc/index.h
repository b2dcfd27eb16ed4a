// A resident index (internal layout shared by the C ABI and the server).
#pragma once

#include <stddef.h>
#include <stdint.h>

struct rmq_index_s {
  int device;
  const int32_t* A;  // caller's array, read by partial-block scans
  int64_t n;
  int kshift;        // block size k = 2^kshift
  int64_t nb;        // number of blocks
  int levels;        // Sparse Table levels
  uint64_t* st;      // level-major levels x nb keys (device)
  size_t bytes;
};
