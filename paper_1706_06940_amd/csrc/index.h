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
  int lg;            // table arity l = 2^lg (1: doubling, Section 3.1)
  uint64_t* st;      // level-major levels x nb keys (device)
  uint64_t* sub;     // two block levels (Section 3.3): k1-block minima, else null
  int k1shift;       // k1 = 2^k1shift when sub is set
  int64_t nb1;       // number of k1-blocks
  uint64_t* rec;     // query records of the doubling table, or null
  size_t bytes;      // table + k1-block minima + query records
};
