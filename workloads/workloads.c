/*
 * Native helpers for the synthetic input generators: serial steps that numpy
 * cannot vectorise.  Input construction only; nothing here computes a range
 * minimum.
 */
#include <stdint.h>

/* Apply count swaps a[i[t]] <-> a[j[t]] in order (the paper's permutation
 * workload: the increasing sequence after n/2 random pair swaps). */
void wl_swap_permutation(int32_t *a, int64_t n, const int64_t *i, const int64_t *j,
                         int64_t count)
{
    (void)n;
    for (int64_t t = 0; t < count; t++) {
        int32_t x = a[i[t]];
        a[i[t]] = a[j[t]];
        a[j[t]] = x;
    }
}
