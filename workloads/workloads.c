/*
 * Native helpers for the synthetic input generators: serial steps that numpy
 * cannot vectorise.  Input construction only; nothing here computes a range
 * minimum.
 */
#include <stdint.h>
#include <stdlib.h>

/*
 * Euler tour of a rooted tree given by parent[] (parent[0] = -1, and
 * parent[i] < i for i >= 1, as in a random recursive tree).  Children are
 * visited in increasing id.  Writes, for each of the 2N-1 tour steps, the
 * depth of the visited node and the node itself, and for each node the step
 * of its first visit.  Returns 0, or a negative code on bad input / no memory.
 */
int wl_euler_tour(const int32_t *parent, int64_t N, int32_t *depth, int32_t *node,
                  int32_t *first)
{
    if (N < 1 || parent[0] != -1)
        return -1;
    /* children in CSR form; parent[i] < i keeps each child list sorted */
    int64_t *start = calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *child = malloc(sizeof(int32_t) * (size_t)(N > 1 ? N - 1 : 1));
    int64_t *fill = NULL;
    int32_t *stack_node = NULL;
    int64_t *stack_next = NULL;
    int rc = 0;
    if (!start || !child) {
        rc = -2;
        goto done;
    }
    for (int64_t i = 1; i < N; i++) {
        int32_t p = parent[i];
        if (p < 0 || p >= i) {
            rc = -1;
            goto done;
        }
        start[p + 1]++;
    }
    for (int64_t v = 0; v < N; v++)
        start[v + 1] += start[v];
    fill = malloc(sizeof(int64_t) * (size_t)N);
    if (!fill) {
        rc = -2;
        goto done;
    }
    for (int64_t v = 0; v < N; v++)
        fill[v] = start[v];
    for (int64_t i = 1; i < N; i++)
        child[fill[parent[i]]++] = (int32_t)i;

    /* iterative DFS; the stack holds (node, index of its next child) */
    int64_t cap = 1024;
    stack_node = malloc(sizeof(int32_t) * (size_t)cap);
    stack_next = malloc(sizeof(int64_t) * (size_t)cap);
    if (!stack_node || !stack_next) {
        rc = -2;
        goto done;
    }
    int64_t sp = 0, t = 0;
    stack_node[0] = 0;
    stack_next[0] = start[0];
    depth[t] = 0;
    node[t] = 0;
    first[0] = 0;
    t++;
    while (sp >= 0) {
        int32_t v = stack_node[sp];
        if (stack_next[sp] < start[v + 1]) {
            int32_t c = child[stack_next[sp]++];
            if (sp + 1 == cap) {
                cap *= 2;
                int32_t *sn = realloc(stack_node, sizeof(int32_t) * (size_t)cap);
                if (!sn) {
                    rc = -2;
                    goto done;
                }
                stack_node = sn;
                int64_t *sx = realloc(stack_next, sizeof(int64_t) * (size_t)cap);
                if (!sx) {
                    rc = -2;
                    goto done;
                }
                stack_next = sx;
            }
            sp++;
            stack_node[sp] = c;
            stack_next[sp] = start[c];
            first[c] = (int32_t)t;
            depth[t] = (int32_t)sp;
            node[t] = c;
            t++;
        } else {
            sp--;
            if (sp >= 0) {
                depth[t] = (int32_t)sp;
                node[t] = stack_node[sp];
                t++;
            }
        }
    }
    if (t != 2 * N - 1)
        rc = -3;
done:
    free(start);
    free(child);
    free(fill);
    free(stack_node);
    free(stack_next);
    return rc;
}

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
