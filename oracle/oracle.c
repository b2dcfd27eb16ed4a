/*
 * oracle.c -- CPU oracle for batched range-minimum queries (RMQ).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path never
 * calls it, and it shares no source, header or generated table with the HIP
 * library.
 *
 * Every routine writes out a plain definition from Grabowski & Kowalski,
 * "Faster batched range minimum queries" (arXiv 1706.06940), slowly and in
 * the most obvious way:
 *
 *   oracle_rmq_scan            Section 1, definition of RMQ_A(i, j), with the
 *                              leftmost-minimum variant that Section 1 mentions
 *   oracle_rmq_sparse_table    Section 2, the doubling (Sparse Table)
 *                              observation of Bender and Farach, over blocks
 *                              of b elements; b = 1 is the textbook table
 *   oracle_block_argmin        Section 3.2, minima of the blocks of k elements
 *   oracle_block_sparse_table  Section 3.1 step 3, minima over spans of 2^j
 *                              consecutive blocks
 *   oracle_sort_endpoints      Section 3.1 step 1, the sorted endpoint list E
 *   oracle_remap               Section 3.1 step 1, queries remapped onto A_Q
 *   oracle_contract            Section 3.1 step 2, A_Q and its position map
 *   oracle_contracted_answer   Section 3.1 step 4, minimum over A_Q[Lc..Rc]
 *   oracle_euler_tour          Section 1, the reduction of LCA to RMQ: the
 *                              Euler tour of a rooted tree (depth and node of
 *                              every step, first occurrence of every node)
 *
 * Conventions (the paper is 1-based and leaves ties open): positions are
 * 0-based, query ranges [l, r] are inclusive, and a minimum is the pair
 * (value, position) that is smallest in lexicographic order, i.e. the
 * leftmost position holding the smallest value.  A query is valid when
 * 0 <= l <= r < n; an invalid one gets -1.
 *
 * Parallelism: independent queries / blocks are split over OpenMP threads.
 * That changes no result, since every output is computed on its own.
 */
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

int32_t oracle_num_threads(void) { return (int32_t)omp_get_max_threads(); }

void oracle_set_threads(int32_t t)
{
    if (t > 0)
        omp_set_num_threads(t);
}

static int valid_query(int64_t l, int64_t r, int64_t n) { return 0 <= l && l <= r && r < n; }

/* Leftmost position of the minimum of A[l..r] (l <= r): walk left to right
 * and move only on a strictly smaller value. */
static int64_t scan_argmin(const int32_t *A, int64_t l, int64_t r)
{
    int64_t best = l;
    for (int64_t t = l + 1; t <= r; t++)
        if (A[t] < A[best])
            best = t;
    return best;
}

/* The smaller of two candidate positions: smaller value first, then the
 * smaller position. */
static int64_t better(const int32_t *A, int64_t p, int64_t q)
{
    if (A[p] < A[q])
        return p;
    if (A[q] < A[p])
        return q;
    return p < q ? p : q;
}

static int floor_log2(int64_t x) /* x >= 1 */
{
    int j = 0;
    while ((x >> (j + 1)) != 0)
        j++;
    return j;
}

/* Section 1: out[i] = leftmost argmin of A[L[i]..R[i]], by a linear scan.
 * Returns the number of invalid queries. */
int64_t oracle_rmq_scan(const int32_t *A, int64_t n, const int32_t *L, const int32_t *R,
                        int64_t q, int32_t *out)
{
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int64_t i = 0; i < q; i++) {
        if (!valid_query(L[i], R[i], n)) {
            out[i] = -1;
            bad++;
            continue;
        }
        out[i] = (int32_t)scan_argmin(A, L[i], R[i]);
    }
    return bad;
}

/* Section 2: Sparse Table over the nb = floor(n / b) whole blocks of b
 * elements.  M[j][i] is the minimum over blocks i .. i + 2^j - 1 (only
 * windows that fit are formed): M[0][i] scans block i, and M[j][i] is the
 * smaller of M[j-1][i] and M[j-1][i + 2^(j-1)].  A query takes the whole
 * blocks inside it from two windows of 2^j' blocks, j' = floor(log2(#whole
 * blocks)), which together cover them, and scans its partial blocks (and the
 * tail past the last whole block) element by element.  With b = 1 this is the
 * textbook table.  Returns the number of invalid queries, or -1 if the table
 * could not be allocated. */
int64_t oracle_rmq_sparse_table(const int32_t *A, int64_t n, int64_t b, const int32_t *L,
                                const int32_t *R, int64_t q, int32_t *out)
{
    if (b < 1)
        return -1;
    int64_t nb = n / b;
    int levels = nb >= 1 ? floor_log2(nb) + 1 : 0;
    int32_t *M = NULL;
    if (nb >= 1) {
        M = malloc(sizeof(int32_t) * (size_t)nb * (size_t)levels);
        if (!M)
            return -1;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nb; i++)
            M[i] = (int32_t)scan_argmin(A, i * b, i * b + b - 1);
        for (int j = 1; j < levels; j++) {
            int32_t *prev = M + (size_t)(j - 1) * nb, *cur = M + (size_t)j * nb;
            int64_t half = (int64_t)1 << (j - 1);
            int64_t count = nb - 2 * half + 1; /* windows of 2^j blocks that fit */
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < count; i++)
                cur[i] = (int32_t)better(A, prev[i], prev[i + half]);
        }
    }
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (int64_t i = 0; i < q; i++) {
        int64_t l = L[i], r = R[i];
        if (!valid_query(l, r, n)) {
            out[i] = -1;
            bad++;
            continue;
        }
        int64_t first_blk = (l + b - 1) / b; /* first whole block inside [l, r] */
        int64_t last_blk = (r + 1) / b - 1;  /* last whole block inside [l, r]  */
        if (last_blk >= nb)
            last_blk = nb - 1;
        int64_t best;
        if (first_blk > last_blk) {
            best = scan_argmin(A, l, r);
        } else {
            int64_t cnt = last_blk - first_blk + 1;
            int j = floor_log2(cnt);
            const int32_t *Mj = M + (size_t)j * nb;
            best = better(A, Mj[first_blk], Mj[last_blk - ((int64_t)1 << j) + 1]);
            if (l < first_blk * b)
                best = better(A, scan_argmin(A, l, first_blk * b - 1), best);
            if ((last_blk + 1) * b <= r)
                best = better(A, best, scan_argmin(A, (last_blk + 1) * b, r));
        }
        out[i] = (int32_t)best;
    }
    free(M);
    return bad;
}

/* Section 3.2: pos[j] = argmin of block j = A[j*k .. min((j+1)*k, n) - 1],
 * for j < ceil(n / k); the last block may be short. */
void oracle_block_argmin(const int32_t *A, int64_t n, int64_t k, int32_t *pos)
{
    int64_t nb = (n + k - 1) / k;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nb; j++) {
        int64_t hi = (j + 1) * k < n ? (j + 1) * k : n;
        pos[j] = (int32_t)scan_argmin(A, j * k, hi - 1);
    }
}

/* Section 3.1 step 3 / Section 3.2: st[i*nb + j] = argmin over the blocks
 * j .. min(j + 2^i, nb) - 1, for levels i = 0 .. levels-1, given the block
 * argmins blk[] of A.  A span that would run past the last block is cut at
 * it.  Built by doubling: the span of 2^i blocks is the union of the two
 * spans of 2^(i-1) blocks starting at j and at j + 2^(i-1). */
void oracle_block_sparse_table(const int32_t *A, const int32_t *blk, int64_t nb, int32_t levels,
                               int32_t *st)
{
    for (int64_t j = 0; j < nb; j++)
        st[j] = blk[j];
    for (int32_t i = 1; i < levels; i++) {
        const int32_t *prev = st + (size_t)(i - 1) * nb;
        int32_t *cur = st + (size_t)i * nb;
        int64_t half = (int64_t)1 << (i - 1);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nb; j++)
            cur[j] = j + half < nb ? (int32_t)better(A, prev[j], prev[j + half]) : prev[j];
    }
}

typedef struct {
    int32_t pos;
    int32_t tag;
} endpoint;

static int cmp_endpoint(const void *a, const void *b)
{
    const endpoint *x = a, *y = b;
    if (x->pos != y->pos)
        return x->pos < y->pos ? -1 : 1;
    if (x->tag != y->tag)
        return x->tag < y->tag ? -1 : 1;
    return 0;
}

/* Section 3.1 step 1: the 2q endpoints as (position, tag) pairs, where the
 * left end of query i carries tag 2i and its right end tag 2i+1, sorted by
 * position and then by tag.  Writes the sorted positions and tags.  Returns
 * 0, or -1 if out of memory. */
int oracle_sort_endpoints(const int32_t *L, const int32_t *R, int64_t q, int32_t *pos,
                          int32_t *tag)
{
    endpoint *e = malloc(sizeof(endpoint) * (size_t)(2 * q > 0 ? 2 * q : 1));
    if (!e)
        return -1;
    for (int64_t i = 0; i < q; i++) {
        e[2 * i].pos = L[i];
        e[2 * i].tag = (int32_t)(2 * i);
        e[2 * i + 1].pos = R[i];
        e[2 * i + 1].tag = (int32_t)(2 * i + 1);
    }
    qsort(e, (size_t)(2 * q), sizeof(endpoint), cmp_endpoint);
    for (int64_t s = 0; s < 2 * q; s++) {
        pos[s] = e[s].pos;
        tag[s] = e[s].tag;
    }
    free(e);
    return 0;
}

/* Section 3.1 step 1, remapping: if sorted slot s holds the left end of
 * query i, then Lc[i] = s; if it holds the right end, Rc[i] = s - 1.  Query i
 * then spans the contracted entries Lc[i] .. Rc[i], whose segments
 * [E_s, E_(s+1)] together cover exactly [L[i], R[i]]. */
void oracle_remap(const int32_t *tag, int64_t q, int32_t *Lc, int32_t *Rc)
{
    for (int64_t s = 0; s < 2 * q; s++) {
        int32_t t = tag[s];
        if (t % 2 == 0)
            Lc[t / 2] = (int32_t)s;
        else
            Rc[t / 2] = (int32_t)(s - 1);
    }
}

/* Section 3.1 step 2: for s = 0 .. m-2, aq[s] is the argmin of the closed
 * area A[pos[s] .. pos[s+1]] between consecutive sorted endpoints.  The
 * value A[aq[s]] is the contracted entry A_Q[s] and aq[s] itself is the
 * position map back into A. */
void oracle_contract(const int32_t *A, const int32_t *pos, int64_t m, int32_t *aq)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t s = 0; s < m - 1; s++)
        aq[s] = (int32_t)scan_argmin(A, pos[s], pos[s + 1]);
}

/* Section 3.1 step 4 without blocks: out[i] = the smallest (A[p], p) among
 * p = aq[Lc[i]] .. aq[Rc[i]]. */
void oracle_contracted_answer(const int32_t *A, const int32_t *aq, const int32_t *Lc,
                              const int32_t *Rc, int64_t q, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < q; i++) {
        int64_t best = aq[Lc[i]];
        for (int64_t s = (int64_t)Lc[i] + 1; s <= Rc[i]; s++)
            best = better(A, best, aq[s]);
        out[i] = (int32_t)best;
    }
}

/* Section 1 (LCA reduces to RMQ): the Euler tour of the tree given by
 * parent[] (parent[root] = -1), children visited in increasing id.  The tour
 * lists the node reached by every step of a depth-first walk: the root, then
 * for every edge the child when going down and the parent when coming back
 * up -- 2N - 1 entries.  depth[i] and node[i] describe entry i; first[v] is
 * the index of v's first entry.  Returns 0, or -1 if parent[] is not one
 * tree (no single root, a parent out of range, or nodes the walk from the
 * root never reaches).  Plain and serial: child lists by counting, then an
 * explicit stack of (node, next child index). */
int oracle_euler_tour(const int32_t *parent, int64_t N, int32_t *depth, int32_t *node,
                      int32_t *first)
{
    int64_t root = -1, roots = 0;
    for (int64_t v = 0; v < N; v++) {
        if (parent[v] == -1) {
            root = v;
            roots++;
        } else if (parent[v] < 0 || parent[v] >= N || parent[v] == v) {
            return -1;
        }
    }
    if (roots != 1)
        return -1;
    /* children of p, in increasing id: kids[start[p] .. start[p+1]) */
    int64_t *start = calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *fill = calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *kids = malloc(sizeof(int32_t) * (size_t)(N > 1 ? N - 1 : 1));
    int64_t *stack_node = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *stack_next = malloc(sizeof(int64_t) * (size_t)N);
    int ok = start && fill && kids && stack_node && stack_next;
    if (ok) {
        for (int64_t v = 0; v < N; v++)
            if (v != root)
                start[parent[v] + 1]++;
        for (int64_t p = 0; p < N; p++)
            start[p + 1] += start[p];
        for (int64_t v = 0; v < N; v++)  /* increasing v: each list in id order */
            if (v != root) {
                int64_t p = parent[v];
                kids[start[p] + fill[p]++] = (int32_t)v;
            }
        for (int64_t v = 0; v < N; v++)
            first[v] = -1;
        int64_t len = 0, top = 0;
        stack_node[0] = root;
        stack_next[0] = start[root];
        depth[len] = 0;
        node[len] = (int32_t)root;
        first[root] = 0;
        len++;
        while (top >= 0) {
            int64_t v = stack_node[top];
            if (stack_next[top] < start[v + 1]) {
                int64_t c = kids[stack_next[top]++];  /* go down to the next child */
                if (top + 1 >= N || len >= 2 * N - 1) {
                    ok = 0;
                    break;
                }
                top++;
                stack_node[top] = c;
                stack_next[top] = start[c];
                depth[len] = (int32_t)top;
                node[len] = (int32_t)c;
                first[c] = (int32_t)len;
                len++;
            } else {
                top--;  /* done with v: come back up to its parent */
                if (top >= 0) {
                    depth[len] = (int32_t)top;
                    node[len] = (int32_t)stack_node[top];
                    len++;
                }
            }
        }
        if (len != 2 * N - 1)
            ok = 0;  /* some node is not below the root: a cycle */
    }
    free(start);
    free(fill);
    free(kids);
    free(stack_node);
    free(stack_next);
    return ok ? 0 : -1;
}
