/*
 * rmq.h -- C ABI of an MI355X (gfx950) library for batched, offline range
 * minimum queries, after Grabowski & Kowalski, "Faster batched range minimum
 * queries" (arXiv 1706.06940).
 *
 * Problem (Section 1, definition of RMQ; Section 1, offline setting): given
 * an int32 array A[0..n-1] and a batch of q queries [L[i], R[i]] known
 * beforehand, return for each query the position of the minimum of
 * A[L[i]..R[i]].  This library fixes the tie-break the paper leaves open:
 * the LEFTMOST position holding the minimum value.  Positions are 0-based and
 * ranges inclusive (the paper is 1-based).
 *
 * Two methods compute the same answers:
 *   RMQ_PATH_FULL        Section 3.2 (BbST, no contraction): block minima over
 *                        all of A, a Sparse Table over the blocks, and each
 *                        query from two overlapping power-of-two block spans
 *                        plus speculative reads of its two end blocks.
 *   RMQ_PATH_CONTRACTED  Section 3.1 (BbST_CON): sort the 2q endpoints,
 *                        contract A into A_Q (2q-1 minima of the closed areas
 *                        between consecutive endpoints), then the same block
 *                        Sparse Table and query step on A_Q.
 *
 * Memory: every array argument named A, L, R, out, keys, pos, tag, st, aq,
 * bad_count, stats or workspace is a DEVICE pointer (hipMalloc / torch CUDA
 * tensor memory) owned by the caller.  The library never copies A or the
 * queries (extra space is counted apart from A and Q, as in Section 4).  It
 * owns rmq_index objects and, when no workspace is passed, the per-call
 * scratch, which it takes from the device's stream-ordered pool
 * (hipMallocAsync) and returns on the same stream.  That scratch is as large
 * as the largest any earlier call on the device needed (so calls of mixed
 * sizes reuse one pool block), and the pool keeps freed memory cached; a
 * caller that must bound device memory passes its own workspace.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Every call only enqueues work on it and returns; results are
 * valid once the stream has been synchronised.  Calls on one stream run in
 * order.  An rmq_index is immutable after rmq_build and may be queried from
 * several streams at once.
 *
 * Errors: host-checkable problems return a status synchronously and enqueue
 * nothing.  A query with L > R, L < 0 or R >= n is not a host error: it gets
 * out[i] = -1 and, when opt->bad_count is given, adds one to *bad_count on
 * the device; other queries are unaffected.  q = 0 is a no-op returning
 * RMQ_OK.  No C++ exception crosses this interface.
 *
 * Sort failure: the device radix sort of the CONTRACTED method (and of the
 * LCA build) waits for earlier tiles with a bounded wait.  Should a wait run
 * out (a predecessor stalled for millions of polls), the sort gives up on
 * its order and says so in a device word; nothing reads memory out of
 * bounds and every kernel ends.  The call then reports the failure instead
 * of wrong answers: the CONTRACTED method answers -1 for EVERY query of the
 * batch and adds q to *bad_count; rmq_sort_endpoints writes -1 to every pos
 * and tag; rmq_contract writes -1 to every LR entry; rmq_lca_build returns
 * RMQ_ERR_DEVICE.  (rmq_test_sort_abort forces this path for tests.)
 *
 * Value encoding used by the key-valued outputs (block minima, Sparse Table
 * entries, A_Q): key(p) = ((uint32(A[p]) XOR 0x80000000) << 32) | p, a
 * uint64.  Comparing keys as unsigned integers compares (A[p], p)
 * lexicographically, so the smallest key is the leftmost minimum and every
 * min over keys is exact and order-independent.
 */
#ifndef RMQ_H
#define RMQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rmq_status {
    RMQ_OK = 0,
    RMQ_ERR_INVALID_ARG = 1,      /* bad pointer, size, block size or option */
    RMQ_ERR_OUT_OF_MEMORY = 2,    /* device allocation failed                */
    RMQ_ERR_DEVICE = 3,           /* a HIP runtime call failed               */
    RMQ_ERR_WORKSPACE_SMALL = 4,  /* caller workspace below the needed size  */
    RMQ_ERR_MISALIGNED = 5,       /* a device pointer is not 4/8-byte aligned */
    RMQ_ERR_SCRATCH_LIMIT = 6     /* the call needs more scratch than the fixed
                                     array of rmq_query_batch_noalloc holds   */
} rmq_status;

typedef enum rmq_path {
    RMQ_PATH_AUTO = 0,        /* planner picks FULL or CONTRACTED            */
    RMQ_PATH_FULL = 1,        /* Section 3.2                                 */
    RMQ_PATH_CONTRACTED = 2,  /* Section 3.1                                 */
    RMQ_PATH_ST_CON = 3       /* Section 2: the comparison system
                                 ST-RMQ_CON (Alzamel et al.'s contraction and
                                 a Sparse Table over every entry), for
                                 measuring the paper's method against it.
                                 Its A_Q keeps each endpoint's element and
                                 the region between neighbouring endpoints
                                 (4q - 1 entries, from the sorted endpoints
                                 instead of marks in A's top bits), the
                                 table has floor(log2(4q - 1)) + 1 levels of
                                 4q - 1 keys (the full table, not the cited
                                 work's level-by-level reuse of one array),
                                 and a query reads two entries.  Only
                                 rmq_query_batch_ex / _noalloc and
                                 rmq_workspace_bytes take it, with
                                 block_size, sub_block_size and
                                 table_arity_log2 0 and q <= 2^29; the
                                 planner never picks it.                 */
} rmq_path;

/* Block sizes k are powers of two in [RMQ_MIN_BLOCK, RMQ_MAX_BLOCK]. */
#define RMQ_MIN_BLOCK 16
#define RMQ_MAX_BLOCK (1 << 24)
/* Largest n (positions must fit in the int32 outputs) and largest q. */
#define RMQ_MAX_N 2147483647LL
#define RMQ_MAX_Q (1LL << 30)

/* Number of per-stage timings an rmq_timer can hold.  The stages mirror the
 * four steps of Section 3.1 (Table 1 reports their cumulative shares):
 *   0 sort + remap (CONTRACTED only), 1 contraction or block minima,
 *   2 block Sparse Table, 3 queries. */
#define RMQ_NUM_STAGES 4

typedef struct rmq_timer_s rmq_timer;
typedef struct rmq_index_s *rmq_index;

typedef struct rmq_options {
    int32_t block_size;      /* k; 0 = chosen by the planner                    */
    int32_t path;            /* rmq_path                                         */
    int64_t *bad_count;      /* device int64, optional: += invalid queries       */
    uint64_t *stats;         /* device uint64[2], optional: += scans performed,
                                += entries read by partial-block scans (elements,
                                and k1-block minima with two block levels)       */
    void *workspace;         /* device scratch, optional (see rmq_workspace_bytes) */
    size_t workspace_bytes;
    rmq_timer *timer;        /* optional: records per-stage events on the stream */
    int32_t sub_block_size;  /* Section 3.3, two block levels: k1, the size of the
                                small blocks whose minima are also kept (0 = one
                                level).  A power of two, 16 <= k1 < k.  With path
                                AUTO or FULL the plain method's blocks over A, with
                                path CONTRACTED the blocks over A_Q; partial blocks
                                of size k are then read as k1-block minima plus
                                at most two partial k1-blocks.  With block_size 0,
                                k is the power of two nearest
                                sqrt(m) * log2(m)^(2/3) (at least 2 * k1), m = n
                                for the plain method and 2q for A_Q. */
    int32_t table_arity_log2; /* Section 3.1, the table over powers of l instead
                                 of 2: l = 2^table_arity_log2.  0 or 1: the
                                 doubling table (l = 2).  2..5 (l = 4..32):
                                 level i holds the minima of l^i consecutive
                                 blocks, there are floor(log2(nb - 2) /
                                 log2(l)) + 1 levels for nb > 3 blocks (1
                                 otherwise), and a query reads at most l of
                                 them.  Level i >= 1 is stored by residue
                                 class mod s = l^i: block b's entry is at
                                 r * floor(nb / s) + min(r, nb mod s) + b / s
                                 with r = b mod s, so the windows one query
                                 reads at a level are adjacent.  Both methods,
                                 the resident index and the LCA front-end;
                                 the batched and served calls keep the
                                 doubling table. */
    int32_t no_query_records; /* nonzero: do not build query records.  By
                                 default a doubling table of nb blocks and L
                                 levels with one block level (no
                                 sub_block_size) also gets, when
                                 32 * nb * L bytes <= 8 MiB, two records per
                                 block: for every
                                 level t, the block's minimum paired with the
                                 window of 2^t blocks starting just after it,
                                 and paired with the window ending just
                                 before it (16-byte pairs).  A query then
                                 reads each end block's key and the window
                                 beside it with one 16-byte load instead of
                                 two 8-byte ones.  Same answers either way. */
    int32_t sub_block_size2; /* Section 3.3 with three block levels: k2, the
                                size of still smaller blocks whose minima are
                                kept under the k1-blocks (0 = none).  A power
                                of two, 16 <= k2 < k1; needs sub_block_size and
                                the plain method (path AUTO or FULL) in a
                                single call (not the contracted method, the
                                resident index, batches or the server).  A
                                partial k1-block is then read as k2-block
                                minima plus at most two partial k2-blocks.
                                Same answers. */
} rmq_options;

/* A human-readable name for a status code (static storage). */
const char *rmq_status_string(rmq_status s);

/* Library version string (static storage).  "rmq-gfx950 1.1": rmq_options
 * ends with sub_block_size2 and rmq_path has RMQ_PATH_ST_CON; a caller built
 * against 1.0's shorter rmq_options must be rebuilt. */
const char *rmq_version(void);

/* ----------------------------------------------------------------------------
 * One offline batch (Section 1, offline setting): build whatever the chosen
 * method needs from A and answer all q queries.  out[i] receives the leftmost
 * argmin of A[L[i]..R[i]] (int32), or -1 for an invalid query.
 *   A    int32[n], 1 <= n <= RMQ_MAX_N
 *   L, R int32[q], 0 <= q <= RMQ_MAX_Q
 *   out  int32[q]; may not alias A, L or R
 * rmq_query_batch uses the planner with default options. */
rmq_status rmq_query_batch(const int32_t *A, int64_t n, const int32_t *L, const int32_t *R,
                           int64_t q, int32_t *out, void *stream);

/* As rmq_query_batch, with options (opt may be NULL). */
rmq_status rmq_query_batch_ex(const int32_t *A, int64_t n, const int32_t *L, const int32_t *R,
                              int64_t q, int32_t *out, void *stream, const rmq_options *opt);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops that may not call the allocator): rmq_query_batch_ex
 * with its scratch taken from a fixed device array of the library,
 * RMQ_NOALLOC_SCRATCH_BYTES large, instead of the stream-ordered pool.  Each
 * device holds its own array from the first call made with it current until
 * the process ends; that first call looks up the array's address, later
 * calls allocate nothing at all (no hipMalloc, hipMallocAsync or hipFree).
 * opt->workspace must be NULL (and workspace_bytes 0); every other option is
 * as for rmq_query_batch_ex.  A call whose rmq_workspace_bytes(n, q, opt)
 * exceeds RMQ_NOALLOC_SCRATCH_BYTES returns RMQ_ERR_SCRATCH_LIMIT and enqueues
 * nothing (the plain method fits at every n; the contracted one up to about
 * q = 2e6).  All calls on one device share the one array and every call
 * rewrites what it reads of it, so calls on ONE stream are safe in any order,
 * while calls that overlap on one device (other streams, other host threads
 * without ordering) race on the array and may return wrong answers. */
#define RMQ_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
rmq_status rmq_query_batch_noalloc(const int32_t *A, int64_t n, const int32_t *L,
                                   const int32_t *R, int64_t q, int32_t *out, void *stream,
                                   const rmq_options *opt);

/* Device scratch bytes rmq_query_batch_ex needs for (n, q, opt->block_size,
 * opt->path) after planning; 0 on invalid arguments.  A caller-provided
 * workspace must be at least this large and 256-byte aligned. */
size_t rmq_workspace_bytes(int64_t n, int64_t q, const rmq_options *opt);

/* The planner's choice of block size and path for (n, q) -- the automated
 * selection of k that Section 5 leaves as future work -- among one-level
 * plans (what batches use).  Either output pointer may be NULL. */
rmq_status rmq_plan(int64_t n, int64_t q, int32_t *block_size, int32_t *path);

/* The plan a call with path AUTO and no block sizes takes: as rmq_plan, but
 * the measured table may also choose two block levels (Section 3.3), given
 * as *sub_block_size > 0 (0: one level).  Any output pointer may be NULL. */
rmq_status rmq_plan_ex(int64_t n, int64_t q, int32_t *block_size, int32_t *path,
                       int32_t *sub_block_size);

/* Measured plans for the planner: for a call with path AUTO, rmq_plan picks
 * the entry nearest to (n, q) in (log2 n, log2 q) and uses its block size and
 * method; with no table (count 0 clears it) it falls back to the built-in
 * rule.  The table is copied; process-wide. */
typedef struct rmq_plan_entry {
    int64_t n, q;
    int32_t block_size;
    int32_t path;                 /* RMQ_PATH_FULL or RMQ_PATH_CONTRACTED          */
    int32_t sub_block_size;       /* > 0: two block levels (FULL only), k1 < k     */
    int32_t one_level_block_size; /* with two levels: the best one-level k, used
                                     where two levels are not offered (batches);
                                     0 = block_size                              */
} rmq_plan_entry;
rmq_status rmq_planner_set_table(const rmq_plan_entry *entries, int32_t count);

/* Block size a call with block_size 0 uses for the given path (FULL or
 * CONTRACTED): about sqrt(n)/8 for FULL (Section 3.2 takes k = Theta(sqrt(n))
 * for the average case); for CONTRACTED about sqrt(2q)/2 (Section 3.1's
 * O(1 + k^2/q) average query cost).  0 on invalid arguments. */
int32_t rmq_default_block(int64_t n, int64_t q, int32_t path);

/* Sub-block size (Section 3.3) a call with block_size 0 and sub_block_size 0
 * uses for the given path: 0 (one block level) for FULL, whose path AUTO
 * takes two levels from the planner's table instead (rmq_plan_ex); for
 * CONTRACTED 0 below 2^22 queries and 256 from there (then rmq_default_block
 * gives the smallest block from 16384 whose table over A_Q fits 144 KiB, so
 * that the query kernel keeps it in LDS).  Two levels over A_Q gain for
 * uniform queries and can lose on mixes of short ranges (q = 1e7; n = 1e8:
 * 0.84 -> 0.76 ms uniform, 1.61 -> 1.73 ms with half short ranges; n = 1e9
 * with half short ranges: 2.48 -> 1.89 ms); such callers can pass the block
 * sizes.  0 on invalid arguments. */
int32_t rmq_default_sub_block(int64_t n, int64_t q, int32_t path);

/* ----------------------------------------------------------------------------
 * Resident index (Section 3.2): block minima and the block Sparse Table of A
 * with block size k, kept in device memory for any number of later query
 * batches.  A must stay alive and unmodified while the index is used, since
 * partial-block scans read it.  opt->block_size 0 picks k ~ sqrt(n)
 * (Section 3.2 sets k = Theta(sqrt(n))); opt->path is ignored.  With
 * opt->sub_block_size > 0 the index has two block levels (Section 3.3): the
 * k1-block minima are kept beside the table and partial blocks are read
 * through them.  opt->table_arity_log2 > 1 builds the table over powers of
 * l instead of 2 (Section 3.1).  *idx is set only on success.  The build is enqueued on
 * `stream`. */
rmq_status rmq_build(const int32_t *A, int64_t n, const rmq_options *opt, void *stream,
                     rmq_index *idx);

/* Answer a batch on a resident index (Section 3.1 step 4 on A's blocks). */
rmq_status rmq_query_index(rmq_index idx, const int32_t *L, const int32_t *R, int64_t q,
                           int32_t *out, void *stream);

/* As rmq_query_index with options; only bad_count and stats are used. */
rmq_status rmq_query_index_ex(rmq_index idx, const int32_t *L, const int32_t *R, int64_t q,
                              int32_t *out, void *stream, const rmq_options *opt);

/* Device bytes rmq_build(A, n, opt, ...) allocates for the index (the
 * table, the k1-block minima with two block levels, the query records when
 * built; the same figure rmq_index_info reports afterwards), for admission
 * by footprint before building.  0 on invalid arguments. */
size_t rmq_build_bytes(int64_t n, const rmq_options *opt);

/* Free an index.  The caller must make sure no enqueued work still uses it. */
rmq_status rmq_index_free(rmq_index idx);

/* Facts about an index (any output pointer may be NULL).  bytes counts the
 * device memory the index holds: the table, for a two-level index the
 * k1-block minima (8 * ceil(n / k1)), and its query records if it has them
 * (rmq_options.no_query_records). */
rmq_status rmq_index_info(rmq_index idx, int64_t *n, int32_t *block_size, int64_t *num_blocks,
                          int32_t *levels, size_t *bytes);

/* Copy of the index's Sparse Table (level-major, levels x num_blocks uint64
 * keys; level 0 = block minima; level i spans 2^i blocks, or l^i for a table
 * over powers of l, whose levels i >= 1 are in residue-class order -- see
 * rmq_options.table_arity_log2) into device memory `st`, on `stream`. */
rmq_status rmq_index_copy_table(rmq_index idx, uint64_t *st, void *stream);

/* Device bytes of a resident index for (n, k): 8 * nb * levels with
 * nb = ceil(n / k) and levels = floor(log2(max(nb - 2, 1))) + 1 -- the spans
 * of 2^j blocks that a query strictly inside A can use (Table 2 reports this
 * footprint as a share of the 4n bytes of A).  0 on invalid arguments. */
size_t rmq_index_bytes(int64_t n, int32_t block_size);

/* Number of Sparse Table levels for nb blocks (see rmq_index_bytes). */
int32_t rmq_table_levels(int64_t num_blocks);

/* Bytes of the query records built beside a one-level doubling table of nb
 * blocks (see rmq_options.no_query_records); 0 when none are built. */
size_t rmq_query_record_bytes(int64_t num_blocks);

/* Levels of the table over powers of l = 2^table_arity_log2 (Section 3.1;
 * see rmq_options.table_arity_log2) for nb blocks; 0 on invalid arguments.
 * table_arity_log2 0 or 1 gives rmq_table_levels. */
int32_t rmq_table_levels_ary(int64_t num_blocks, int32_t table_arity_log2);

/* ----------------------------------------------------------------------------
 * Lowest common ancestors through RMQ (Section 1: in the Euler tour of a
 * rooted tree, the LCA of u and v is the node of minimum depth between the
 * first occurrences of u and v).  Built entirely on the device: the children
 * of each node ordered by id (stable radix sort of (parent, child)), the
 * tour's arcs linked and ranked (list ranking by sampled sublists and
 * pointer jumping over the samples), the depth array D, the tour's node
 * array and each node's first position, and a resident RMQ index over D.
 * ------------------------------------------------------------------------- */
typedef struct rmq_lca_s *rmq_lca;

/* parent: device int32[num_nodes]; parent[root] = -1 for exactly one root,
 * every other entry in [0, num_nodes) and the parent links acyclic.
 * 1 <= num_nodes <= 2^30.  The tour visits children in increasing id; it
 * has 2 * num_nodes - 1 entries.  opt->block_size, sub_block_size and
 * table_arity_log2 choose the RMQ index over D as for rmq_build (NULL:
 * defaults).  The call waits
 * for the device (it checks the input and the tour) and returns
 * RMQ_ERR_INVALID_ARG for a forest, a parent out of range or a cycle, and
 * RMQ_ERR_DEVICE if the sort of the children gave up (see "Sort failure").
 * Temporary device memory: about 75 bytes per node, freed before return. */
rmq_status rmq_lca_build(const int32_t *parent, int64_t num_nodes, const rmq_options *opt,
                         void *stream, rmq_lca *out);

/* out[i] = LCA(u[i], v[i]) (int32); -1, and opt->bad_count += 1, for a node
 * id outside [0, num_nodes).  u, v, out: device int32[q]; opt may be NULL. */
rmq_status rmq_lca_query(rmq_lca h, const int32_t *u, const int32_t *v, int64_t q, int32_t *out,
                         void *stream, const rmq_options *opt);

/* Copies of the tour into caller device buffers (any may be NULL):
 * depth int32[2N-1], node int32[2N-1], first int32[N]; on `stream`. */
rmq_status rmq_lca_copy_tour(rmq_lca h, int32_t *depth, int32_t *node, int32_t *first,
                             void *stream);

/* num_nodes and the device bytes held (tour arrays and the RMQ index). */
rmq_status rmq_lca_info(rmq_lca h, int64_t *num_nodes, size_t *bytes);

/* Free the structure; no enqueued work may still use it. */
rmq_status rmq_lca_free(rmq_lca h);

/* ----------------------------------------------------------------------------
 * The steps of the two methods, one call each, for callers that want a
 * single stage (and for checking each stage on its own).  All enqueue on
 * `stream` and return at once.
 *
 * Section 3.2 / Section 3.1 step 3, first half: keys[j] = min key over block
 * j = A[j*k .. min((j+1)*k, n) - 1], j < ceil(n/k).  keys: uint64[ceil(n/k)]. */
rmq_status rmq_block_minima(const int32_t *A, int64_t n, int32_t block_size, uint64_t *keys,
                            void *stream);

/* Same over a key array (the contracted array A_Q of the CONTRACTED path):
 * keys[j] = min of src[j*k .. min((j+1)*k, m) - 1]. */
rmq_status rmq_block_minima_keys(const uint64_t *src, int64_t m, int32_t block_size,
                                 uint64_t *keys, void *stream);

/* Section 3.1 step 3 (Section 2's doubling on blocks): given level 0 in
 * st[0 .. nb-1], fill levels 1 .. levels-1 of the level-major table
 * st[levels][nb], where st[j][b] = min(st[0][b .. min(b + 2^j, nb) - 1]). */
rmq_status rmq_sparse_table_build(uint64_t *st, int64_t num_blocks, int32_t levels,
                                  void *stream);

/* Section 3.1 step 1: the 2q endpoints (L[i], tag 2i) and (R[i], tag 2i+1)
 * sorted by (position, tag) with a device LSD radix sort.  pos, tag:
 * int32[2q].  Endpoint positions must lie in [0, n); an invalid query's
 * endpoints are sorted as position 0.  Needs rmq_sort_workspace_bytes(q).
 * If the sort gives up (see "Sort failure" above), every pos and tag is -1. */
rmq_status rmq_sort_endpoints(const int32_t *L, const int32_t *R, int64_t q, int64_t n,
                              int32_t *pos, int32_t *tag, void *workspace,
                              size_t workspace_bytes, void *stream);
size_t rmq_sort_workspace_bytes(int64_t q);

/* Section 3.1 steps 1-2 after the sort: remap each query onto contracted
 * indices -- LR[2i] = Lc[i], the slot of its left end, and LR[2i+1] = Rc[i],
 * the slot of its right end minus one -- and build A_Q: aq[s] = min key over
 * the CLOSED area A[pos[s] .. pos[s+1]], s = 0 .. 2q-2.  pos, tag: the
 * output of rmq_sort_endpoints.  LR: int32[2q] (8-byte aligned);
 * aq: uint64[2q-1].  Takes its scratch from the stream-ordered pool.  The
 * remap buckets the tags with one more sort sweep; if that sweep gives up
 * (see "Sort failure" above), every LR entry is -1. */
rmq_status rmq_contract(const int32_t *A, int64_t n, const int32_t *pos, const int32_t *tag,
                        int64_t q, int32_t *LR, uint64_t *aq, void *stream);

/* ----------------------------------------------------------------------------
 * Batches of arrays.  Many independent arrays, each with its own batch of
 * queries, answered together: the planner picks each array's block size,
 * method and block levels (the automated choice of k left open in Section
 * 5; two block levels, Section 3.3, where its measured table chooses
 * them), and the arrays that take the plain method (Section 3.2) run as ONE
 * launch per phase for all of them -- block minima, the k-block minima from
 * the k1-block minima (arrays with two levels), each round of Sparse Table
 * levels, queries -- instead of a few launches per array.  For those
 * launches an item that fixes neither block size nor method gets blocks of
 * at least n / 1024 elements (one Sparse Table round then builds every
 * table), and 1024-element sub-blocks under blocks of more than 4096.  A
 * batch owns its device scratch and a device table describing the arrays;
 * inputs and outputs stay the caller's.
 * Pointers in the items must stay valid, and the arrays unmodified, for the
 * batch's life: runs reuse them. */
typedef struct rmq_batch_item {
    const int32_t *A;        /* device int32[n]                             */
    int64_t n;
    const int32_t *L, *R;    /* device int32[q]                             */
    int64_t q;
    int32_t *out;            /* device int32[q]                             */
    int32_t block_size;      /* 0 = planner                                 */
    int32_t path;            /* rmq_path; AUTO = planner                    */
} rmq_batch_item;

typedef struct rmq_batch_s *rmq_batch;

#define RMQ_BATCH_FUSED 0     /* one launch per phase over all plain-path arrays */
#define RMQ_BATCH_PER_ITEM 1  /* the single-array sequence for each array        */

/* Plan every item and allocate the batch's scratch (synchronous). */
rmq_status rmq_batch_create(const rmq_batch_item *items, int32_t count, rmq_batch *out);

/* Enqueue one run of the whole batch on `stream`.  use_graph != 0 records the
 * run's launches into a hipGraph on first use (per mode) and replays it
 * afterwards; it needs a non-null stream. */
rmq_status rmq_batch_run(rmq_batch b, int32_t mode, int32_t use_graph, void *stream);

/* The block size and method the planner gave item i. */
rmq_status rmq_batch_item_plan(rmq_batch b, int32_t i, int32_t *block_size, int32_t *path);

/* As rmq_batch_item_plan, and the sub-block size k1 when the planner gave
 * the item two block levels (Section 3.3; 0: one level).  Any output
 * pointer may be NULL. */
rmq_status rmq_batch_item_plan_ex(rmq_batch b, int32_t i, int32_t *block_size, int32_t *path,
                                  int32_t *sub_block_size);

/* Device scratch the batch holds for its items. */
size_t rmq_batch_workspace_bytes(rmq_batch b);

/* Free a batch; no enqueued run may still be using it. */
rmq_status rmq_batch_free(rmq_batch b);

/* ----------------------------------------------------------------------------
 * Serving.  A server keeps arrays and their block Sparse Tables resident
 * (Section 3.2's index, built once per array) and answers query requests as
 * they arrive.  Requests wait in a queue; a dispatcher thread packs whatever
 * is pending into the next free slot -- a stream with its own pinned staging
 * buffer (and device query buffers with RMQ_SERVER_COPY_QUERIES) -- while
 * their queries fit the slot (admission by footprint: the slots' buffers are
 * carved from budget_bytes), and answers the whole coalesced batch with one
 * query launch over the resident tables, which reads the queries from the
 * staging buffer and writes the answers there (or, copying, from and to the
 * device buffers); requests that arrive meanwhile go to the next slot, so
 * batches overlap on the device.  A completion thread copies each request's
 * answers to its output buffer.  All threads are native; the calls below are
 * thread-safe. */
#define RMQ_SERVER_COPY_QUERIES 1  /* flags: queries and answers through device
                                      buffers (one H2D and one D2H copy per
                                      batch) instead of being read and written
                                      in the pinned staging buffers by the
                                      query kernel itself (the default)       */
typedef struct rmq_server_config {
    int32_t num_streams;             /* slots in flight, 1..16                    */
    int32_t max_tables;              /* resident arrays the server can hold       */
    int32_t max_requests_per_batch;  /* requests coalesced into one launch        */
    int32_t flags;                   /* 0 or RMQ_SERVER_COPY_QUERIES              */
    size_t budget_bytes;             /* bytes of in-flight query buffers, split
                                        over the slots (12 B a query + segment
                                        tables): pinned host memory, plus as
                                        much device memory with the copy flag */
    size_t hbm_budget_bytes;         /* device memory (HBM) the server may hold:
                                        the resident tables, the table
                                        descriptors and, with the copy flag,
                                        the slots' device buffers; 0 = no
                                        limit.  rmq_server_add_array refuses a
                                        table that would exceed it */
    int32_t sub_block_size;          /* 0: one block level; else k1 (a power of
                                        two, 16 <= k1 < k): every table gets two
                                        block levels (Section 3.3), as
                                        rmq_build with this sub_block_size */
} rmq_server_config;

typedef struct rmq_server_stats {
    int64_t submitted, completed, batches, queries;
    int64_t slot_capacity;           /* queries one slot (one batch) can hold     */
    int64_t max_inflight;            /* most batches seen on the device at once   */
    size_t index_bytes;              /* device bytes of the resident tables       */
    size_t hbm_bytes;                /* all device bytes the server holds and
                                        admits against hbm_budget_bytes        */
} rmq_server_stats;

typedef struct rmq_request_info {
    double t_submit, t_launch, t_done;  /* rmq_server_clock() seconds           */
    int32_t batch_requests;             /* requests in the batch it went with   */
    int32_t reserved;
} rmq_request_info;

typedef struct rmq_server_s *rmq_server;

rmq_status rmq_server_create(const rmq_server_config *cfg, rmq_server *out);

/* Build and keep a resident index of device array A (k = block_size, 0 = auto;
 * two block levels when the server's config has a sub_block_size);
 * synchronous.  A must stay alive and unmodified for the server's life.
 * Admission by footprint: returns RMQ_ERR_OUT_OF_MEMORY, building nothing,
 * when the table's rmq_build_bytes would take the server's device memory
 * above cfg.hbm_budget_bytes, and RMQ_ERR_INVALID_ARG when max_tables are
 * already resident (or being added by other threads). */
rmq_status rmq_server_add_array(rmq_server s, const int32_t *A, int64_t n, int32_t block_size,
                                int32_t *table_id);

/* Queue q >= 1 queries on a resident array.  L, R and out are HOST pointers
 * that must stay valid until rmq_server_wait returns for the ticket; out
 * receives the leftmost argmin of each query (-1 for an invalid one).  q may
 * not exceed the slot capacity (see rmq_server_stats). */
rmq_status rmq_server_submit(rmq_server s, int32_t table_id, const int32_t *L, const int32_t *R,
                             int64_t q, int32_t *out, uint64_t *ticket);

/* A request with its arrival time on rmq_server_clock(). */
typedef struct rmq_request_spec {
    int32_t table_id;
    int32_t reserved;
    const int32_t *L, *R;   /* host */
    int64_t q;
    int32_t *out;           /* host */
    double t_arrival;
} rmq_request_spec;

/* Submit count requests, each at its arrival time (a load generator for an
 * arrival process fixed in advance, e.g. Poisson); blocks in the calling
 * thread until the last one is submitted.  tickets[i] gets request i's
 * ticket. */
rmq_status rmq_server_submit_schedule(rmq_server s, int32_t count, const rmq_request_spec *specs,
                                      uint64_t *tickets);

/* Block until the request is answered; releases the ticket (wait once). */
rmq_status rmq_server_wait(rmq_server s, uint64_t ticket, rmq_request_info *info);

rmq_status rmq_server_stats_get(rmq_server s, rmq_server_stats *out);

/* The server's clock (seconds, monotonic), for timestamps comparable with
 * rmq_request_info. */
double rmq_server_clock(void);

/* Drain every queued request, stop the threads and free everything. */
rmq_status rmq_server_destroy(rmq_server s);

/* ----------------------------------------------------------------------------
 * For tests of the failure report only; not for production callers.
 * on != 0: every endpoint or pair sort enqueued afterwards in this process
 * starts with its abort word already set, as if a bounded wait had run out,
 * so that each wait ends at its first unpublished predecessor, every kernel
 * exits normally, and the call reports the failure as described under "Sort
 * failure".  on = 0 restores normal sorting.  Process-wide. */
rmq_status rmq_test_sort_abort(int32_t on);

/* ----------------------------------------------------------------------------
 * Per-stage timing (Table 1's stages).  A timer collects HIP events that
 * rmq_query_batch_ex records on its stream; rmq_timer_read waits for them and
 * returns the milliseconds of each stage of the last call that used the
 * timer (0 for stages that did not run) and the total. */
rmq_status rmq_timer_create(rmq_timer **t);
rmq_status rmq_timer_read(rmq_timer *t, float *stage_ms, float *total_ms);
rmq_status rmq_timer_destroy(rmq_timer *t);

#ifdef __cplusplus
}
#endif

#endif /* RMQ_H */
