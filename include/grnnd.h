/*
 * grnnd.h -- C ABI of the MI355X (gfx950) GRNND graph-construction library.
 *
 * The library builds an out-degree-bounded approximate nearest-neighbour
 * graph with the GPU-parallel Relative NN-Descent method of Li, Chang, Li and
 * Miyazaki (GRNND): random initial pools (Alg. 3), T1 outer
 * iterations of T2 update rounds (Alg. 4, Eq. 2, disordered propagation,
 * Section 3.3) over fixed-capacity double-buffered pools (Section 3.5), with
 * reverse-edge sampling between outer iterations (Section 3.6), and a last
 * strict RNG pass (Eq. 1, Alg. 2's scan without redirection) that yields the
 * output rows.
 *
 * Conventions shared by every call:
 *   - Every function returns GRNND_OK (0) or a negative status; the text of the
 *     last error on the calling thread is returned by grnnd_last_error().
 *   - Array arguments are DEVICE pointers owned by the caller, unless a comment
 *     says "host". The library keeps no pointer after a call returns.
 *   - Calls are asynchronous on the HIP stream passed as `stream` (hipStream_t
 *     cast to void*; NULL is the default stream). Outputs are valid once the
 *     caller has synchronised that stream. Argument errors are reported
 *     synchronously; device faults surface at the caller's synchronisation.
 *   - Scratch memory is the caller's: a `workspace` of at least the size that
 *     the matching *_workspace_size call reports. No call of this header
 *     allocates or frees device memory.
 *   - points: n rows of d float32, row-major, contiguous (row stride d).
 *   - Keys are squared L2 distances (metric GRNND_METRIC_L2) or negated inner
 *     products (GRNND_METRIC_IP). Pool and graph rows are sorted by
 *     (key, id) ascending and padded at the end with id -1 / key +inf.
 *   - Ids are int32: n must be below 2^31.
 *   - Limits: 2 <= n, 1 <= d <= 4096, 1 <= R <= 64.
 */
#ifndef GRNND_H
#define GRNND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define GRNND_OK 0
#define GRNND_EINVAL (-1)   /* bad argument (null pointer, out-of-range size) */
#define GRNND_ENOSPACE (-2) /* workspace smaller than the reported size */
#define GRNND_EDEVICE (-3)  /* a HIP call failed */
#define GRNND_EBUDGET (-4)  /* server: the request can never fit the HBM budget */
#define GRNND_ENOTSUP (-5)  /* valid request this build cannot serve */

/* ---- metrics ---- */
#define GRNND_METRIC_L2 0
#define GRNND_METRIC_IP 1

/* ---- candidate arrival order in an update round (Section 3.3, 4.3) ---- */
#define GRNND_ORDER_DISORDERED 0
#define GRNND_ORDER_ASCENDING 1
#define GRNND_ORDER_DESCENDING 2

/* ---- distance-tile precision ----
 * The update rounds and the output pass decide Eq. 2 / Eq. 1 comparisons
 * from a Gram tile of the candidates' rows on the matrix cores. FP32 tiles
 * use the FP32 points. The narrow forms gather a copy of y = x - c instead
 * (c = column means rounded to integers for L2, 0 for IP), made once per
 * call, in BF16 or FP16, or in OCP FP8-e4m3 with a power-of-two scale per
 * row; the tile accumulates in FP32. Per row the copy records its exact
 * rounding error |s q - y| and |y|, which bound every tile entry's error; a
 * comparison inside that bound (plus the FP32 one) is re-decided with the
 * canonical FP32 distance, and stored keys are always canonical FP32
 * distances. Every decision therefore equals the FP32 tile's, and the
 * output is bit-identical to an FP32 build; the narrow forms differ only in
 * bytes gathered and in the number of re-decided comparisons
 * (GRNND_STAT_RECHECKS). */
#define GRNND_PREC_FP32 0
#define GRNND_PREC_BF16 1
#define GRNND_PREC_FP16 2
#define GRNND_PREC_FP8_E4M3 3

/* ---- kinds of grnnd_step ---- */
#define GRNND_STEP_UPDATE 0  /* one UPDATE_NEIGHBORS_PARALLEL round (Alg. 4) */
#define GRNND_STEP_REVERSE 1 /* one REVERSE_EDGE_SAMPLING pass (Section 3.6) */

#define GRNND_MAX_R 64

/* ---- device statistics counters (uint64, accumulated with +=) ---- */
#define GRNND_NSTATS 11
#define GRNND_STAT_TILE_PAIRS 0  /* sum of K(K-1)/2 over vertex-rounds      */
#define GRNND_STAT_RECHECKS 1    /* tile decisions re-evaluated directly    */
#define GRNND_STAT_REDIRECTS 2   /* candidates redirected (Eq. 2)           */
#define GRNND_STAT_SURVIVORS 3   /* candidates kept by their own vertex     */
#define GRNND_STAT_ITEMS 4       /* items merged into write pools           */
#define GRNND_STAT_CANDIDATES 5  /* sum of K (candidate rows gathered)      */
#define GRNND_STAT_INIT_DISTS 6  /* distances of the initial pools          */
#define GRNND_STAT_FINAL_PAIRS 7 /* sum of K(K-1)/2 of the output pass      */
#define GRNND_STAT_OVERFLOW 8    /* items beyond their destination's bucket
                                    of R slots (moved by the overflow pass)  */
#define GRNND_STAT_LONG_MERGES 9 /* write-pool merges of more than 64 items
                                    (merged in 128-item chunks)             */
#define GRNND_STAT_DEFERRED 10   /* redirect keys the merge computed (rows of
                                    512 or more elements; candidates the
                                    destination already held are skipped)   */

/*
 * Construction parameters (the symbols of the paper's Table 1).
 *   S         initial neighbours per vertex, 1..R (Alg. 3)
 *   T1, T2    outer iterations, update rounds per outer iteration (Alg. 3)
 *   rho       reverse-edge sampling ratio in (0, 1) (Section 3.6)
 *   order     GRNND_ORDER_* arrival order of candidates in a round
 *   precision GRNND_PREC_* of the candidate distance tile
 *   reverse   GRNND_REVERSE_* reading of the "top rho k" neighbours a vertex
 *             sends itself to in reverse-edge sampling (Section 3.6)
 *   check     debugging aid, 0 or 1: with 1, grnnd_step first verifies that
 *             its read pool is canonical (see grnnd_step) and fails with
 *             GRNND_EINVAL naming the first offending row and what is wrong;
 *             this costs one pass over the pool that also recomputes every
 *             key's distance, and a synchronization of `stream`. Other
 *             calls ignore it.
 */
typedef struct grnnd_params {
    int32_t S;
    int32_t T1;
    int32_t T2;
    float rho;
    int32_t order;
    int32_t precision;
    int32_t reverse;
    int32_t check;
} grnnd_params;

/* ---- reverse-edge sampling: which floor(rho k) of a row's k entries ----
 * HASH: the first in hash order h(seed, 0x2000 + t1, v, id), standing for the
 * random pool order that disordered propagation leaves in the paper's
 * design (a canonical pool is sorted, so the library draws that order);
 * NEAREST: the nearest, the first by (key, id). */
#define GRNND_REVERSE_HASH 0
#define GRNND_REVERSE_NEAREST 1

/* Fills *p (host) with the defaults: S = R, T1 = iters, T2 = 4, rho = 0.6,
 * DISORDERED order, FP32 tiles, HASH reverse sampling, no pool check. EINVAL on a null
 * pointer or R/iters < 1. */
int grnnd_params_default(grnnd_params *p, int32_t R, int32_t iters);

/* Workspace bytes (host out) needed by grnnd_build / grnnd_build_ex /
 * grnnd_init_pools / grnnd_step / grnnd_finalize for these sizes. `p` may be
 * NULL for the defaults. The same workspace serves every one of those calls.
 * EINVAL on sizes or parameters that the builds would refuse. */
int grnnd_workspace_size(int64_t n, int32_t d, int32_t R, const grnnd_params *p,
                         size_t *bytes);

/*
 * Full construction with default parameters and `iters` outer iterations
 * (Alg. 3 followed by the output pass). Writes out_adj (n x R int32):
 * row v holds at most R neighbours of v, ascending by (key, id), -1 padded;
 * no self loops, no duplicates, at least one neighbour, and every kept pair
 * (u, w) of a row satisfies d(u, w) >= max(key_u, key_w) (Eq. 1).
 * Deterministic: the same inputs and seed give the same bits.
 */
int grnnd_build(const float *points, int64_t n, int32_t d, int32_t metric, int32_t R,
                int32_t iters, uint64_t seed, int32_t *out_adj, void *workspace,
                size_t ws_bytes, void *stream);

/* As grnnd_build with explicit parameters. out_keys (n x R float, nullable)
 * receives the keys of out_adj. dev_stats (GRNND_NSTATS uint64, nullable) is
 * incremented by the counters listed above. */
int grnnd_build_ex(const float *points, int64_t n, int32_t d, int32_t metric, int32_t R,
                   const grnnd_params *p, uint64_t seed, int32_t *out_adj,
                   float *out_keys, uint64_t *dev_stats, void *workspace,
                   size_t ws_bytes, void *stream);

/*
 * Batched construction: `count` independent collections of the same d,
 * metric, R and parameters built together, every kernel launch of the build
 * covering the vertices of all of them (the serving form's shared launches).
 * The collections' points are copied into one concatenated array of the
 * workspace; a collection's random draws use its own seed on its local ids
 * and its candidates never leave it (initial draws stay inside it, and every
 * later candidate comes from its own pools), so each collection's out_adj /
 * out_keys equals grnnd_build_ex on it alone with its seed, bit for bit.
 * items: host array of count entries; 1 <= count <= 64; each n >= 2 and the
 * n sum below 2^31. dev_stats (nullable) receives the counters summed over
 * the batch. The workspace is grnnd_batch_workspace_size bytes (256-byte
 * aligned).
 */
typedef struct grnnd_batch_item {
    const float *points; /* device, n x d FP32, row-major, 16-byte aligned if d % 4 == 0 */
    int64_t n;
    uint64_t seed;
    int32_t *out_adj;    /* device, n x R */
    float *out_keys;     /* device, n x R, nullable */
} grnnd_batch_item;

int grnnd_batch_workspace_size(const int64_t *ns, int32_t count, int32_t d, int32_t R,
                               const grnnd_params *p, size_t *bytes);
int grnnd_build_batch(const grnnd_batch_item *items, int32_t count, int32_t d, int32_t metric,
                      int32_t R, const grnnd_params *p, uint64_t *dev_stats, void *workspace,
                      size_t ws_bytes, void *stream);

/* Initial pools only (Alg. 3): for each v, the first min(S, n-1)
 * distinct ids != v of the hash stream h(seed, 0x3000, v, j) mod n, with
 * their keys, as a sorted padded pool (n x R ids and keys). */
int grnnd_init_pools(const float *points, int64_t n, int32_t d, int32_t metric,
                     int32_t R, int32_t S, uint64_t seed, int32_t *out_ids,
                     float *out_keys, uint64_t *dev_stats, void *workspace,
                     size_t ws_bytes, void *stream);

/*
 * One step on caller-held pools (the read pool in_*, the write pool out_*;
 * each n x R; they must not overlap). The read pool must be canonical: in
 * each row v the valid entries come first and hold ids in [0, n), none equal
 * to v and none twice, strictly ascending by (key, id), each key the
 * canonical FP32 distance d(v, id); the rest of the row is id -1 with key
 * +inf (the form every call of this library writes). A pool that is not
 * canonical gives undefined results unless p->check is set, which makes the
 * call verify it first and fail with GRNND_EINVAL.
 *   kind GRNND_STEP_UPDATE: one update round `round` (Alg. 4 with Eq. 2) in
 *     the order p->order; out = the first R by (key, id) of the items sent
 *     to each vertex, one per id (smallest key).
 *   kind GRNND_STEP_REVERSE: the reverse-edge sampling after outer iteration
 *     `round` (used as t1; Section 3.6) with ratio p->rho and reading
 *     p->reverse.
 * `p` may be NULL for the defaults. Chaining init, steps and finalize with
 * the schedule of Alg. 3 reproduces grnnd_build_ex bit for bit.
 */
int grnnd_step(const float *points, int64_t n, int32_t d, int32_t metric, int32_t R,
               const int32_t *in_ids, const float *in_keys, int32_t *out_ids,
               float *out_keys, uint64_t seed, uint32_t round, int32_t kind,
               const grnnd_params *p, uint64_t *dev_stats, void *workspace,
               size_t ws_bytes, void *stream);

/* Output pass on a canonical pool: per row, Alg. 2's scan in ascending
 * (key, id) with the strict test of Eq. 1 and no redirection; writes the
 * kept ids (and keys, nullable) ascending, -1 / +inf padded. */
int grnnd_finalize(const float *points, int64_t n, int32_t d, int32_t metric,
                   int32_t R, const int32_t *in_ids, const float *in_keys,
                   int32_t *out_adj, float *out_keys, uint64_t *dev_stats,
                   void *workspace, size_t ws_bytes, void *stream);

/*
 * Distance-tile probe, for measuring the tiles the update rounds decide Eq. 2
 * from (Eq. 2 compares d(u, w) with max(d(v, u), d(v, w)) for candidates u,
 * w of v). For each of nv candidate sets (rows of ids, nv x R int32, valid
 * ids first, -1 padded; K valid entries) the tile of precision p->precision
 * is formed exactly as in a round, and for every ordered pair (i, j), i != j,
 * of its first K entries writes, at [(q R + i) R + j] (each output nv x R x R
 * float32):
 *   out_tile  the tile's distance of the pair,
 *   out_band  the half-width of the band around a threshold inside which a
 *             round re-decides the comparison with the canonical distance,
 *   out_canon the canonical FP32 distance (the one stored as a key).
 * Entries with i == j or i, j >= K are not written. The workspace is the
 * build's (grnnd_workspace_size for n, d, R, p). Test and measurement use.
 */
int grnnd_tile_probe(const float *points, int64_t n, int32_t d, int32_t metric, int32_t R,
                     const grnnd_params *p, const int32_t *ids, int64_t nv, float *out_tile,
                     float *out_band, float *out_canon, void *workspace, size_t ws_bytes,
                     void *stream);

/* Workspace bytes for grnnd_search and grnnd_medoid (host out). */
int grnnd_search_workspace_size(int64_t n, int32_t d, int64_t nq, size_t *bytes);

/*
 * Approximate medoid, the entry point of the evaluation search (Section 4.1
 * searches every graph with one routine from one entry): the id of the point
 * nearest in L2 to the mean of all points, ties by the smaller id, written to
 * *out_entry (device int64). Computed in FP64: column sums of the rows, then
 * mean = sum / n; for each point sum_k (x_k - mean_k)^2 in coordinate order,
 * each subtraction, product and sum rounded separately. The metric of the
 * graph does not enter. points: n x d FP32, row stride d, any alignment.
 * The workspace is grnnd_search's (grnnd_search_workspace_size with any nq),
 * 256-byte aligned. EINVAL for null pointers or n, d out of range;
 * ENOSPACE for a short workspace.
 */
int grnnd_medoid(const float *points, int64_t n, int32_t d, int64_t *out_entry,
                 void *workspace, size_t ws_bytes, void *stream);

int grnnd_search(const float *points, int64_t n, int32_t d, int32_t metric,
                 const int32_t *adj, int32_t R, int64_t entry, const float *queries,
                 int64_t nq, int32_t k, int32_t L, int32_t *out_ids, float *out_keys,
                 void *workspace, size_t ws_bytes, void *stream);

/*
 * Kernel timing. While enabled, every launch the library makes is bracketed
 * by two HIP events recorded on the stream of that launch, tagged with its
 * kernel class (GRNND_PROF_*). grnnd_profile_read waits for the recorded
 * events, writes per class the total milliseconds (ms, host array of
 * GRNND_NPROF doubles) and the number of launches (launches, host array of
 * GRNND_NPROF int64), and forgets them. Process-wide; not for concurrent
 * callers. The library creates and destroys the events itself.
 */
#define GRNND_NPROF 6
#define GRNND_PROF_INIT 0    /* initial pools                     */
#define GRNND_PROF_UPDATE 1  /* update-round candidate kernel     */
#define GRNND_PROF_MERGE 2   /* allocation + scatter + merge      */
#define GRNND_PROF_REVERSE 3 /* reverse-sampling emit kernel      */
#define GRNND_PROF_FINAL 4   /* output-pass kernel                */
#define GRNND_PROF_SEARCH 5  /* search kernel                     */
int grnnd_profile_enable(int on);
int grnnd_profile_read(double *ms, int64_t *launches);

/*
 * Build server (continuous batching of many graph builds on one GPU).
 *
 * A server owns nothing but host bookkeeping: the caller gives it a device
 * arena (budget_bytes, 256-byte aligned) from which every admitted build's
 * workspace is carved, and a number of slots, each a stream of its own
 * (default priority). A host thread admits queued requests in arrival order
 * whenever a slot is free and the arena has room, batching queued requests
 * of the head request's class into one build whose launches cover all of
 * them (grnnd_build_batch; see grnnd_server_set_batch), enqueues the build
 * on the slot's stream, and retires it when its completion event has passed,
 * returning its arena range; builds in different slots overlap on the
 * device. A request's result does not depend on what else runs: it equals
 * grnnd_build_ex on its own stream, bit for bit.
 *
 * grnnd_request: points (device, n x d FP32, row-major, 16-byte aligned),
 * metric, R, params (NULL: the defaults for R with T1 = 4), seed, and the
 * outputs out_adj (device, n x R int32) and out_keys (device, n x R FP32,
 * nullable). All of them are the caller's and must stay valid until the
 * request is done; the points must be completely written when the request
 * is submitted (the server's streams do not wait for any other stream).
 */
typedef struct grnnd_request {
    const float *points;
    int64_t n;
    int32_t d;
    int32_t metric;
    int32_t R;
    const grnnd_params *params;
    uint64_t seed;
    int32_t *out_adj;
    float *out_keys;
} grnnd_request;

typedef struct grnnd_server grnnd_server;

#define GRNND_REQ_QUEUED 0
#define GRNND_REQ_RUNNING 1
#define GRNND_REQ_DONE 2

typedef struct grnnd_server_stats {
    int64_t submitted;
    int64_t completed;
    int64_t failed;
    int64_t peak_inflight;     /* most builds running at once            */
    uint64_t peak_arena_bytes; /* most arena bytes in use at once        */
    int64_t batches;           /* batched builds of two or more requests */
    int64_t batched_requests;  /* requests served by those               */
} grnnd_server_stats;

/* Creates a server on the current device. slots in [1, 64]. EINVAL on bad
 * arguments, EDEVICE if a stream cannot be created. */
int grnnd_server_create(void *arena, size_t budget_bytes, int32_t slots, grnnd_server **out);
/* Queues a request (validated here; EBUDGET if its workspace exceeds the
 * budget) and returns its ticket (host out). */
int grnnd_server_submit(grnnd_server *s, const grnnd_request *r, uint64_t *ticket);
/* State of a ticket (GRNND_REQ_* or the negative status it failed with) and,
 * once done, its latency from submission to completion in seconds (either
 * pointer may be NULL). EINVAL for an unknown ticket. */
int grnnd_server_poll(grnnd_server *s, uint64_t ticket, int32_t *state, double *latency_s);
/* Batching of queued requests (the default is 16 requests, 2^18 points):
 * when a slot frees, the head request and the queued requests of its class
 * (equal d, metric, R and parameters), each of at most max_points points and
 * together at most max_requests requests and max_points points, run as one
 * grnnd_build_batch whose launches cover all of them; every request's result
 * is still that of its build alone. max_requests = 1 turns batching off. */
int grnnd_server_set_batch(grnnd_server *s, int32_t max_requests, int64_t max_points);
/* Blocks until every submitted request is done or failed. */
int grnnd_server_drain(grnnd_server *s);
int grnnd_server_stats_read(grnnd_server *s, grnnd_server_stats *out);
/* Drains, stops the admission thread, destroys the streams and the server. */
int grnnd_server_destroy(grnnd_server *s);

/*
 * Allocation-free construction, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, semantics and result as grnnd_build_ex,
 * bit for bit, without the workspace: the scratch memory is a static device
 * array of the library, GRNND_NOALLOC_SCRATCH_BYTES bytes per GPU, reserved
 * when the library's code is loaded on that GPU and held until the process
 * ends. The call allocates and frees nothing. Sizes whose workspace
 * (grnnd_workspace_size) exceeds the array are refused with GRNND_ENOSPACE
 * before anything is enqueued. Every call on one GPU uses that GPU's one
 * array: calls that overlap on a GPU (other streams or host threads before
 * the earlier call's work has completed) race and give undefined results;
 * calls in order on one stream are safe. Each call clears what must start
 * at zero itself.
 */
#define GRNND_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int grnnd_build_noalloc(const float *points, int64_t n, int32_t d, int32_t metric, int32_t R,
                        const grnnd_params *p, uint64_t seed, int32_t *out_adj,
                        float *out_keys, uint64_t *dev_stats, void *stream);

/* Text of the last error on the calling thread ("" if none). */
const char *grnnd_last_error(void);

/* Library version, as major * 10000 + minor * 100 + patch. */
int grnnd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRNND_H */
