/*
 * tc.h — C ABI of the MI355X (gfx950) degree-partitioned sampling triangle
 * counter.
 *
 * The method is that of Kolountzakis, Miller, Peng and Tsourakakis,
 * "Efficient Triangle Counting in Large Graphs via Degree-based Vertex
 * Partitioning" (arXiv:1011.0468): sparsify the graph by keeping each edge
 * with probability p (section 3.1), split the vertices at m^(1/2) into light
 * and heavy sets (section 3.2), count exactly on the sparsified graph and
 * rescale by 1/p^3 (section 3.1; the "Sparsified + Exact" columns of Table 2),
 * plus the random-projection trace estimator of section 5.1 and the
 * three-pass semi-streaming variant of section 5.2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Graphs are simple and undirected (Table 1: G([n],E)); vertex ids are
 *   0-based int32 in [0, n).  Input pairs may be directed, repeated or
 *   self-loops; they are symmetrised and cleaned (section 4.1).
 * - Every call returns a tc_status.  On error no output is written and a
 *   message is available from tc_last_error() on the calling thread.  No C++
 *   exception crosses this boundary.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *   enqueued on it; every call that produces host-visible outputs synchronises
 *   that stream before returning.
 * - Device memory is obtained through the allocator installed with
 *   tc_set_allocator (default: a process-wide caching pool over hipMalloc).
 * - Results are deterministic functions of (graph, p, seed, k).  tc_params
 *   changes only the speed and the reported light/heavy split, never the
 *   triangle count.
 * - All counts are exact int64.  Limits: n <= 2^31-1, 2 * num_pairs <= 2^31-1
 *   (int32 CSR), else TC_ERR_OVERFLOW.
 */
#ifndef TC_H_
#define TC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TC_OK = 0,
    TC_ERR_INVALID = 1,   /* bad argument: null pointer, id out of range, p outside (0,1], ... */
    TC_ERR_OOM = 2,       /* the allocator returned NULL */
    TC_ERR_DEVICE = 3,    /* a HIP runtime call or kernel launch failed */
    TC_ERR_OVERFLOW = 4,  /* a size or an integer bound exceeds what the int32/int64 layout holds */
    TC_ERR_BUDGET = 5     /* a request does not fit the memory budget of a server */
} tc_status;

/* Opaque graph handle: owns a device CSR (row_ptr int32[n+1], col int32[2m]
   with each list sorted ascending, the row index of every CSR entry, and
   deg int32[n]; a graph from tc_build_csr also keeps one byte per entry, a
   class of the neighbour's degree that orders degrees) until tc_graph_free. */
typedef struct tc_graph_s* tc_graph;

/* Light/heavy threshold (section 3.2 uses deg <= m^(1/2) for light).  A vertex
   of the counted graph is heavy iff heavy_den^2 * deg^2 > heavy_num^2 * m,
   evaluated exactly (no overflow).  heavy_num = 0 makes every non-isolated
   vertex heavy.  heavy_num and heavy_den above 32768 (and heavy_num < 0 or
   heavy_den < 1) give TC_ERR_INVALID, also in tc_tuning. */
typedef struct {
    int32_t heavy_num;   /* default 1 */
    int32_t heavy_den;   /* default 1, must be >= 1 */
    int32_t use_tuned;   /* 1: take launch parameters from the autotuner's table */
} tc_params;

/* Result of one exact count (on the graph itself, or on one sparsified copy). */
typedef struct {
    int64_t triangles;        /* T = T_L + T_H */
    int64_t light;            /* T_L: triangles with at least one light vertex */
    int64_t heavy;            /* T_H: triangles with three heavy vertices */
    int64_t m;                /* edges of the counted graph (m' after sampling) */
    int64_t n_heavy;          /* |H| */
    /* work statistics of the light phase (for throughput models) */
    int64_t light_sources;    /* light vertices u with out-degree d+(u) >= 2 */
    int64_t light_out_edges;  /* sum of d+(u) over those u (oriented pairs (u, v)) */
    int64_t wedges;           /* sum of C(d+(u), 2) over those u */
    int64_t gather;           /* sum over those pairs of d+(v) (list entries read if every pair
                                 streamed N+(v)) */
    int64_t probes;           /* list entries actually streamed and tested: pair (u, v) streams
                                 the members of N+(u) ranked above v (all of N+(u) when
                                 d+(u) > 1024) or N+(v), the shorter within the staging cap,
                                 and nothing when no member of N+(u) ranks above v */
    int64_t items_small;      /* work items of the wave-per-item kernel */
    int64_t items_large;      /* work items of the block-per-item kernel */
    int64_t model_bytes_small;/* bytes the wave-per-item kernel must read (list model) */
    int64_t model_bytes_large;/* bytes the block-per-item kernel must read (list model) */
} tc_counts;

/* Device allocator used for every internal buffer and graph.  alloc returns
   NULL on failure (the call then fails with TC_ERR_OOM).  Passing NULL for
   both restores the built-in caching pool.  Not thread-safe against
   concurrent calls. */
typedef void* (*tc_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*tc_free_fn)(void* ptr, void* stream, void* ctx);
tc_status tc_set_allocator(tc_alloc_fn alloc, tc_free_fn free_, void* ctx);

/* Build the simple undirected graph of the pairs (src[i], dst[i]), i < num_pairs
   (section 4.1: duplicates and self-loops removed; section 4.2: sorted
   neighbour lists).  src/dst are device pointers if on_device, else host
   pointers (copied in).  They are borrowed for the call.  Ids outside [0,n)
   give TC_ERR_INVALID.  *out receives a new handle. */
tc_status tc_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                       int32_t on_device, void* stream, tc_graph* out);

/* Size queries.  Any output pointer may be NULL. */
tc_status tc_graph_info(tc_graph g, int64_t* n, int64_t* m, int32_t* max_deg);

/* Borrowed device pointers to the CSR (valid until tc_graph_free):
   row_ptr int32[n+1], col int32[2m]. */
tc_status tc_graph_csr(tc_graph g, const int32_t** row_ptr, const int32_t** col);

/* Copy the CSR out into caller buffers: row_ptr[n+1], col[2m] and deg[n]
   (any may be NULL), device pointers if on_device, else host pointers. */
tc_status tc_graph_read(tc_graph g, int32_t* row_ptr, int32_t* col, int32_t* deg, int32_t on_device, void* stream);

/* Edge sparsification (section 3.1): a new graph keeping each undirected edge
   {u,v} iff (mix64(mix64(min<<32 | max) ^ mix64(seed ^ 0x54435F53414D504C)) >> 11)
   < floor(p * 2^53), where mix64 is the SplitMix64 output function.  p must be
   finite and in (0,1]. */
tc_status tc_sample(tc_graph g, double p, uint64_t seed, void* stream, tc_graph* out_sampled);

/* Exact triangle count of g with the light/heavy split (section 3.2; the
   "Exact" columns of Table 2).  prm may be NULL (defaults). */
tc_status tc_count_exact(tc_graph g, const tc_params* prm, void* stream, tc_counts* out);

/* Sparsify-then-count estimate (section 3.1): for each seed s, T_s is the exact
   count of the graph sampled with (p, s), and est_s = (double)T_s / ((p*p)*p).
   num_seeds >= 1, 1 <= num_groups <= num_seeds, num_seeds % num_groups == 0.
   mom_est receives the median of means of the group means (groups of
   num_seeds/num_groups consecutive seeds; for an even number of groups the
   mean of the two middle group sums, divided once).  per_seed[num_seeds],
   per_seed_est[num_seeds] and mom_est may each be NULL. */
tc_status tc_estimate(tc_graph g, double p, const uint64_t* seeds, int32_t num_seeds,
                      int32_t num_groups, const tc_params* prm, void* stream,
                      tc_counts* per_seed, double* per_seed_est, double* mom_est);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   single-seed form of tc_estimate, bit-identical to tc_estimate(g, p, &seed,
   1, 1, prm, stream, out, est, NULL), whose every intermediate buffer lives
   in one fixed device array of 64 MiB that the library reserves per GPU (held
   until the process ends).  The call makes no hipMalloc, hipFree or other
   allocating call; it enqueues on `stream` and synchronises it before
   returning.  The graph g (built earlier, e.g. by tc_build_csr) and the host
   outputs are the caller's.  A count that needs more scratch than the array
   holds (roughly graphs beyond a few hundred thousand edges) is refused with
   TC_ERR_BUDGET before any device work.  Calls on one GPU share its array:
   the library serialises them (one at a time per device), and the array keeps
   the last call's contents; each call clears what it needs.  Profiling hooks
   record nothing during this call.  est may be NULL.  Other errors as
   tc_estimate. */
tc_status tc_estimate_noalloc(tc_graph g, double p, uint64_t seed, const tc_params* prm, void* stream,
                              tc_counts* out, double* est);

/* One stage of tc_estimate_adaptive. */
typedef struct {
    double p;          /* keep probability of the stage */
    double estimate;   /* median of means of its seeds, as tc_estimate's mom_est */
    int64_t m_sum;     /* sum of m' over its seeds (edges counted) */
} tc_stage;

/* Adaptive keep probability: the remarks after Table 2 recommend varying p
   and reading the estimate where it settles; section 3.3 balances the sampling
   term pm against the counting term.  Stage k (k = 0, 1, ..) runs tc_estimate
   with p_k = min(1, p0 * 2^k), the num_seeds seeds seed0 + k * num_seeds + i
   (i < num_seeds, modulo 2^64) and num_groups groups.  The search stops after
   the first stage k >= 1 whose estimate E_k is positive and satisfies
   |E_k - E_{k-1}| <= tol * E_k (double arithmetic; an estimate of 0 never
   counts as settled), after a stage with
   p_k = 1 (the exact count), or after max_stages stages.  stages[max_stages]
   (host) receives the stages run and *num_stages their number.  *p_balance
   (may be NULL) receives min(1, (m^(1/2) ln(n) / (E tol^2))^(2/5)), the p at
   which section 3.3's two terms balance with t = E, the last estimate, and
   epsilon = tol (1 if E <= 0 or tol = 0).  p0 in (0, 1], tol >= 0 and
   finite, max_stages >= 1; num_seeds and num_groups as for tc_estimate.
   Errors as tc_estimate; stages written before an error stay valid. */
tc_status tc_estimate_adaptive(tc_graph g, double p0, double tol, uint64_t seed0, int32_t num_seeds,
                               int32_t num_groups, int32_t max_stages, const tc_params* prm, void* stream,
                               tc_stage* stages, int32_t* num_stages, double* p_balance);

/* Triple sampling (section 3.2, "Triple Sampling"; the Simple and Hybrid
   columns of Table 2) on g, or on g sparsified with (p, sample_seed) as
   tc_sample does when p < 1.  The candidate set U of the counted graph, in
   order: vertices u ascending; a vertex of the wedge kind gives its pairs of
   neighbour positions a < b in colex order ((0,1), (0,2), (1,2), (0,3), ..),
   the triple (N(u)[a], u, N(u)[b]), closed iff N(u)[a] and N(u)[b] are
   adjacent; a vertex of the extension kind gives, for each neighbour
   position a (v = N(u)[a]) and each neighbour position j of v
   (w = N(v)[j]), the triple (u, v, w), closed iff w != u and w is adjacent
   to u.  hybrid = 0 (Simple): every vertex is of the wedge kind; hybrid = 1:
   the extension kind iff deg^2 > m (degree and m of the counted graph).
   Sample i < num_samples is triple r_i = floor(h_i |U| / 2^64) with
   h_i = mix64(mix64(i) ^ mix64(triple_seed ^ 0x54435F545249504C)); a closed
   sample weighs 60 / (3 + its extension-kind vertices), so each triangle's
   appearances in U weigh 60 in all.  estimate =
   ((double)|U| * (double)weight_sum) / (60.0 * (double)num_samples), then
   divided by (p*p)*p.  num_samples >= 1; errors as tc_sample. */
typedef struct {
    int64_t size;        /* |U| */
    int64_t weight_sum;  /* sum of the closed samples' weights */
    int64_t closed;      /* closed samples */
    int64_t m;           /* edges of the counted graph */
    double estimate;     /* of the triangle count of g */
} tc_triple_result;

tc_status tc_triple_estimate(tc_graph g, double p, uint64_t sample_seed, int32_t hybrid, int64_t num_samples,
                             uint64_t triple_seed, void* stream, tc_triple_result* out);

/* Semi-streaming estimate (section 5.2 and its Lemma): three passes over the
   edges of g, with g's adjacency lists in order (the layout of tc_graph).
   Edges are numbered as upper entries: edge r is the (r - upre[u])-th
   neighbour above u of the vertex u with upre[u] <= r < upre[u+1], where
   upre is the exclusive prefix over u of the neighbours above u.
   Pass 1 draws s1 = ceil(d m^(1/2) ln n) edges with replacement (draw i is
   edge floor(h m / 2^64), h = mix64(mix64(i) ^ mix64(seed ^
   0x54435F5354524D31))); their endpoints are the candidates, and the
   candidates with deg^2 > m form H.  Pass 2 draws num_samples elements with
   replacement (draw j is element floor(h' |U| / 2^64), h' = mix64(mix64(j) ^
   mix64(seed ^ 0x54435F5354524D32))) of U = L followed by X: L holds, for
   every vertex u outside H (ascending), its pairs of neighbour positions
   a < b in colex order, closed iff N(u)[a] and N(u)[b] are adjacent; X holds,
   for every h of H (ascending) and every edge e = (v, w) in edge order, the
   pair (h; e), closed iff h is not in e and h is adjacent to v and w.  Pass 3
   looks up the closing edges the draws ask for (one for a wedge, two for a
   pair whose vertex is not in its edge, none otherwise).  estimate =
   ((double)|U| * (double)closed) / (3.0 * (double)num_samples), 0 when
   num_samples = 0; every field is 0 except m, draws1 when n < 2 or m = 0.
   d > 0 and finite and num_samples >= 0, else TC_ERR_INVALID;
   TC_ERR_OVERFLOW if num_samples > 2^28 or s1 > 2^40.  The device memory it
   takes (through the allocator) is at most 72 num_samples + 49 (n + 1) bytes
   plus 17 KiB and the scans' scratch. */
typedef struct {
    int64_t draws1;      /* s1, the edge draws of pass 1 */
    int64_t candidates;  /* distinct endpoints of the pass-1 draws */
    int64_t heavy;       /* |H| */
    int64_t light_size;  /* |L| */
    int64_t size;        /* |U| = |L| + |H| m */
    int64_t queries;     /* closing-edge lookups of pass 3 */
    int64_t closed;      /* closed draws */
    int64_t m;           /* edges of g */
    double estimate;     /* of the triangle count of g */
} tc_stream_result;

tc_status tc_stream_estimate(tc_graph g, double d, int64_t num_samples, uint64_t seed, void* stream,
                             tc_stream_result* out);

/* Random-projection estimator (section 5.1) with Rademacher vectors: for
   l < k, x_l[i] = +1 if bit (l & 63) of
   mix64(mix64((l >> 6) << 32 | i) ^ mix64(seed ^ 0x52505F5452414345)) is 0, else -1;
   q[l] = x_l^T A^3 x_l computed exactly in int64, and *tri_est = (sum_l q[l]
   summed in 128-bit) / (6k).  q is a host array of k entries; tri_est may be
   NULL.  TC_ERR_OVERFLOW, before any sweep, if k * sum over directed edges
   (i,j) of deg_i * deg_j reaches 2^62 (q_l and their sum could then leave
   int64). */
tc_status tc_rp_trace(tc_graph g, int32_t k, uint64_t seed, void* stream, int64_t* q, double* tri_est);

/* ---- autotuner ------------------------------------------------------------ */

/* Launch parameters of the count (none of them changes T; the heavy multiplier
   changes the reported light/heavy split). */
typedef struct {
    int32_t heavy_num, heavy_den; /* heavy iff heavy_den^2 deg^2 > heavy_num^2 m */
    int32_t small_dmax;           /* anchors with out-degree <= this use one wave per item (1..128) */
    int32_t vmajor_cap;           /* pairs (u,v) whose streamed part of N+(u) is no longer than
                                     d+(v), with d+(v) <= cap, are closed from v's side; 0 closes
                                     every pair from u's side */
    int32_t blocks_per_cu;        /* persistent grid of the wave-per-item kernel (1..16) */
} tc_tuning;

/* Entries are keyed by the graph signature (n, m) and the operating point
   (sampled or not, p); calls with tc_params.use_tuned = 1 use them.
   tc_tune_get returns the stored entry, or the defaults if there is none. */
tc_status tc_tune_set(tc_graph g, double p, const tc_tuning* t);
tc_status tc_tune_get(tc_graph g, double p, tc_tuning* t);

/* Time every candidate of a fixed grid (vmajor_cap in {0, 1024},
   small_dmax in {64, 128}, and, if search_heavy, the heavy multiplier c =
   heavy_num/heavy_den in {1/4, 1/2, 1, 2}; else the multiplier of the stored
   entry or 1) on the graph sampled with (p, seed) (best of two runs each),
   store the fastest and return it in *best (may be NULL).  Candidates within
   3% of the fastest are ties, resolved towards the defaults (c = 1, then
   vmajor_cap 1024, then small_dmax 128).  Candidates whose heavy block bound
   exceeds its limit (TC_ERR_OVERFLOW) are skipped.  Counts of all candidates
   must agree; TC_ERR_DEVICE otherwise. */
tc_status tc_autotune(tc_graph g, double p, uint64_t seed, int32_t search_heavy, void* stream, tc_tuning* best);

/* Release a graph (NULL is ignored). */
void tc_graph_free(tc_graph g);

/* Message of the last failed call on this thread ("" if none). */
const char* tc_last_error(void);

/* ---- serving ------------------------------------------------------------- */

/* A server answers independent estimate requests (the sparsify-then-count
   estimate of section 3.1 for one seed, or the exact count for p = 1) with a
   fixed device memory arena and a fixed number of concurrent lanes.

   - Admission: a request needs tc_request_bytes() of the arena, the sum of the
     sizes of every device allocation its CSR build and count make.  Requests
     are released at their arrival time and admitted strictly in submission
     order, each as soon as a contiguous range of that size is free.  A request
     that needs more than the whole budget is rejected at submission
     (TC_ERR_BUDGET).  The arena is allocated once, at creation, through the
     installed allocator; nothing is allocated from the device while serving.
   - Lanes: each lane is a host worker thread with its own stream (default
     priority).  lanes = 1 serves one request at a time in arrival order.
   - Fusion (fuse_max_pairs > 0): a group of small requests is admitted as one
     reservation (the sum bound of the group's union build and count) and
     its requests complete together; reserved_bytes and peak_bytes of each
     result are the group's.
   - Results equal those of tc_build_csr + tc_estimate with the same (p, seed)
     and default tc_params, bit for bit, whatever else is in flight.
   - Thread safety: every tc_server_* call may come from any thread. */
typedef struct tc_server_s* tc_server;

typedef struct {
    int64_t budget_bytes;   /* device arena size (rounded down to 256 B); 0 admits nothing */
    int32_t lanes;          /* concurrent requests, 1..16 */
    int32_t fuse_max_pairs; /* 0: every request runs alone.  > 0: a request given as pairs with at most
                               this many pairs is fused with the released requests of the same kind
                               queued right behind it (at most 64, at most 8 x fuse_max_pairs pairs in
                               all): their graphs are built as one disjoint union and counted by one
                               pass of the kernels, each request sampled with its own (p, seed) and
                               counted into its own results, bit-identical to running it alone */
} tc_server_config;

typedef struct {
    uint64_t id;            /* caller's tag, copied to the result */
    tc_graph graph;         /* resident graph to count, or NULL to build one from the pairs below;
                               borrowed until the request's result has been polled */
    int64_t n;              /* pairs input: vertex count and pairs in host memory, borrowed until */
    int64_t num_pairs;      /*   the result has been polled (the same rules as tc_build_csr) */
    const int32_t* src;
    const int32_t* dst;
    double p;               /* keep probability in (0, 1]; 1 counts exactly */
    uint64_t seed;          /* sampling seed (unused for p = 1) */
    double arrival_s;       /* release time on the server clock (tc_server_clock); earlier = now */
} tc_request;

typedef struct {
    uint64_t id;
    int32_t status;          /* tc_status of this request */
    int32_t lane;            /* lane that ran it */
    tc_counts counts;        /* as tc_estimate's per_seed entry */
    double estimate;         /* counts.triangles / ((p*p)*p) */
    double arrival_s;        /* release time: max(arrival_s, time of submission) */
    double start_s;          /* admission time */
    double done_s;           /* result ready; latency = done_s - arrival_s */
    int64_t reserved_bytes;  /* arena bytes reserved at admission (tc_request_bytes) */
    int64_t peak_bytes;      /* high-water mark of its allocations inside the reservation */
    int64_t spilled_bytes;   /* allocations that did not fit and went to the installed allocator (0 expected) */
    char message[96];        /* error text when status != TC_OK */
} tc_result;

typedef struct {
    int64_t submitted, completed, rejected, queued, running;
    int64_t arena_bytes, arena_used, arena_peak, spilled_bytes;
} tc_server_info;

/* Arena bytes a request needs; no device work.  TC_ERR_INVALID / OVERFLOW for
   requests tc_server_submit would refuse. */
tc_status tc_request_bytes(const tc_request* r, int64_t* bytes);
/* New server; its clock starts at 0.  TC_ERR_OOM if the arena cannot be allocated. */
tc_status tc_server_create(const tc_server_config* cfg, tc_server* out);
/* Seconds on the server clock. */
tc_status tc_server_clock(tc_server s, double* now_s);
/* Queue a copy of *r (the arrays it points to stay borrowed).  Does not block. */
tc_status tc_server_submit(tc_server s, const tc_request* r);
/* Move up to cap finished results into out[], in completion order.  Waits up
   to timeout_s seconds (< 0: no limit) until at least one result is ready or
   nothing is queued or running; *got receives the number written. */
tc_status tc_server_poll(tc_server s, tc_result* out, int32_t cap, double timeout_s, int32_t* got);
tc_status tc_server_stats(tc_server s, tc_server_info* out);
/* Wait for every submitted request, then release the server (NULL is
   ignored).  Results not yet polled are discarded. */
void tc_server_destroy(tc_server s);

/* ---- measurement hooks --------------------------------------------------- */

/* When enabled, every kernel launch is bracketed by HIP events on its stream
   and its duration accumulated under the kernel's name. */
tc_status tc_profile_enable(int32_t on);
/* Restrict profiling to the kernels named in a comma-separated list (NULL or
   "" = every kernel). */
tc_status tc_profile_select(const char* names);
tc_status tc_profile_reset(void);
/* Accumulated milliseconds and launch count of a named kernel (0 if unseen). */
tc_status tc_profile_read(const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
