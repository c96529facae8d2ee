/*
 * tc.h - exact triangle counting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libtc.so. It implements the data-parallel hot path of Tom and
 * Karypis, "A 2D Parallel Triangle Counting Algorithm for Distributed-Memory
 * Architectures" (ICPP 2019): a simple undirected graph is reordered by
 * non-decreasing degree, split into its upper triangular part U, and for every
 * nonzero (i, j) of U the map-based intersection of Section 3.1 counts
 * c(i, j) = |Adj>(i) & Adj>(j)| (Eq. 1), reduced to the exact total of Eq. 2.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers on the current HIP device (for
 *    example the data_ptr() of a torch tensor on a ROCm device). Host pointers
 *    have no prefix.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *    is enqueued on it and outputs are written asynchronously; the caller
 *    synchronises the stream before reading them, and keeps inputs alive until
 *    then. Only tc_preprocess and the batch/server set-up calls synchronise.
 *  - No C++ exception crosses the ABI. On failure an entry point returns a
 *    non-zero tc_status, leaves its outputs unspecified, allocates nothing
 *    that outlives the call, and tc_last_error() describes the failure (per
 *    host thread).
 *  - A tc_graph is immutable after tc_preprocess, so calls on one graph from
 *    several streams or threads may run concurrently.
 *  - Device temporaries come from a per-device cache inside the library
 *    (tc_release_cached_memory returns it); running out of device memory in
 *    any call is TC_ENOMEM and leaves the library usable.
 *  - Environment: TC_SORT_WIDE_WORDS=1 makes every internal radix sort use
 *    the 64-bit look-back words that sorts of 2^31 keys or more take (a test
 *    switch; results are identical).
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TC_OK = 0,
  TC_EINVAL = 1,     /* bad argument (null pointer, n <= 0, id out of [0, n), bad mode) */
  TC_ENOMEM = 2,     /* device or host allocation failed */
  TC_EDEVICE = 3,    /* a HIP runtime call failed */
  TC_EOVERFLOW = 4,  /* a size exceeds the library's index widths (see tc_preprocess) */
  TC_EBUSY = 5,      /* server: no capacity right now */
  TC_ECANCELED = 6   /* server: request was cancelled */
} tc_status;

/* Opaque, device-resident preprocessed graph. */
typedef struct tc_graph tc_graph;

/* Per-edge support modes (tc_edge_support). */
enum {
  TC_SUPPORT_FULL = 0,     /* triangles containing the edge; sums to 3T */
  TC_SUPPORT_ORIENTED = 1  /* c(i, j) of Eq. 1 for the nonzero (i, j) of U; sums to T */
};

/* Summary of a preprocessed graph (tc_graph_info). */
typedef struct {
  int64_t n;               /* vertices */
  int64_t m_raw;           /* input pairs */
  int64_t m;               /* edges of the simple graph = nonzeros of U */
  int64_t wedges_plus;     /* W+ = sum over rows a of C(|U_a|, 2) */
  int64_t probes;          /* hash lookups tc_count performs: W+ without the
                              intersections whose hashed row is empty */
  int64_t tasks;           /* nonzeros (i, j) of U with at least one probe */
  int64_t max_out_degree;  /* max |U_a| */
  int64_t device_bytes;    /* device memory held by the handle */
} tc_info;

/*
 * tc_preprocess - build the device-resident graph (Section 5.3 and Section 2).
 *
 * Input: m_raw pairs (d_src[e], d_dst[e]), int32 vertex ids in [0, n), device
 * memory owned by the caller. Duplicates, both orientations and self loops are
 * legal: the pairs are reduced to the simple undirected graph (Section 6.1).
 * Vertices are ranked by non-decreasing degree, ties by original id (the
 * counting-sort relabelling of Section 5.3 with a fixed tie order); each edge
 * {u, v} becomes the nonzero (min rank, max rank) of U (the upper/lower split
 * of Section 5.3 by global position); rows of U are sorted ascending (which
 * Section 5.2's pruning of needless intersections relies on).
 *
 * Output: *out receives a new handle (free with tc_graph_free). The handle
 * owns its device memory. The call synchronises `stream` once it has read
 * back the sizes.
 *
 * Errors: TC_EINVAL for null pointers, n < 1, m_raw < 0 or an id outside
 * [0, n) (no handle is returned); TC_EOVERFLOW if m_raw >= 2^32 - 1 or the
 * simple graph has 2^32 - 256 or more edges (positions in U are 32-bit);
 * TC_ENOMEM / TC_EDEVICE on allocation or runtime failure. Graphs of 2^30
 * edges or more are counted with 64-bit probe addresses; batch plans and one
 * rank's block take probe sides below 2^30 entries (TC_EOVERFLOW otherwise).
 */
tc_status tc_preprocess(const int32_t* d_src, const int32_t* d_dst, int64_t m_raw, int32_t n,
                        void* stream, tc_graph** out);

/* tc_graph_info - sizes and work counts of a handle (host struct *out). */
tc_status tc_graph_info(const tc_graph* g, tc_info* out);

/*
 * tc_graph_export - copy U and the relabelling to caller buffers:
 * d_row_ptr int64[n + 1], d_col int32[m] (rows sorted ascending, every entry
 * greater than its row), d_perm int32[n] with d_perm[original id] = rank.
 * Any of the three may be NULL to skip it. Asynchronous on `stream`.
 */
tc_status tc_graph_export(const tc_graph* g, int64_t* d_row_ptr, int32_t* d_col, int32_t* d_perm,
                          void* stream);

/*
 * tc_count - exact number of triangles, T of Eq. 2, written to the device
 * int64 *d_count. Runs the <j,i,k> map-based intersection of Section 3.1: for
 * every row j of U that some task needs, U_j is hashed in LDS (direct
 * low-bit addressing with linear probing: Section 5.2's change to the
 * hashing routine), and for each nonzero (i, j) the entries of U_i after j are looked
 * up in it. Asynchronous on `stream`; allocates nothing.
 */
tc_status tc_count(const tc_graph* g, int64_t* d_count, void* stream);

/*
 * tc_edge_support - per-edge triangle values for the m nonzeros of U, in the
 * order of tc_graph_export's d_col (row-major). mode TC_SUPPORT_FULL: the
 * number of triangles containing the edge (sum = 3T); TC_SUPPORT_ORIENTED:
 * c(i, j) of Eq. 1 (sum = T). d_support is int32[m] (caller-owned device
 * memory, overwritten); d_count (nullable) receives T. Asynchronous; allocates
 * nothing. TC_EINVAL for an unknown mode or a null d_support with m > 0.
 */
tc_status tc_edge_support(const tc_graph* g, int mode, int32_t* d_support, int64_t* d_count,
                          void* stream);

/*
 * tc_block_count - one rank's share of the 2D cyclic decomposition of
 * Section 5.1 at its real shape, for a q x q grid (1 <= q <= 64), rank (x, y)
 * with 0 <= x, y < q. Under the C[L] task convention of Section 5.1 the rank
 * owns the tasks (i, j) of U with j % q == x and i % q == y; it hashes the rows
 * j == x (mod q) and probes the rows i == y (mod q), stored in a rank-local CSR
 * indexed by v / q (the transformed index of Section 5.1) with a list of
 * non-empty rows (the doubly sparse traversal of Section 5.2).
 * d_count (int64) receives the triangles its tasks close; d_per_shift
 * (nullable, int64[q]) receives, for each shift z of Eq. 5, the part whose
 * closing vertex k has k % q == (x + y + z) % q. The rank-local structures are
 * built on `stream` in memory the call allocates and frees (the call
 * synchronises `stream`).
 */
tc_status tc_block_count(const tc_graph* g, int32_t q, int32_t x, int32_t y, int64_t* d_count,
                         int64_t* d_per_shift, void* stream);

/* ---- ablations of the paper's optimizations (Section 7.3) ------------------ */

/* Flags of tc_graph_variant (combinable). */
enum {
  TC_VARIANT_IJK = 1,      /* <i,j,k> enumeration: for every nonzero (i, j) of U, U_i is hashed and
                              all of U_j is looked up (instead of hashing U_j and looking up
                              U_i's entries after j) */
  TC_VARIANT_NO_DCSR = 2,  /* no doubly sparse traversal (Section 5.2): every hashed row is
                              visited, also rows without work, and intersections whose hashed
                              list is empty are kept */
  TC_VARIANT_MUL_HASH = 4  /* no direct-AND addressing (Section 5.2's hashing
                              change undone): every table is addressed by a multiplicative hash
                              (top bits of k * 0x9E3779B1) with linear probing */
};

/*
 * tc_graph_variant - a graph handle that counts g's triangles with some of
 * the optimizations of Section 5.2 undone, for the measurements of Section
 * 7.3 (runtime gained by each). The new handle shares g's U (g must outlive
 * it; free it with tc_graph_free) and has a work set of its own: tc_count on
 * it gives the same T; tc_graph_info reports its probes and tasks (with
 * TC_VARIANT_IJK, probes = the sum of |U_j| over the nonzeros (i, j)).
 * Only tc_count, tc_graph_info, tc_graph_class_stats, tc_graph_export and
 * tc_graph_free accept a variant (others: TC_EINVAL). Synchronises
 * `stream`. TC_EINVAL for unknown flags.
 */
tc_status tc_graph_variant(const tc_graph* g, int32_t flags, void* stream, tc_graph** out);

/* ---- uses of the counts (Section 1: clustering coefficients, k-truss) ------- */

/*
 * tc_vertex_triangles - number of triangles through every vertex, indexed by
 * original vertex id: d_tri is device int64[n] (caller-owned, overwritten).
 * Computed from the per-edge support of TC_SUPPORT_FULL: the two edges a
 * triangle has at v each count it once, so t(v) is half their sum. The sum
 * over all vertices is 3T. Asynchronous on `stream` except for one
 * synchronisation after the internal column sort; allocates temporaries
 * (the support array and U's column lists: about 16 m + 8 n bytes).
 */
tc_status tc_vertex_triangles(const tc_graph* g, int64_t* d_tri, void* stream);

/*
 * tc_clustering - local clustering coefficients (Section 1 names them as a
 * use of triangle counts): d_cc[u] = t(u) / C(d(u), 2) as a double (0 when
 * the degree d(u) < 2), indexed by original vertex id; each is one correctly
 * rounded division of two exact integers. d_tri (nullable) receives t(u) as
 * tc_vertex_triangles does; d_sums (nullable, device int64[2]) receives
 * sum_u t(u) = 3T and sum_u C(d(u), 2), the numerator and denominator of the
 * transitivity. At least one output is required (TC_EINVAL otherwise).
 * Same synchronisation and temporaries as tc_vertex_triangles.
 */
tc_status tc_clustering(const tc_graph* g, double* d_cc, int64_t* d_tri, int64_t* d_sums, void* stream);

/*
 * tc_transitivity - global clustering coefficient 3T / sum_u C(d(u), 2)
 * (0 if no vertex has two neighbours) into the host double *out.
 * Synchronises `stream`.
 */
tc_status tc_transitivity(const tc_graph* g, double* out, void* stream);

/*
 * tc_truss - trussness of every edge (Section 1 names the k-truss as a use
 * of per-edge triangle counts). The k-truss is the largest subgraph in which
 * every edge lies in at least k - 2 of the subgraph's triangles; an edge's
 * trussness is the largest k whose k-truss contains it (>= 2). d_tau is
 * device int32[m] in U order (the order of tc_graph_export's d_col);
 * *kmax (host, nullable) receives the largest trussness (0 without edges).
 * Computed by peeling from the TC_SUPPORT_FULL support: each round removes
 * the edges whose support in the remaining graph is below k - 2 and takes
 * the triangles they close out of their other edges' support. Synchronises
 * `stream` once per round; allocates temporaries (about 28 m + 8 n bytes).
 * TC_EOVERFLOW for 2^31 or more edges.
 */
tc_status tc_truss(const tc_graph* g, int32_t* d_tau, int32_t* kmax, void* stream);

/*
 * tc_block_stats - the work of rank (x, y) of the q x q grid of tc_block_count
 * (Section 7.2 measures its balance across ranks and shifts, Table
 * "r_l_imb", and how the number of intersections grows with the number of
 * ranks, Table "opcount"). d_out is device int64[2 + 2 q]:
 *   [0]         tasks: nonzeros (i, j) of the rank whose row i has entries
 *               after j and whose U_j is not empty;
 *   [1]         probes: lookups of those tasks (entries of U_i after j);
 *   [2 + z]     the probes whose closing vertex k falls in shift z's class,
 *               (k - x - y) mod q == z (Eq. 5);
 *   [2 + q + z] the intersections shift z performs when the shifts run one
 *               by one: tasks whose probe list and U_j both hold an entry of
 *               that class.
 * Same argument rules as tc_block_count; allocates temporaries; synchronises
 * `stream` (rank extraction).
 */
tc_status tc_block_stats(const tc_graph* g, int32_t q, int32_t x, int32_t y, int64_t* d_out, void* stream);

/* ---- batched counting ---------------------------------------------------- */

/* Opaque plan for counting a fixed set of graphs in one persistent launch. */
typedef struct tc_batch tc_batch;

/*
 * tc_batch_create - plan one persistent launch over `num_graphs` handles
 * (host array of handles; graphs may repeat). The work units of every graph
 * (the packs and item groups its own tc_count would launch) are merged into
 * one device queue, by default largest first (longest-processing-time order).
 * tuning_json is a flat JSON object choosing the schedule (NULL or "": the
 * tuning table's "batch" entry for this many edges, else the defaults):
 *   "blocks_per_cu" (int, 0 = as many as LDS allows), "lds_cap_log2" (int in
 *   [6, 14]: item rows whose table exceeds 2^cap slots are looked up in HBM
 *   instead of LDS), "order" ("lpt" | "input"), "graph" (1 = launch through a
 *   captured HIP graph, 0 = plain launches), "chunk" (int, units taken per
 *   queue atomic, default 1, 0 = about 16 atomics per work-group), and the
 *   row-bucket thresholds (see tc_graph_retune; when any is named, the
 *   unnamed ones take their defaults): graphs cut by others are
 *   counted through retuned copies the plan builds and holds (about one
 *   work-decomposition build per distinct graph);
 *   tc_batch_autotune's output is accepted as is. Unknown keys: TC_EINVAL.
 *   The handles must outlive the plan. Synchronises `stream`.
 */
tc_status tc_batch_create(const tc_graph* const* graphs, int32_t num_graphs,
                          const char* tuning_json, void* stream, tc_batch** out);

/*
 * tc_batch_count - per-graph exact counts into the device int64[num_graphs]
 * d_counts (same order as the handles), equal to tc_count's. Two kernels: one
 * clears the counts and the queue counter, one persistent launch drains the
 * queue; with "graph": 1 they run as one HIP graph (captured on the first call
 * for a given d_counts), and when `stream` is itself being captured they are
 * recorded into the caller's graph. Asynchronous. Calls that overlap on one
 * plan race (the plan holds the queue counter).
 */
tc_status tc_batch_count(tc_batch* plan, int64_t* d_counts, void* stream);

void tc_batch_free(tc_batch* plan);

/* The plan's schedule and size as JSON (units, grid, LDS bytes, ...) into the
 * host buffer out[cap]; TC_EINVAL if it does not fit. */
tc_status tc_batch_describe(const tc_batch* plan, char* out, size_t cap);

/* One-shot convenience: create a plan, count, free it (synchronises). */
tc_status tc_count_batched(const tc_graph* const* graphs, int32_t num_graphs, int64_t* d_counts,
                           const char* tuning_json, void* stream);

/*
 * tc_count_batched_noalloc - tc_count_batched for callers that cannot
 * allocate device memory (code that runs while a HIP graph is being captured,
 * tight serving loops, harnesses that forbid hipMalloc). Same per-graph
 * counts as tc_count_batched (d_counts: device int64[num_graphs], handle
 * order), with the default schedule in graph order. Everything else the call
 * needs - the queue counter, the graphs' kernel arguments and unit lists -
 * lives in a fixed 64 MiB device array of the library (one per GPU, held
 * until the process ends); the call allocates no device memory and frees
 * none. A batch that needs more of it than 64 MiB (about 2 million work
 * units: graphs x their packs and item groups) fails with TC_EOVERFLOW and a
 * message naming the size. Calls on one GPU share that array: calls that
 * overlap on one GPU (concurrent streams or threads) race and give wrong
 * counts. Synchronises `stream`.
 */
tc_status tc_count_batched_noalloc(const tc_graph* const* graphs, int32_t num_graphs, int64_t* d_counts,
                                   void* stream);

/*
 * tc_batch_autotune - time candidate schedules on these graphs: LDS caps that
 * change the plan x unit orders x blocks per CU, then units per queue atomic,
 * then the row-bucket thresholds one at a time (each candidate counting
 * retuned copies of the graphs, tc_graph_retune; since a plan with other
 * thresholds builds such copies when it is created, they are kept only if they
 * beat the graphs' own by 2% or more). Writes {"key": ..., "best":
 * {...}, "plan": {...}, "candidates": [...]} into the host buffer
 * out_json[cap]; "best" (schedule and, if they won, thresholds) can be passed
 * to tc_batch_create and is stored in the tuning table under "key", the
 * entry for batches of this many edges. Synchronises `stream`; allocates and
 * frees its own scratch.
 */
tc_status tc_batch_autotune(const tc_graph* const* graphs, int32_t num_graphs, void* stream,
                            char* out_json, size_t cap);

/* ---- row-bucket thresholds and the tuning table ------------------------------
 *
 * The work of a graph is cut into classes (tc_graph_class_stats) by five
 * thresholds, a flat JSON object of integers:
 *   "heavy_min"   (0 .. 2^24, default 32768): rows b with fewer probes than
 *                 this, and tables of at most 2^10 slots, are packed several
 *                 to a work-group; the others get work-groups of their own;
 *   "pack_target" (1024 .. 2^24, default 65536): probes per pack (plus one
 *                 row's);
 *   "pack_slots"  (1024 .. 16384, default 4096): LDS table slots per pack
 *                 (plus one row's table);
 *   "wave_chunk"  (1024 .. 32767, default 32767): probes per wave item of a
 *                 row with work-groups of its own, at most;
 *   "min_groups"  (0 .. 2^22, default 16384): a class of such rows whose
 *                 probes would fill fewer work-groups than this gets smaller
 *                 wave items (down to 1024 probes) so that it fills the GPU;
 *                 a class too small to fill them even then keeps wave_chunk
 *                 (few large units suit a batch of many small graphs).
 * They change how the work is scheduled, never a count. Graphs take theirs
 * from the tuning table when tc_preprocess builds them (the defaults when the
 * table has no entry for their size).
 *
 * The tuning table maps keys "<arch>/<CUs>cu/<kind>_e<k>" to flat JSON
 * objects: kind "graph" holds thresholds for graphs of 2^k .. 2^(k+1) - 1
 * edges, kind "batch" a tc_batch_create schedule for batches of that many
 * edges in total. A lookup takes the entry of the same arch, CU count and
 * kind whose k is nearest, at most two classes away (ties: the smaller). The
 * table starts empty, is read from the file TC_TUNING_FILE names (at the
 * first lookup; a malformed or unreadable file is an error of the call that
 * triggered it), and is filled by tc_tuning_load/set and the autotuners.
 */

/* Merge the entries of a tuning file (one JSON object of key: flat object)
 * into the table. TC_EINVAL: unreadable or malformed (nothing merged). */
tc_status tc_tuning_load(const char* path);
/* Write the whole table to `path` (through a temporary file and a rename). */
tc_status tc_tuning_save(const char* path);
/* The entry a lookup of `key` finds (exact, else the nearest class) into
 * out[cap] as text; "" if none. TC_EINVAL if it does not fit. */
tc_status tc_tuning_get(const char* key, char* out, size_t cap);
/* Set the entry of `key` to the flat JSON object `json` (NULL: remove it). */
tc_status tc_tuning_set(const char* key, const char* json);
/* The key of the current device for kind "graph" or "batch" and `edges`. */
tc_status tc_tuning_key(const char* kind, int64_t edges, char* out, size_t cap);

/*
 * tc_graph_retune - a new handle counting the same graph with its work cut by
 * other thresholds (params_json: any of the five keys; the others keep g's).
 * It shares g's U (g must outlive it), owns only its work decomposition, and
 * is a plain graph for every call. Synchronises `stream`.
 */
tc_status tc_graph_retune(const tc_graph* g, const char* params_json, void* stream, tc_graph** out);

/* The thresholds g's work was cut with, as a flat JSON object, into out[cap]. */
tc_status tc_graph_work_params(const tc_graph* g, char* out, size_t cap);

/*
 * tc_graph_autotune - time tc_count on g under candidate thresholds (each
 * parameter in turn over a few values, the others held at the best so far),
 * store the best in the tuning table under the "graph" key of g's size, so
 * that later tc_preprocess calls for graphs of that size use it, and write
 * {"key": ..., "best": {...}, "candidates": [...]} into out_json[cap].
 * Synchronises `stream`.
 */
tc_status tc_graph_autotune(const tc_graph* g, void* stream, char* out_json, size_t cap);

/* ---- served form: a request loop with continuous batching ------------------- */

/*
 * A server owns a scheduler thread and a pool of preprocessing threads on the
 * device current at tc_server_create. Requests (count or support of one
 * graph, given as a host edge list) are admitted in arrival order while the
 * in-flight requests stay within `max_slots` and their estimated device
 * footprint (edge list, preprocessing temporaries, the graph, the support
 * array) fits `hbm_budget_bytes` together with the cached graphs; cached
 * graphs no request uses are evicted least recently used first when room is
 * needed. Admitted requests are preprocessed concurrently on the pool's
 * streams; on every scheduler tick all requests whose graph is ready run in
 * one persistent launch per operation (tc_batch's kernel and work units), so
 * requests that arrive while a tick runs are preprocessed meanwhile and join
 * the next tick. Results are the same integers as tc_count/tc_edge_support.
 * A request with a non-zero graph_key keeps its graph cached on the device:
 * later requests with that key skip preprocessing (their edge list may be
 * NULL while the key is resident).
 */
typedef struct tc_server tc_server;

enum { TC_REQ_COUNT = 0, TC_REQ_SUPPORT_FULL = 1, TC_REQ_SUPPORT_ORIENTED = 2 };

typedef struct {
  int32_t op;           /* TC_REQ_* */
  int32_t n;            /* vertices (ids in [0, n)) */
  int64_t m_raw;        /* pairs in src/dst (support ops: also the capacity of support_out) */
  const int32_t* src;   /* host arrays, kept alive by the caller until the request is done */
  const int32_t* dst;
  uint64_t graph_key;   /* 0: not cached; else the caller's name for this graph */
  int32_t* support_out; /* support ops: host int32[m_raw]; receives the first m entries (U order) */
} tc_request;

typedef struct {
  tc_status status;     /* TC_OK, or the request's failure (TC_ECANCELED if cancelled) */
  int32_t cache_hit;    /* 1 if the graph was resident (no preprocessing) */
  int64_t count;        /* triangles */
  int64_t m;            /* edges of the simple graph (entries written to support_out) */
  double t_submit;      /* seconds on the server's clock: submitted, admitted, */
  double t_admit;       /*   graph ready, result visible to the host */
  double t_ready;
  double t_done;
} tc_result;

/* options_json (nullable), flat object: "prep_threads" (default: half the
 * host's threads, 1 .. 8), "lds_cap_log2" and "blocks_per_cu" (the batch
 * schedule of every tick), "lpt" (1: a tick's units largest first, which
 * costs a sort and a synchronisation of the tick stream; default 0: request
 * order), "ticks" (ticks in flight, 1 or 2; default 1; with 2, a tick of at
 * least two ready requests is planned and launched while one runs, both on
 * the tick stream). A tick
 * takes the ready requests whose share of its batch plans (kernel arguments
 * and work units) still fits the budget, at least one. */
tc_status tc_server_create(int64_t hbm_budget_bytes, int32_t max_slots, const char* options_json,
                           tc_server** out);
/* Queue a request; *ticket identifies it. TC_EINVAL for a malformed request. */
tc_status tc_server_submit(tc_server* s, const tc_request* req, int64_t* ticket);
/* Result of a ticket: TC_OK and *out filled (the ticket is consumed) once it is
 * done; TC_EBUSY if not done yet and wait == 0 (wait != 0 blocks until done);
 * TC_EINVAL for an unknown ticket. */
tc_status tc_server_poll(tc_server* s, int64_t ticket, int32_t wait, tc_result* out);
/* Cancel a request not yet admitted (its result: TC_ECANCELED); TC_EBUSY if it
 * is already admitted. */
tc_status tc_server_cancel(tc_server* s, int64_t ticket);
/* Counters (requests, ticks, cache hits, evictions, peak reserved bytes, ...)
 * as JSON into the host buffer out[cap]. */
tc_status tc_server_stats(tc_server* s, char* out, size_t cap);
/* Stop the threads (pending requests are cancelled, admitted ones finish) and
 * free every device allocation of the server. */
void tc_server_destroy(tc_server* s);

/* ---- work classes and phase timers (profiling) ------------------------------ */

/* tc_count splits the hashed rows j into work classes, one kernel launch each:
 * 0 pack_small / 1 pack_large - light rows packed, up to 256 per work-group,
 *   their tables built together;
 * 2 wg_small / 3 wg_large / 4 wg_huge / 5 wg_giant - heavy rows, a
 *   work-group's four waves share one LDS table of the row (at most 1024 /
 *   4096 / 8192 / 16384 slots); 6 global - rows of more than 8192 entries,
 *   looked up by binary search in HBM. */
#define TC_NUM_CLASSES 7

typedef struct {
  int64_t workgroups;   /* work-groups of the class's launch */
  int64_t rows;         /* hashed rows j in the class */
  int64_t table_keys;   /* sum of |U_j| over those rows (table build reads) */
  int64_t tasks;        /* nonzeros (i, j) whose probes the class performs */
  int64_t probes;       /* lookups the class performs */
  int64_t table_slots;  /* largest table of the class (slots) */
} tc_class_stats;

/* Per-class work of a graph (host array of TC_NUM_CLASSES entries). */
tc_status tc_graph_class_stats(const tc_graph* g, tc_class_stats* out);
/* Name of a class ("pack_small", ...) or NULL. */
const char* tc_class_name(int32_t cls);

/* Phase timer: while attached to the calling host thread, every kernel the
 * library launches from that thread is bracketed by two HIP events recorded
 * on the launch's stream and tagged with the kernel's name (count kernels as
 * "count:<class>", "support_full:<class>", ...). Up to `capacity` launches are
 * recorded; later ones are counted as dropped. */
typedef struct tc_timer tc_timer;
tc_status tc_timer_create(int32_t capacity, tc_timer** out);
/* Attach `t` to the calling thread (NULL detaches). */
tc_status tc_timer_attach(tc_timer* t);
/* Waits for the recorded events and writes a JSON object
 * {"<name>": {"launches": n, "total_ms": x, "avg_ms": y, "min_ms": a,
 *  "max_ms": b}, ..., "_dropped": d} into buf (NUL-terminated; TC_EINVAL if
 * it does not fit). */
tc_status tc_timer_summary(tc_timer* t, char* buf, int64_t buf_bytes);
/* Forget recorded launches (events are reused). */
tc_status tc_timer_reset(tc_timer* t);
void tc_timer_free(tc_timer* t);

/* ---- device memory --------------------------------------------------------- */

/* The library keeps device blocks it has freed (graph arrays, temporaries)
 * for reuse instead of returning them to the runtime: hipFree can block the
 * host for milliseconds. Cached free bytes are bounded by a quarter of the
 * device's memory and are released when an allocation runs out of memory.
 * tc_release_cached_memory returns every cached block of every device to the
 * runtime (waits for pending work on them). */
void tc_release_cached_memory(void);
/* Bytes handed out, cached free, and the peak handed out, on the current device. */
tc_status tc_memory_stats(int64_t* in_use_bytes, int64_t* cached_bytes, int64_t* peak_bytes);

/* ---- misc ----------------------------------------------------------------- */

void tc_graph_free(tc_graph* g);
const char* tc_status_string(tc_status s);
/* Message of the last failure on this host thread ("" if none). */
const char* tc_last_error(void);
/* Library version string. */
const char* tc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
