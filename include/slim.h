/*
 * slim.h -- C ABI of libslim.so: Slim Graph's Triangle p-1-Reduction and
 * uniform edge sampling on AMD Instinct MI355X (gfx950).
 *
 * Paper: M. Besta et al., "Slim Graph: Practical Lossy Graph Compression for
 * Approximate Graph Processing, Storage, and Analytics", SC'19
 * (arXiv 1912.08950).
 *
 * Conventions
 *   - Every call returns SLIM_OK (0) or a negative SLIM_E* code; the detail
 *     is in slim_last_error() (thread-local, valid until the next call on
 *     the same thread).  No C++ exception crosses this interface.
 *   - "d_" pointers are device (HBM) pointers owned by the caller; the
 *     library never frees caller memory.  Compute calls allocate no device
 *     memory: their scratch is a caller workspace.  (A batch holds a HIP
 *     graph and a small pinned host buffer of its own.)
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Compute calls only enqueue work on it and return; outputs and stats
 *     are valid once the stream has been synchronised.  Calls on one stream
 *     are ordered; calls that share a workspace must not overlap.
 *   - Graphs are undirected and simple, stored as a symmetric CSR:
 *     row_off: int64[n+1] with row_off[0] = 0 and row_off[n] = nnz;
 *     col: uint32[nnz], each row strictly increasing (sorted, no duplicate),
 *     no self-loop, and (u,v) present iff (v,u) present.  nnz = 2m.  Vertex
 *     ids are uint32, so n <= 2^32 - 1; the DAG edge ids are uint32, so
 *     m <= 2^32 - 1.
 *   - Results are deterministic functions of (graph, p, seed): bit-exact
 *     across runs, launch shapes and devices.
 */
#ifndef SLIM_H_
#define SLIM_H_

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SLIM_API __attribute__((visibility("default")))
#else
#define SLIM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ errors */
#define SLIM_OK 0
#define SLIM_EINVAL (-1)  /* bad argument or input graph violating the contract */
#define SLIM_ENOMEM (-2)  /* caller workspace smaller than slim_workspace_size() */
#define SLIM_EBUDGET (-3) /* request larger than a configured memory budget */
#define SLIM_EDEVICE (-4) /* HIP runtime error (launch, sync, device query) */
#define SLIM_EAGAIN (-5)  /* not ready yet (non-blocking queries) */

/* Message for the last failing call on this thread ("" if none). */
SLIM_API const char* slim_last_error(void);
/* Static name of an error code. */
SLIM_API const char* slim_strerror(int code);
/* Library version as 10000*major + 100*minor + patch. */
SLIM_API int slim_version(void);

/* ------------------------------------------------------------ graphs */
typedef struct slim_graph slim_graph_t; /* opaque, library-owned */

#define SLIM_VALIDATE 1u /* slim_load_csr flag: check the CSR contract on the device */

/*
 * Wrap a device-resident CSR (the graph model of section 2: G = (V,E),
 * |V| = n, |E| = m, kept as adjacency arrays as the paper's mappings do).
 * The arrays are borrowed: they must stay alive and unchanged until
 * slim_graph_free().  With SLIM_VALIDATE the contract above is checked by a
 * device kernel (sortedness, no self-loop, ids < n, offsets, symmetry); this
 * synchronises `stream` and returns SLIM_EINVAL naming the first violation.
 * Without it the call enqueues nothing.  Errors: SLIM_EINVAL (null
 * pointers, n or m out of range, odd nnz, invalid CSR), SLIM_EDEVICE.
 */
SLIM_API int slim_load_csr(const int64_t* d_row_off, const uint32_t* d_col, uint64_t n, uint64_t nnz,
                  uint32_t flags, void* stream, slim_graph_t** out);

/* Release a graph handle (NULL is ignored). */
SLIM_API void slim_graph_free(slim_graph_t* g);

/* ------------------------------------------------- compression calls */
#define SLIM_OP_TR 1   /* Triangle p-1-Reduction */
#define SLIM_OP_ES 2   /* uniform edge sampling */
#define SLIM_OP_TR2 3  /* Triangle p-2-Reduction */
#define SLIM_OP_MCTR 4 /* Min-Count Triangle p-1-Reduction */
#define SLIM_OP_SPECTRAL 5 /* spectral sparsification (p carries upsilon) */
#define SLIM_OP_EOTR 6 /* Edge-Once Triangle p-1-Reduction */

/* Device workspace (bytes) that `op` needs on graph `g`. */
SLIM_API int slim_workspace_size(const slim_graph_t* g, int op, uint64_t* bytes);

/* Per-call counters, written to device memory by the call. */
typedef struct slim_stats {
  uint64_t n;         /* vertices (unchanged by both operations) */
  uint64_t m_in;      /* undirected input edges, nnz/2 */
  uint64_t triangles; /* T: triangles of the input graph (TR; 0 for ES) */
  uint64_t selected;  /* triangles selected for reduction (TR; 0 for ES) */
  uint64_t deleted;   /* undirected edges removed */
  uint64_t m_out;     /* undirected output edges = m_in - deleted */
} slim_stats_t;

/*
 * Triangle p-1-Reduction (section 4.3; kernel `p-1-reduction` of the kernel
 * listing): each triangle {a<b<c} of the INPUT graph is selected
 * independently with probability p; a selected triangle deletes one of its
 * three edges, chosen uniformly.  All triangles are decided on the input
 * graph in one pass; deleting an edge twice is the same as once.
 *
 *   p      probability that a triangle is selected, 0 <= p <= 1
 *          (NaN or outside -> SLIM_EINVAL).  p = 0 copies the graph;
 *          p = 1 removes every input triangle.
 *   seed   64-bit key of the counter-based random source: Philox4x32-10
 *          (Salmon et al., SC'11) with key (seed mod 2^32, seed div 2^32) and
 *          counter (a,b,c,0); the triangle is selected iff word 0 of the
 *          output is < floor(p*2^32) (2^32 when p = 1), and deletes edge
 *          k = floor(word1 * 3 / 2^32) of ({a,b}, {a,c}, {b,c}).
 *   d_ws   device workspace of at least slim_workspace_size(g, SLIM_OP_TR)
 *          bytes, 256-byte aligned (ws_bytes smaller -> SLIM_ENOMEM).
 *   d_out_row_off  int64[n+1]: output CSR offsets (same n, same ids).
 *   d_out_col      uint32[nnz] capacity: output CSR columns; entries past
 *                  d_out_row_off[n] are left unspecified.
 *   d_stats  optional (may be NULL) device slim_stats_t.
 * The output is again a symmetric CSR with sorted rows.
 */
SLIM_API int slim_triangle_reduce(const slim_graph_t* g, double p, uint64_t seed, void* d_ws,
                         uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                         slim_stats_t* d_stats, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, output and errors as slim_triangle_reduce, with the workspace
 * taken from a fixed device array of SLIM_NOALLOC_WS_BYTES (512 MiB) that
 * the library holds on every GPU it runs on until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); its first call on a device looks up that array's address there.
 * A graph whose slim_workspace_size(g, SLIM_OP_TR) exceeds the array ->
 * SLIM_ENOMEM (R-MAT scale 20, about 2^25 CSR entries, fits; scale 21 does
 * not).  The graph must live on the current device (else SLIM_EINVAL).
 * All calls on one GPU share that GPU's array: calls that overlap on one
 * GPU (on different streams or threads) race and must be serialised by the
 * caller; every call clears what it needs cleared itself.
 */
#define SLIM_NOALLOC_WS_BYTES (512ull << 20)
SLIM_API int slim_triangle_reduce_noalloc(const slim_graph_t* g, double p, uint64_t seed,
                                          int64_t* d_out_row_off, uint32_t* d_out_col,
                                          slim_stats_t* d_stats, void* stream);

/*
 * Uniform edge sampling (section 4.2.2; kernel `random_uniform`): each
 * undirected edge {a<b} is deleted independently with probability p
 * (Table `tab:theory-schemes`: (1-p)m edges remain), decided once from
 * Philox4x32-10 with counter (a,b,0,1): deleted iff word 0 < floor(p*2^32)
 * (2^32 when p = 1).  Arguments, layout and errors as slim_triangle_reduce
 * with op SLIM_OP_ES.
 */
SLIM_API int slim_edge_sample(const slim_graph_t* g, double p, uint64_t seed, void* d_ws,
                     uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                     slim_stats_t* d_stats, void* stream);

/*
 * Any of the operations above by op code, with the arguments, layout and
 * errors of slim_triangle_reduce (workspace: slim_workspace_size(g, op)).
 *   SLIM_OP_TR    as slim_triangle_reduce.
 *   SLIM_OP_ES    as slim_edge_sample.
 *   SLIM_OP_TR2   Triangle p-2-Reduction (section 4.3, x = 2): a selected
 *                 triangle loses two edges chosen uniformly -- every edge
 *                 except k of slim_triangle_reduce's draw.
 *   SLIM_OP_MCTR  Min-Count Triangle p-1-Reduction (section 4.3): t_e =
 *                 triangles of the input graph on edge e; a selected
 *                 triangle loses its edge of smallest t_e; among tied edges
 *                 (in the order {a,b}, {a,c}, {b,c}) the one at index
 *                 floor(word1 * ties / 2^32).
 *   SLIM_OP_SPECTRAL  as slim_spectral_sparsify with upsilon = p (any value
 *                 >= 0) and no weights.
 *   SLIM_OP_EOTR  Edge-Once Triangle p-1-Reduction (section 4.3; the
 *                 conditions of section 6.2: an edge is considered for
 *                 deletion at most once, a considered triangle loses one
 *                 edge).  Triangles are selected as by slim_triangle_reduce
 *                 and ordered by priority (word 2 of the same Philox
 *                 output, then the ids a, b, c).  In that order a selected
 *                 triangle is considered iff none of its three edges is
 *                 considered yet; it then deletes edge k and its three edges
 *                 become considered.  The output is the same as that
 *                 sequential walk: the GPU reaches it in rounds, each
 *                 considering every selected triangle that is first in
 *                 priority among the undecided ones sharing an edge with it.
 *                 The number of rounds depends on the data: the call
 *                 synchronises `stream` (after each "eo_rounds" rounds, see
 *                 slim_tune_set) and returns when the output is complete;
 *                 so do batch runs and server batches holding such a job.
 *                 Every deleted edge keeps a two-edge path (the output is a
 *                 2-spanner).  selected counts the Bernoulli selections,
 *                 deleted the considered triangles.  The workspace holds
 *                 about 200 bytes per edge more than SLIM_OP_TR's, mostly
 *                 two lists of the triangles still undecided in late rounds.
 */
SLIM_API int slim_compress(const slim_graph_t* g, int op, double p, uint64_t seed, void* d_ws,
                           uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                           slim_stats_t* d_stats, void* stream);

/*
 * Spectral sparsification (section 4.2.1; kernel spectral_sparsify): the
 * edge {a<b} stays with probability p_ab = min(1, upsilon / min(d_a, d_b))
 * (degrees of the input graph; the paper suggests upsilon = p log n or
 * p m/n) and a kept edge weighs 1/p_ab.  Decided once per edge from
 * Philox4x32-10 with counter (a,b,0,2): kept iff word 0 < floor(p_ab * 2^32)
 * (2^32 when p_ab = 1), p_ab computed in IEEE double precision.
 *   upsilon         >= 0 (NaN or negative -> SLIM_EINVAL).
 *   d_out_weight    optional float32[nnz] capacity: weight (float)(1/p_ab)
 *                   of every output entry, aligned with d_out_col.
 * Other arguments as slim_edge_sample (workspace:
 * slim_workspace_size(g, SLIM_OP_SPECTRAL)).
 */
SLIM_API int slim_spectral_sparsify(const slim_graph_t* g, double upsilon, uint64_t seed,
                                    void* d_ws, uint64_t ws_bytes, int64_t* d_out_row_off,
                                    uint32_t* d_out_col, float* d_out_weight, slim_stats_t* d_stats,
                                    void* stream);

/* ------------------------------------------------------------ batches
 * Many graphs in one launch sequence: the graphs are gathered into one
 * union CSR in the workspace (graph g's vertex and entry ranges follow
 * graph g-1's), every phase runs once over the union with work tiles that
 * never straddle two graphs, and each graph's output is written to its own
 * arrays.  A batch job computes exactly what the single-graph call with the
 * same (graph, op, p, seed) computes, bit for bit; jobs of one batch may
 * mix TR and ES and differ in p and seed.  The paper runs its kernels as
 * independent concurrent instances (section 4.5, runtime listing
 * `lst:general`, `run_kernels`); batching
 * many graphs into one device pass is this library's systems extension.
 *
 * The first slim_batch_run captures the launch sequence into a HIP graph;
 * later runs with the same workspace and knobs replay it as one graph
 * launch.  Per-graph descriptors (output pointers, tile prefixes) live in a
 * table at the start of the workspace that every run refreshes with one
 * host-to-device copy, so a workspace may serve other calls between two
 * runs of a batch.
 */
typedef struct slim_job_params {
  int32_t op;    /* any SLIM_OP_* code (SLIM_OP_SPECTRAL: p carries upsilon) */
  int32_t pad;   /* must be 0 */
  double p;      /* as slim_compress */
  uint64_t seed; /* as slim_triangle_reduce / slim_edge_sample */
} slim_job_params_t;

typedef struct slim_out {
  int64_t* row_off;    /* device int64[n+1] */
  uint32_t* col;       /* device uint32[nnz] capacity (may be NULL if nnz = 0) */
  slim_stats_t* stats; /* optional device stats */
  float* weight;       /* optional device float32[nnz]: SLIM_OP_SPECTRAL weights */
} slim_out_t;

typedef struct slim_batch slim_batch_t; /* opaque, library-owned */

/*
 * Build a batch over `count` >= 1 loaded graphs (all on the current
 * device; handles and their arrays must outlive the batch) with one job
 * each.  The union must satisfy the single-graph limits: sum of n <= 2^32-1
 * and sum of m <= 2^32-1.  Errors: SLIM_EINVAL (NULL, bad op/p, limits,
 * graphs on another device), SLIM_EDEVICE.
 */
SLIM_API int slim_batch_create(const slim_graph_t* const* graphs, const slim_job_params_t* jobs,
                               uint32_t count, slim_batch_t** out);
/* Device workspace (bytes) of slim_batch_run, independent of the knobs. */
SLIM_API int slim_batch_workspace_size(const slim_batch_t* b, uint64_t* bytes);
/*
 * Run every job of the batch on `stream`.  outs[g] receives graph g's
 * result (out arrays as in slim_triangle_reduce).  d_ws: at least
 * slim_batch_workspace_size bytes, 256-byte aligned.  Runs that share a
 * batch or a workspace must not overlap.  A batch with a SLIM_OP_EOTR job
 * waits for `stream` before it returns (its rounds past the captured ones,
 * if any, then run as direct launches).  Errors: SLIM_EINVAL, SLIM_ENOMEM
 * (workspace too small), SLIM_EDEVICE.
 */
SLIM_API int slim_batch_run(slim_batch_t* b, void* d_ws, uint64_t ws_bytes, const slim_out_t* outs,
                            void* stream);
/*
 * Scheduling knobs of one batch (same keys as slim_tune_set, plus
 * "use_graph" 0/1: replay a captured HIP graph, default 1; "verbose" 0/1:
 * slim_batch_tune reports each candidate's time on stderr).  Results never
 * depend on them.
 */
SLIM_API int slim_batch_set(slim_batch_t* b, const char* key, int64_t value);
SLIM_API int slim_batch_get(const slim_batch_t* b, const char* key, int64_t* value);
/*
 * Autotuner: picks the batch's triangle tile size, blocks per CU and hash
 * chunk by timing real runs (coordinate descent over the candidates, each
 * timed with HIP events as the best of two replays), then keeps the best.
 * With a non-NULL `cache_path` the choice is looked up first under a key of
 * (device, CU count, batch size, union size) and, if absent, appended to
 * that text file after tuning.  Runs the batch several times: outs hold a
 * valid result afterwards.  Synchronises `stream`.
 */
SLIM_API int slim_batch_tune(slim_batch_t* b, void* d_ws, uint64_t ws_bytes, const slim_out_t* outs,
                             const char* cache_path, void* stream);
/*
 * Host copy of the per-graph counters of the batch's most recent run
 * (per_graph: `count` records, in graph order; the same values the run wrote
 * to outs[g].stats, kept in device memory that the batch owns, so it does
 * not matter whether outs[g].stats was set).  Waits for that run to finish.
 * The paper's per-graph quantities: n, m, T, the selected and deleted counts
 * (section 4.3; A_S of section 5 uses T).  Errors: SLIM_EINVAL (NULL, no run
 * yet), SLIM_EDEVICE.
 */
SLIM_API int slim_batch_stats(slim_batch_t* b, slim_stats_t* per_graph);
/* Release a batch (NULL is ignored).  The caller synchronises the streams
 * of its runs first. */
SLIM_API void slim_batch_free(slim_batch_t* b);

/* ------------------------------------------------------------ serving
 * A compression service inside the process: jobs arrive one at a time
 * (from any thread), are admitted while the server's device memory stays
 * within an HBM budget, and run in batches formed continuously -- each of
 * `n_streams` workers takes every admitted job that is waiting when it
 * becomes free, so jobs arriving while others are on the GPU start as soon
 * as a worker and memory are free, and the batches of different workers
 * overlap on the device.  Each job computes exactly what the single-graph
 * call computes for its (graph, op, p, seed).  The paper's runtime
 * (section 4.5, listing `lst:general`) runs one graph at a time; the server
 * is this library's systems extension.
 *
 * Memory: a job holds (a) a device copy of its CSR if it was submitted from
 * host memory, (b) its output CSR, from admission until slim_result_release,
 * and (c) its share of its batch's workspace while the batch runs.  Jobs
 * are admitted while the sum of these reservations (each rounded up to an
 * allocation size class, the workspace share with 10% headroom) stays within
 * hbm_budget_bytes.  Device memory comes from a sub-allocating arena that
 * the server owns and frees at slim_serve_destroy: it takes chunks of 2 GiB
 * (or one request's size, if larger) from the runtime, carves requests from
 * them best-fit in 4 KiB units, and merges a freed range with free
 * neighbours; a chunk goes back to the runtime only when it is entirely free
 * and a new chunk would take the arena past 1.125 x the budget, so steady
 * serving calls neither hipMalloc nor hipFree.
 */
#define SLIM_HOST 0u   /* slim_job_t.where: CSR arrays in host memory */
#define SLIM_DEVICE 1u /* slim_job_t.where: CSR arrays in device memory */

typedef struct slim_serve_cfg {
  uint64_t hbm_budget_bytes; /* device memory the server may hold for jobs (> 0) */
  uint32_t max_slots;        /* admitted, unreleased jobs at most (0 = 65536) */
  uint32_t n_streams;        /* workers, each with its own stream (0 = 2; <= 16) */
  uint32_t max_batch;        /* jobs per batch at most (0 = 4096) */
  uint32_t pad;              /* must be 0 */
} slim_serve_cfg_t;

typedef struct slim_job {
  int32_t op;           /* an op code of slim_compress */
  int32_t pad;          /* must be 0 */
  double p;             /* as slim_triangle_reduce / slim_edge_sample */
  uint64_t seed;
  const int64_t* row_off; /* CSR (the contract of slim_load_csr; not validated here) */
  const uint32_t* col;
  uint64_t n, nnz;
  uint32_t where;       /* SLIM_HOST: copied to the device when the job's batch
                           starts, so the arrays must stay valid until the job is
                           done; SLIM_DEVICE: borrowed until slim_result_release */
  uint32_t pad2;        /* must be 0 */
} slim_job_t;

typedef struct slim_result {
  int32_t status;          /* SLIM_OK, or the code the job failed with */
  int32_t pad;
  const int64_t* row_off;  /* device int64[n+1], server-owned until release */
  const uint32_t* col;     /* device uint32[m_out*2], server-owned until release */
  uint64_t n;
  slim_stats_t stats;      /* host copy */
  double queue_ms;         /* submit -> batch start */
  double latency_ms;       /* submit -> result ready (host clock) */
} slim_result_t;

typedef struct slim_serve_stats {
  uint64_t submitted, completed, failed, cancelled, queued, running, batches;
  double mean_batch_jobs;
  double p50_ms, p99_ms, mean_ms, max_ms; /* latency of completed jobs */
  double jobs_per_s;   /* completed / (last completion - first submission) */
  double edges_per_s;  /* sum of m_in of completed jobs / the same span */
  uint64_t hbm_in_use, hbm_peak, hbm_budget;
} slim_serve_stats_t;

typedef struct slim_server slim_server_t; /* opaque, library-owned */

/* Start a server on the current device.  Errors: SLIM_EINVAL, SLIM_EDEVICE. */
SLIM_API int slim_serve_create(const slim_serve_cfg_t* cfg, slim_server_t** out);
/*
 * Queue a job; *ticket identifies it.  A job that could never fit
 * (its memory alone exceeds the budget) -> SLIM_EBUDGET; bad op/p/sizes ->
 * SLIM_EINVAL.  Never blocks on the device.
 */
SLIM_API int slim_serve_submit(slim_server_t* s, const slim_job_t* job, uint64_t* ticket);
/* Result of a finished job; SLIM_EAGAIN if it is not finished yet. */
SLIM_API int slim_serve_poll(slim_server_t* s, uint64_t ticket, slim_result_t* res);
/* Blocks until the job is finished, then as slim_serve_poll. */
SLIM_API int slim_serve_wait(slim_server_t* s, uint64_t ticket, slim_result_t* res);
/*
 * Completion queue: returns the next finished job (in the order jobs finish)
 * that this call has not returned before and that is not yet released, with
 * its ticket.  timeout_ms < 0 waits without limit, 0 only looks; SLIM_EAGAIN
 * when none finished in time.
 */
SLIM_API int slim_serve_next(slim_server_t* s, int64_t timeout_ms, uint64_t* ticket,
                             slim_result_t* res);
/* Drops a job that has not started (SLIM_OK); SLIM_EAGAIN once it runs. */
SLIM_API int slim_serve_cancel(slim_server_t* s, uint64_t ticket);
/* Copies a finished job's output CSR into caller memory (host or device;
 * row_off: n+1 entries, col: 2*m_out entries).  Synchronous. */
SLIM_API int slim_serve_copy(slim_server_t* s, uint64_t ticket, int64_t* row_off, uint32_t* col);
/* Returns a finished job's memory to the server and forgets the ticket. */
SLIM_API int slim_result_release(slim_server_t* s, uint64_t ticket);
/* Counters and latency percentiles since creation or the last reset. */
SLIM_API int slim_serve_stats(slim_server_t* s, slim_serve_stats_t* out);
SLIM_API int slim_serve_reset_stats(slim_server_t* s);
/* Stops the workers (running batches finish; queued jobs are dropped) and
 * frees the server's device memory.  NULL is ignored. */
SLIM_API void slim_serve_destroy(slim_server_t* s);

/* ------------------------------------------------- scheduling knobs
 * Process-wide settings that change launch shapes and the split of work
 * only: results are bit-identical under every setting (the test suite runs
 * the parity checks under several).  Keys:
 *   "tri_chunk"          out(x) entries hashed in LDS per pass, 32..2048
 *   "tri_blocks_per_cu"  resident blocks per CU of the triangle kernel, 1..64
 *   "tri_tile"           CSR entries per triangle work tile: 256, 512 or 1024
 *   "eo_rounds"          Edge-Once rounds enqueued before the host checks
 *                        whether more are needed, 1..64 (default 16)
 *   "eo_list_try"        Edge-Once: a bidding round also writes its undecided
 *                        triangles to a list (later rounds run on the list)
 *                        once the previous round's undecided count is at most
 *                        this percent of the list capacity (three triangles
 *                        per edge); a list that overflows is dropped and the
 *                        next round tries again.  0..100000 (default 250)
 * Unknown key or value out of range -> SLIM_EINVAL.
 */
SLIM_API int slim_tune_set(const char* key, int64_t value);
SLIM_API int slim_tune_get(const char* key, int64_t* value);

/* ------------------------------------------------------- phase timing
 * When enabled, every compute call brackets each of its phases with HIP
 * events on its own stream (section 7 times compression routines; this is
 * how the per-kernel durations are taken).  slim_profile_read() waits for
 * the events of the most recent compute call and returns up to `max`
 * {name, milliseconds} pairs in launch order; *count gets the number of
 * phases.  Phases of slim_triangle_reduce: "rank", "orient", "triangles",
 * "compact"; of slim_edge_sample: "sample".  Off by default.
 */
typedef struct slim_phase {
  char name[24];
  float ms;
} slim_phase_t;

SLIM_API int slim_profile_enable(int on);
SLIM_API int slim_profile_read(slim_phase_t* out, int max, int* count);

/* ------------------------------------------------- accuracy metrics
 * Kullback-Leibler divergence of the degree distribution of a compressed
 * graph from that of its input (section 5 measures information loss by
 * D_KL(P||Q) = sum_i P(i) log2(P(i)/Q(i)), in bits): P(k) and Q(k) are the
 * fractions of the n vertices that have degree k in the input CSR and in
 * the compressed CSR (same n, same ids; degree = row length).  The result
 * is >= 0, 0 iff both graphs have the same degree counts, and +infinity
 * when some degree occurs in the input but in no vertex of the output.
 *   d_row_off_p  device int64[n+1]: offsets of the input graph (P).
 *   d_row_off_q  device int64[n+1]: offsets of the compressed graph (Q).
 *   n            vertices, < 2^32 (n = 0 gives 0).
 *   d_ws         device workspace of slim_degree_kl_workspace(n) bytes,
 *                256-byte aligned (smaller -> SLIM_ENOMEM).
 *   d_out        device double[1]: the divergence.
 * The offsets are taken as given (non-decreasing from 0, as slim_load_csr
 * requires); a row longer than n, impossible in a simple graph, counts as
 * degree n.  Enqueued on `stream`.  The sum runs in a fixed order for a
 * given n, so the result is reproducible bit for bit.  Errors: SLIM_EINVAL
 * (NULL pointers, n >= 2^32), SLIM_ENOMEM, SLIM_EDEVICE.
 */
SLIM_API int slim_degree_kl_workspace(uint64_t n, uint64_t* bytes);
SLIM_API int slim_degree_kl(const int64_t* d_row_off_p, const int64_t* d_row_off_q, uint64_t n,
                            void* d_ws, uint64_t ws_bytes, double* d_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SLIM_H_ */
