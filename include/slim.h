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
 *     library never allocates device memory and never frees caller memory.
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
#define SLIM_OP_TR 1 /* Triangle p-1-Reduction */
#define SLIM_OP_ES 2 /* uniform edge sampling */

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

/* ------------------------------------------------- scheduling knobs
 * Process-wide settings that change launch shapes and the split of work
 * only: results are bit-identical under every setting (the test suite runs
 * the parity checks under several).  Keys:
 *   "tri_chunk"          out(x) entries hashed in LDS per pass, 32..2048
 *   "tri_blocks_per_cu"  resident blocks per CU of the triangle kernel, 1..64
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

#ifdef __cplusplus
}
#endif
#endif /* SLIM_H_ */
