/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, obviously-correct C reference for compression
 * kernels of Slim Graph (Besta et al., "Slim Graph: Practical Lossy Graph
 * Compression for Approximate Graph Processing, Storage, and Analytics",
 * SC'19):
 *
 *   - Triangle p-1-Reduction (section 4.3, kernel `p-1-reduction` of the
 *     kernel listing `lst:kernels`): every triangle of the input graph is
 *     selected independently with probability p, and each selected triangle
 *     deletes one of its three edges chosen uniformly at random.
 *   - Uniform edge sampling (section 4.2.2, kernel `random_uniform`): every
 *     edge is deleted independently with probability p.
 *   - The Triangle p-2, Min-Count and Edge-Once variants (section 4.3) and
 *     spectral sparsification (section 4.2.1), below.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU path (its own
 * Philox, its own listing, its own compaction) and the product never calls
 * it.
 *
 * Readings of points the paper leaves open (each restated where it is used):
 *   R1  p in TR is the probability that a triangle is selected for
 *       reduction (section 4.3 calls p the sampling probability of a
 *       triangle; Table `tab:tcv`: 0.9-1-TR leaves fewer triangles than
 *       0.2-1-TR).
 *   R2  p in edge sampling is the probability that an edge is deleted
 *       (Table `tab:theory-table`: (1-p)m edges remain; Table `tab:tcv`:
 *       the uniform columns scale as (1-p)^3).
 *   R3  Snapshot semantics: the triangle set is that of the input graph, all
 *       kernel instances run once, concurrently (section 4.5, runtime
 *       listing `lst:general`: a single `run_kernels` pass); deleting an
 *       already deleted edge is a no-op.
 *   R8  Triangle p-2-Reduction (section 4.3: x in {1,2} edges of a selected
 *       triangle are removed, chosen u.a.r.): the two removed edges are the
 *       ones other than edge k of R4, i.e. the kept edge is uniform.
 *   R9  Min-Count Triangle p-1-Reduction (section 4.3): t_e = triangles of
 *       the input graph that contain e; a selected triangle removes its
 *       edge of smallest t_e, ties broken uniformly by word x1 among the
 *       tied edges in the order of R4.
 *   R10 Spectral sparsification (section 4.2.1, kernel spectral_sparsify):
 *       the kernel keeps an edge when rand <= p_uv, so p_uv is the keep
 *       probability; upsilon is passed in directly (the paper suggests
 *       p log n or p m/n); the counter domain of the edge draw is (u,v,0,2).
 *   R11 Edge-Once Triangle p-1-Reduction (section 4.3; the bounds of
 *       section 6.2 need that every edge is considered at most once and
 *       that no considered triangle loses two edges): the selected
 *       triangles (R1) are taken one at a time in increasing priority
 *       (x2, a, b, c), x2 being Philox output word 2 of the triangle's
 *       counter (R4); a triangle is considered iff none of its three edges
 *       is considered yet, and then deletes its edge k (R4) while all three
 *       of its edges become considered.  The considered triangles are the
 *       greedy maximal edge-disjoint set of selected triangles in priority
 *       order.  (The listing's branch that sets `considered` is read as
 *       applying to every considered triangle's edges.)
 *   R4  The random source `SG.rand` is unspecified in the paper; here it is
 *       Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *       key = (seed mod 2^32, seed div 2^32).  For the triangle {a<b<c}
 *       (ids sorted) the counter is (a,b,c,0); for the edge {a<b} it is
 *       (a,b,0,1).  Output word x0 decides: selected / deleted iff
 *       x0 < thr(p), thr(p) = floor(p * 2^32) (2^32 for p = 1).  Output word
 *       x1 picks the deleted edge of a selected triangle:
 *       k = floor(x1 * 3 / 2^32), 0 -> {a,b}, 1 -> {a,c}, 2 -> {b,c}.
 *
 * Build: gcc -O2 -shared -fPIC slim_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------- Philox4x32-10
 * Salmon et al., SC'11, section 3.3 (the Philox S-box).  A round maps the
 * counter words (x0,x1,x2,x3) with round key (k0,k1) to
 *   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))
 * where hi/lo are the halves of the 64-bit product; between rounds the key
 * advances by the Weyl constants (W0,W1).  Ten rounds.
 */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += ORC_PHILOX_W0;
      k1 += ORC_PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Selection threshold: an event of probability p happens iff x0 < thr(p). */
int orc_threshold(double p, uint64_t* thr) {
  if (!(p >= 0.0 && p <= 1.0)) return -1; /* also rejects NaN */
  if (p >= 1.0)
    *thr = 4294967296ull;
  else
    *thr = (uint64_t)floor(p * 4294967296.0);
  return 0;
}

int orc_edge_triangle_counts(uint64_t n, const int64_t* row_off, const uint32_t* col,
                             uint32_t* t);

/* ------------------------------------------------------ graph helpers */

typedef struct {
  uint64_t n;
  const int64_t* row_off;
  const uint32_t* col;
} orc_graph;

/* Check the input contract: n < 2^32, offsets monotone from 0, ids < n,
 * rows strictly increasing (sorted, no duplicates), no self-loops, and every
 * edge present in both directions.  Returns 0 if valid. */
int orc_validate(uint64_t n, const int64_t* row_off, const uint32_t* col) {
  if (n > 0xffffffffull) return -1;
  if (row_off[0] != 0) return -2;
  for (uint64_t r = 0; r < n; ++r) {
    if (row_off[r + 1] < row_off[r]) return -3;
    for (int64_t j = row_off[r]; j < row_off[r + 1]; ++j) {
      if ((uint64_t)col[j] >= n) return -4;
      if (col[j] == r) return -5;
      if (j > row_off[r] && col[j] <= col[j - 1]) return -6;
    }
  }
  for (uint64_t r = 0; r < n; ++r) {
    for (int64_t j = row_off[r]; j < row_off[r + 1]; ++j) {
      uint32_t c = col[j];
      int64_t lo = row_off[c], hi = row_off[c + 1];
      int found = 0;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < r)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < row_off[c + 1] && col[lo] == r) found = 1;
      if (!found) return -7;
    }
  }
  return 0;
}

/* CSR position of b in row a, or -1. */
static int64_t orc_find(const orc_graph* g, uint32_t a, uint32_t b) {
  int64_t lo = g->row_off[a], hi = g->row_off[a + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < g->row_off[a + 1] && g->col[lo] == b) return lo;
  return -1;
}

/* Position that identifies the undirected edge {x,y}: the CSR position of
 * the copy stored in the row of the smaller id. */
static int64_t orc_edge_slot(const orc_graph* g, uint32_t x, uint32_t y) {
  return x < y ? orc_find(g, x, y) : orc_find(g, y, x);
}

/* ------------------------------------------------- triangle listing
 * The "forward" algorithm (Schank and Wagner, WEA 2005; Latapy, TCS 2008):
 * order vertices by (degree, id); A(u) = neighbours of u ranked above u,
 * kept in id order; every triangle with rank order x < y < z is reported
 * exactly once, at u = x, v = y, w = z, as w in A(x) and w in A(y).  Work is
 * O(m^{3/2}), the bound the paper quotes for mining all triangles (4.3).
 */
typedef void (*orc_tri_fn)(void* ctx, uint32_t x, uint32_t y, uint32_t z);

static int orc_rank_less(const orc_graph* g, uint32_t a, uint32_t b) {
  int64_t da = g->row_off[a + 1] - g->row_off[a];
  int64_t db = g->row_off[b + 1] - g->row_off[b];
  return da < db || (da == db && a < b);
}

static int orc_for_each_triangle(const orc_graph* g, orc_tri_fn fn, void* ctx) {
  uint64_t n = g->n;
  int64_t* a_off = (int64_t*)malloc((n + 1) * sizeof(int64_t));
  if (!a_off) return -1;
  a_off[0] = 0;
  for (uint64_t u = 0; u < n; ++u) {
    int64_t k = 0;
    for (int64_t j = g->row_off[u]; j < g->row_off[u + 1]; ++j)
      if (orc_rank_less(g, (uint32_t)u, g->col[j])) ++k;
    a_off[u + 1] = a_off[u] + k;
  }
  uint32_t* a_col = (uint32_t*)malloc((size_t)(a_off[n] > 0 ? a_off[n] : 1) * sizeof(uint32_t));
  if (!a_col) {
    free(a_off);
    return -1;
  }
  for (uint64_t u = 0; u < n; ++u) {
    int64_t k = a_off[u];
    for (int64_t j = g->row_off[u]; j < g->row_off[u + 1]; ++j)
      if (orc_rank_less(g, (uint32_t)u, g->col[j])) a_col[k++] = g->col[j];
  }
  for (uint64_t u = 0; u < n; ++u) {
    for (int64_t e = a_off[u]; e < a_off[u + 1]; ++e) {
      uint32_t v = a_col[e];
      int64_t i = a_off[u], ie = a_off[u + 1];
      int64_t j = a_off[v], je = a_off[v + 1];
      while (i < ie && j < je) {
        if (a_col[i] < a_col[j])
          ++i;
        else if (a_col[i] > a_col[j])
          ++j;
        else {
          fn(ctx, (uint32_t)u, v, a_col[i]);
          ++i;
          ++j;
        }
      }
    }
  }
  free(a_off);
  free(a_col);
  return 0;
}

static void orc_sort3(uint32_t* a, uint32_t* b, uint32_t* c) {
  uint32_t t;
  if (*a > *b) { t = *a; *a = *b; *b = t; }
  if (*b > *c) { t = *b; *b = *c; *c = t; }
  if (*a > *b) { t = *a; *a = *b; *b = t; }
}

/* ---- list all triangles as id-sorted triples (test helper) */
typedef struct {
  uint32_t* out;
  uint64_t cap, count;
} orc_list_ctx;

static void orc_list_cb(void* vctx, uint32_t x, uint32_t y, uint32_t z) {
  orc_list_ctx* c = (orc_list_ctx*)vctx;
  orc_sort3(&x, &y, &z);
  if (c->count < c->cap) {
    c->out[3 * c->count + 0] = x;
    c->out[3 * c->count + 1] = y;
    c->out[3 * c->count + 2] = z;
  }
  c->count++;
}

/* Writes up to `cap` triangles; returns the total count in *count. */
int orc_list_triangles(uint64_t n, const int64_t* row_off, const uint32_t* col, uint32_t* out,
                       uint64_t cap, uint64_t* count) {
  orc_graph g = {n, row_off, col};
  orc_list_ctx c = {out, cap, 0};
  int rc = orc_for_each_triangle(&g, orc_list_cb, &c);
  *count = c.count;
  return rc;
}

/* ---------------------------------------- Triangle p-1-Reduction (4.3)
 * stats[0..5] = {n, m_in, T, selected, deleted, m_out}.
 * out_row_off has n+1 entries; out_col must hold nnz entries.
 */
typedef struct {
  const orc_graph* g;
  uint64_t thr;
  uint32_t key[2];
  uint8_t* del; /* indexed by orc_edge_slot */
  uint64_t T, selected;
  int err;
} orc_tr_ctx;

static void orc_tr_cb(void* vctx, uint32_t x, uint32_t y, uint32_t z) {
  orc_tr_ctx* c = (orc_tr_ctx*)vctx;
  orc_sort3(&x, &y, &z);
  uint32_t ctr[4] = {x, y, z, 0u};
  uint32_t r[4];
  orc_philox4x32_10(ctr, c->key, r);
  c->T++;
  /* kernel p-1-reduction: the triangle is reduced with probability p (R1) */
  if ((uint64_t)r[0] < c->thr) {
    c->selected++;
    /* rand(triangle): one of the three edges, uniformly (R4) */
    uint32_t k = (uint32_t)(((uint64_t)r[1] * 3u) >> 32);
    uint32_t ea = k == 2 ? y : x;
    uint32_t eb = k == 0 ? y : z;
    int64_t slot = orc_edge_slot(c->g, ea, eb);
    if (slot < 0)
      c->err = 1;
    else
      c->del[slot] = 1; /* SG.del: idempotent (R3) */
  }
}

static void orc_compact(const orc_graph* g, const uint8_t* del, int64_t* out_row_off,
                        uint32_t* out_col) {
  int64_t k = 0;
  out_row_off[0] = 0;
  for (uint64_t r = 0; r < g->n; ++r) {
    for (int64_t j = g->row_off[r]; j < g->row_off[r + 1]; ++j) {
      uint32_t c = g->col[j];
      int64_t slot = (uint64_t)c > r ? j : orc_find(g, c, (uint32_t)r);
      if (!del[slot]) out_col[k++] = c;
    }
    out_row_off[r + 1] = k;
  }
}

int orc_triangle_reduce(uint64_t n, const int64_t* row_off, const uint32_t* col, double p,
                        uint64_t seed, int64_t* out_row_off, uint32_t* out_col, uint64_t* stats) {
  orc_graph g = {n, row_off, col};
  uint64_t nnz = (uint64_t)row_off[n];
  orc_tr_ctx c;
  memset(&c, 0, sizeof(c));
  if (orc_threshold(p, &c.thr)) return -1;
  c.g = &g;
  c.key[0] = (uint32_t)seed;
  c.key[1] = (uint32_t)(seed >> 32);
  c.del = (uint8_t*)calloc(nnz > 0 ? nnz : 1, 1);
  if (!c.del) return -2;
  if (orc_for_each_triangle(&g, orc_tr_cb, &c) || c.err) {
    free(c.del);
    return -3;
  }
  uint64_t deleted = 0;
  for (uint64_t j = 0; j < nnz; ++j) deleted += c.del[j];
  orc_compact(&g, c.del, out_row_off, out_col);
  free(c.del);
  stats[0] = n;
  stats[1] = nnz / 2;
  stats[2] = c.T;
  stats[3] = c.selected;
  stats[4] = deleted;
  stats[5] = nnz / 2 - deleted;
  return 0;
}

/* ------------------------------- Triangle p-x-Reduction variants (4.3)
 * variant 1: p-1 (as orc_triangle_reduce); variant 2: Triangle
 * p-2-Reduction, where a selected triangle loses x = 2 of its edges chosen
 * uniformly, i.e. keeps the one edge k = floor(x1 * 3 / 2^32) and loses the
 * other two (R8); variant 3: Min-Count Triangle p-1-Reduction, where a
 * selected triangle loses the edge that lies in the fewest triangles of the
 * input graph, ties broken uniformly: among the tied edges, in the order
 * {a,b}, {a,c}, {b,c}, the one at index floor(x1 * ties / 2^32) (R9);
 * variant 4: Edge-Once p-1 (R11, below).  stats as orc_triangle_reduce.
 */
typedef struct {
  const orc_graph* g;
  uint64_t thr;
  uint32_t key[2];
  int variant;
  const uint32_t* tcount; /* variant 3: triangles per CSR entry */
  uint8_t* del;
  uint64_t T, selected;
  int err;
} orc_trx_ctx;

static void orc_trx_cb(void* vctx, uint32_t x, uint32_t y, uint32_t z) {
  orc_trx_ctx* c = (orc_trx_ctx*)vctx;
  orc_sort3(&x, &y, &z);
  uint32_t ctr[4] = {x, y, z, 0u};
  uint32_t r[4];
  orc_philox4x32_10(ctr, c->key, r);
  c->T++;
  if ((uint64_t)r[0] >= c->thr) return;
  c->selected++;
  /* the three edges in the fixed order {x,y}, {x,z}, {y,z} */
  int64_t slot[3] = {orc_edge_slot(c->g, x, y), orc_edge_slot(c->g, x, z),
                     orc_edge_slot(c->g, y, z)};
  if (slot[0] < 0 || slot[1] < 0 || slot[2] < 0) {
    c->err = 1;
    return;
  }
  if (c->variant == 3) {
    uint32_t t[3], tmin;
    for (int e = 0; e < 3; ++e) t[e] = c->tcount[slot[e]];
    tmin = t[0];
    if (t[1] < tmin) tmin = t[1];
    if (t[2] < tmin) tmin = t[2];
    int tied[3], nt = 0;
    for (int e = 0; e < 3; ++e)
      if (t[e] == tmin) tied[nt++] = e;
    uint32_t pick = (uint32_t)(((uint64_t)r[1] * (uint64_t)nt) >> 32);
    c->del[slot[tied[pick]]] = 1;
  } else {
    uint32_t k = (uint32_t)(((uint64_t)r[1] * 3u) >> 32);
    for (int e = 0; e < 3; ++e) {
      int hit = c->variant == 2 ? e != (int)k : e == (int)k;
      if (hit) c->del[slot[e]] = 1;
    }
  }
}

/* ----------------------- Edge-Once Triangle p-1-Reduction (4.3, 6.2)
 * variant 4 (R11): collect the selected triangles with their priority x2
 * and edge choice k, sort them by (x2, a, b, c), then walk them in that
 * order; a triangle none of whose edges is considered yet deletes edge k
 * and marks its three edges considered, any other is skipped.
 *
 * With `buckets` > 1 the same walk is done in pieces, to bound the memory
 * the selected triangles take: the x2 range [0, 2^32) is cut into `buckets`
 * consecutive ranges, and for each range in increasing order the triangles
 * are listed again, the selected ones whose x2 falls in it are collected,
 * sorted and walked.  Every triangle of an earlier range precedes every
 * triangle of a later one in the order (x2, a, b, c), so the walk visits the
 * triangles in the same order as with one range.
 */
typedef struct {
  uint32_t pri, a, b, c, k;
} orc_eo_tri;

typedef struct {
  uint64_t thr;
  uint32_t key[2];
  uint64_t pri_lo, pri_hi; /* collect selected triangles with x2 in [lo, hi) */
  orc_eo_tri* sel;
  uint64_t T, selected, count, cap;
  int err;
} orc_eo_ctx;

static void orc_eo_cb(void* vctx, uint32_t x, uint32_t y, uint32_t z) {
  orc_eo_ctx* c = (orc_eo_ctx*)vctx;
  orc_sort3(&x, &y, &z);
  uint32_t ctr[4] = {x, y, z, 0u};
  uint32_t r[4];
  orc_philox4x32_10(ctr, c->key, r);
  c->T++;
  if ((uint64_t)r[0] >= c->thr) return;
  c->selected++;
  if ((uint64_t)r[2] < c->pri_lo || (uint64_t)r[2] >= c->pri_hi) return;
  if (c->count == c->cap) {
    uint64_t cap = c->cap ? 2 * c->cap : 1024;
    orc_eo_tri* s = (orc_eo_tri*)realloc(c->sel, cap * sizeof(orc_eo_tri));
    if (!s) {
      c->err = 1;
      return;
    }
    c->sel = s;
    c->cap = cap;
  }
  orc_eo_tri t = {r[2], x, y, z, (uint32_t)(((uint64_t)r[1] * 3u) >> 32)};
  c->sel[c->count++] = t;
}

static int orc_eo_cmp(const void* pa, const void* pb) {
  const orc_eo_tri* a = (const orc_eo_tri*)pa;
  const orc_eo_tri* b = (const orc_eo_tri*)pb;
  if (a->pri != b->pri) return a->pri < b->pri ? -1 : 1;
  if (a->a != b->a) return a->a < b->a ? -1 : 1;
  if (a->b != b->b) return a->b < b->b ? -1 : 1;
  if (a->c != b->c) return a->c < b->c ? -1 : 1;
  return 0;
}

int orc_triangle_reduce_eo(uint64_t n, const int64_t* row_off, const uint32_t* col, double p,
                           uint64_t seed, uint32_t buckets, int64_t* out_row_off,
                           uint32_t* out_col, uint64_t* stats) {
  orc_graph g = {n, row_off, col};
  uint64_t nnz = (uint64_t)row_off[n];
  uint64_t thr;
  if (orc_threshold(p, &thr)) return -1;
  if (buckets == 0) return -4;
  uint8_t* del = (uint8_t*)calloc(nnz > 0 ? nnz : 1, 1);
  uint8_t* considered = (uint8_t*)calloc(nnz > 0 ? nnz : 1, 1);
  if (!del || !considered) {
    free(del);
    free(considered);
    return -2;
  }
  uint64_t T = 0, selected = 0;
  int err = 0;
  for (uint32_t bk = 0; bk < buckets && !err; ++bk) {
    orc_eo_ctx c;
    memset(&c, 0, sizeof(c));
    c.thr = thr;
    c.key[0] = (uint32_t)seed;
    c.key[1] = (uint32_t)(seed >> 32);
    c.pri_lo = (uint64_t)bk * 4294967296ull / buckets;
    c.pri_hi = (uint64_t)(bk + 1) * 4294967296ull / buckets;
    if (orc_for_each_triangle(&g, orc_eo_cb, &c) || c.err) {
      free(c.sel);
      err = 1;
      break;
    }
    T = c.T;
    selected = c.selected;
    if (c.count > 1) qsort(c.sel, c.count, sizeof(orc_eo_tri), orc_eo_cmp);
    for (uint64_t i = 0; i < c.count; ++i) {
      const orc_eo_tri* t = &c.sel[i];
      /* the edges in the order of R4: {a,b}, {a,c}, {b,c} */
      int64_t slot[3] = {orc_edge_slot(&g, t->a, t->b), orc_edge_slot(&g, t->a, t->c),
                         orc_edge_slot(&g, t->b, t->c)};
      if (slot[0] < 0 || slot[1] < 0 || slot[2] < 0) {
        err = 1;
        break;
      }
      if (considered[slot[0]] || considered[slot[1]] || considered[slot[2]]) continue;
      del[slot[t->k]] = 1;
      considered[slot[0]] = considered[slot[1]] = considered[slot[2]] = 1;
    }
    free(c.sel);
  }
  free(considered);
  if (err) {
    free(del);
    return -3;
  }
  uint64_t deleted = 0;
  for (uint64_t j = 0; j < nnz; ++j) deleted += del[j];
  orc_compact(&g, del, out_row_off, out_col);
  free(del);
  stats[0] = n;
  stats[1] = nnz / 2;
  stats[2] = T;
  stats[3] = selected;
  stats[4] = deleted;
  stats[5] = nnz / 2 - deleted;
  return 0;
}

int orc_triangle_reduce_x(uint64_t n, const int64_t* row_off, const uint32_t* col, double p,
                          uint64_t seed, int variant, int64_t* out_row_off, uint32_t* out_col,
                          uint64_t* stats) {
  if (variant == 4)
    return orc_triangle_reduce_eo(n, row_off, col, p, seed, 1, out_row_off, out_col, stats);
  if (variant < 1 || variant > 3) return -4;
  orc_graph g = {n, row_off, col};
  uint64_t nnz = (uint64_t)row_off[n];
  orc_trx_ctx c;
  memset(&c, 0, sizeof(c));
  if (orc_threshold(p, &c.thr)) return -1;
  c.g = &g;
  c.key[0] = (uint32_t)seed;
  c.key[1] = (uint32_t)(seed >> 32);
  c.variant = variant;
  c.del = (uint8_t*)calloc(nnz > 0 ? nnz : 1, 1);
  uint32_t* tc = NULL;
  if (!c.del) return -2;
  if (variant == 3) {
    tc = (uint32_t*)malloc((nnz > 0 ? nnz : 1) * sizeof(uint32_t));
    if (!tc) {
      free(c.del);
      return -2;
    }
    if (orc_edge_triangle_counts(n, row_off, col, tc)) {
      free(c.del);
      free(tc);
      return -3;
    }
    c.tcount = tc;
  }
  if (orc_for_each_triangle(&g, orc_trx_cb, &c) || c.err) {
    free(c.del);
    free(tc);
    return -3;
  }
  uint64_t deleted = 0;
  for (uint64_t j = 0; j < nnz; ++j) deleted += c.del[j];
  orc_compact(&g, c.del, out_row_off, out_col);
  free(c.del);
  free(tc);
  stats[0] = n;
  stats[1] = nnz / 2;
  stats[2] = c.T;
  stats[3] = c.selected;
  stats[4] = deleted;
  stats[5] = nnz / 2 - deleted;
  return 0;
}

/* ---------------------------------------- uniform edge sampling (4.2.2)
 * stats[0..5] = {n, m_in, 0, 0, deleted, m_out}.  The decision for {a<b}
 * is taken once from counter (a,b,0,1), so both CSR copies agree.
 */
int orc_edge_sample(uint64_t n, const int64_t* row_off, const uint32_t* col, double p,
                    uint64_t seed, int64_t* out_row_off, uint32_t* out_col, uint64_t* stats) {
  uint64_t thr;
  if (orc_threshold(p, &thr)) return -1;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint64_t nnz = (uint64_t)row_off[n];
  int64_t k = 0;
  uint64_t deleted = 0;
  out_row_off[0] = 0;
  for (uint64_t r = 0; r < n; ++r) {
    for (int64_t j = row_off[r]; j < row_off[r + 1]; ++j) {
      uint32_t c = col[j];
      uint32_t a = (uint64_t)c < r ? c : (uint32_t)r;
      uint32_t b = (uint64_t)c < r ? (uint32_t)r : c;
      uint32_t ctr[4] = {a, b, 0u, 1u};
      uint32_t x[4];
      orc_philox4x32_10(ctr, key, x);
      /* kernel random_uniform: the edge is deleted with probability p (R2) */
      if ((uint64_t)x[0] < thr) {
        if ((uint64_t)c > r) deleted++;
      } else {
        out_col[k++] = c;
      }
    }
    out_row_off[r + 1] = k;
  }
  stats[0] = n;
  stats[1] = nnz / 2;
  stats[2] = 0;
  stats[3] = 0;
  stats[4] = deleted;
  stats[5] = nnz / 2 - deleted;
  return 0;
}

/* ------------------------------- spectral sparsification (4.2.1)
 * Kernel spectral_sparsify: the edge {u<v} stays with probability
 * p_uv = min(1, upsilon / min(d_u, d_v)) (degrees of the input graph) and a
 * kept edge gets weight 1/p_uv.  Decided once per edge from counter
 * (u,v,0,2): kept iff word 0 < floor(p_uv * 2^32) (2^32 when p_uv = 1), with
 * p_uv computed in double precision (R10).  out_w (float, may be NULL) gets the
 * weight of every output entry, (float)(1.0 / p_uv).  stats as
 * orc_edge_sample.  upsilon must be >= 0 (NaN -> -1).
 */
int orc_spectral_sparsify(uint64_t n, const int64_t* row_off, const uint32_t* col, double upsilon,
                          uint64_t seed, int64_t* out_row_off, uint32_t* out_col, float* out_w,
                          uint64_t* stats) {
  if (!(upsilon >= 0.0)) return -1;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint64_t nnz = (uint64_t)row_off[n];
  int64_t k = 0;
  uint64_t deleted = 0;
  out_row_off[0] = 0;
  for (uint64_t r = 0; r < n; ++r) {
    for (int64_t j = row_off[r]; j < row_off[r + 1]; ++j) {
      uint32_t c = col[j];
      uint32_t a = (uint64_t)c < r ? c : (uint32_t)r;
      uint32_t b = (uint64_t)c < r ? (uint32_t)r : c;
      int64_t da = row_off[a + 1] - row_off[a], db = row_off[b + 1] - row_off[b];
      double dmin = (double)(da < db ? da : db);
      double pe = upsilon / dmin;
      if (pe > 1.0) pe = 1.0;
      uint64_t thr;
      orc_threshold(pe, &thr);
      uint32_t ctr[4] = {a, b, 0u, 2u};
      uint32_t x[4];
      orc_philox4x32_10(ctr, key, x);
      if ((uint64_t)x[0] < thr) {
        if (out_w) out_w[k] = (float)(1.0 / pe);
        out_col[k++] = c;
      } else if ((uint64_t)c > r) {
        deleted++;
      }
    }
    out_row_off[r + 1] = k;
  }
  stats[0] = n;
  stats[1] = nnz / 2;
  stats[2] = 0;
  stats[3] = 0;
  stats[4] = deleted;
  stats[5] = nnz / 2 - deleted;
  return 0;
}

/* ------------------------------------------ per-row local TR oracle
 * The output row r of Triangle p-1-Reduction, computed from the definition
 * without listing the whole graph: the edge {r,c} is deleted iff some
 * triangle {r,c,w} (w a common neighbour, found by merging the two full
 * adjacency rows) is selected and picks {r,c}.  Used to check sampled rows
 * of graphs too large for the full oracle.  out_off[i+1]-out_off[i] is the
 * length of the i-th requested row; out_col must hold the sum of the input
 * lengths of the requested rows.
 */
int orc_tr_rows(uint64_t n, const int64_t* row_off, const uint32_t* col, double p, uint64_t seed,
                const uint32_t* rows, uint64_t nrows, int64_t* out_off, uint32_t* out_col) {
  uint64_t thr;
  if (orc_threshold(p, &thr)) return -1;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  int64_t k = 0;
  out_off[0] = 0;
  for (uint64_t i = 0; i < nrows; ++i) {
    uint32_t r = rows[i];
    if ((uint64_t)r >= n) return -2;
    for (int64_t j = row_off[r]; j < row_off[r + 1]; ++j) {
      uint32_t c = col[j];
      int deleted = 0;
      int64_t a = row_off[r], ae = row_off[r + 1];
      int64_t b = row_off[c], be = row_off[c + 1];
      while (a < ae && b < be && !deleted) {
        if (col[a] < col[b])
          ++a;
        else if (col[a] > col[b])
          ++b;
        else {
          uint32_t x = r, y = c, z = col[a];
          orc_sort3(&x, &y, &z);
          uint32_t ctr[4] = {x, y, z, 0u};
          uint32_t h[4];
          orc_philox4x32_10(ctr, key, h);
          if ((uint64_t)h[0] < thr) {
            uint32_t kk = (uint32_t)(((uint64_t)h[1] * 3u) >> 32);
            uint32_t ea = kk == 2 ? y : x;
            uint32_t eb = kk == 0 ? y : z;
            uint32_t lo = r < c ? r : c, hi = r < c ? c : r;
            if (ea == lo && eb == hi) deleted = 1;
          }
          ++a;
          ++b;
        }
      }
      if (!deleted) out_col[k++] = c;
    }
    out_off[i + 1] = k;
  }
  return 0;
}

/* ------------------------------------------ per-edge triangle counts
 * t[j] = number of triangles of the input graph that contain the undirected
 * edge of CSR entry j = (r,c) (the t_e of R9).  Every triangle is listed
 * once (the forward listing above) and adds one to each of its three edges,
 * counted at the copy in the row of the smaller id; the copy in the other
 * row then takes the same count.  (Merging the two full rows of every entry
 * gives the same numbers but costs the sum of squared degrees.)
 */
typedef struct {
  const orc_graph* g;
  uint32_t* t;
  int err;
} orc_count_ctx;

static void orc_count_cb(void* vctx, uint32_t x, uint32_t y, uint32_t z) {
  orc_count_ctx* c = (orc_count_ctx*)vctx;
  orc_sort3(&x, &y, &z);
  int64_t slot[3] = {orc_edge_slot(c->g, x, y), orc_edge_slot(c->g, x, z),
                     orc_edge_slot(c->g, y, z)};
  for (int e = 0; e < 3; ++e) {
    if (slot[e] < 0)
      c->err = 1;
    else
      c->t[slot[e]]++;
  }
}

int orc_edge_triangle_counts(uint64_t n, const int64_t* row_off, const uint32_t* col,
                             uint32_t* t) {
  orc_graph g = {n, row_off, col};
  uint64_t nnz = (uint64_t)row_off[n];
  memset(t, 0, (size_t)nnz * sizeof(uint32_t));
  orc_count_ctx c = {&g, t, 0};
  if (orc_for_each_triangle(&g, orc_count_cb, &c) || c.err) return -3;
  for (uint64_t r = 0; r < n; ++r)
    for (int64_t j = row_off[r]; j < row_off[r + 1]; ++j)
      if ((uint64_t)col[j] < r) t[j] = t[orc_find(&g, col[j], (uint32_t)r)];
  return 0;
}
