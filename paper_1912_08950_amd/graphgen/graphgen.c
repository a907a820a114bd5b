/*
 * Seeded synthetic graph generators: Erdos-Renyi G(n,q) and R-MAT.
 *
 * Both produce an undirected simple graph as a symmetric CSR with strictly
 * increasing rows, no self-loops and uint32 vertex ids (int64 row offsets).
 * This file holds no part of the compression method: it only draws input
 * graphs, and the same output feeds the GPU path and the CPU oracle.
 *
 * Determinism: every random draw comes from a counter-based stream keyed by
 * (seed, row) for G(n,q) and (seed, sample index) for R-MAT, so the graph
 * does not depend on the number of OpenMP threads.  The stream is the
 * SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC graphgen.c -o libslimgen.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- RNG */

static inline uint64_t gg_mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t s;
} gg_rng;

static inline gg_rng gg_stream(uint64_t seed, uint64_t domain, uint64_t id) {
  gg_rng r;
  r.s = gg_mix64(gg_mix64(seed ^ (domain * 0xd1b54a32d192ed03ull)) + id);
  return r;
}

static inline uint64_t gg_next(gg_rng* r) {
  r->s += 0x9e3779b97f4a7c15ull;
  uint64_t z = r->s;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

/* uniform double in [0,1) from the top 53 bits */
static inline double gg_unit(gg_rng* r) {
  return (double)(gg_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------- edge list -> CSR */

static void gg_sort_u32(uint32_t* a, int64_t len, uint32_t* tmp) {
  if (len <= 64) {
    for (int64_t i = 1; i < len; ++i) {
      uint32_t x = a[i];
      int64_t j = i - 1;
      while (j >= 0 && a[j] > x) {
        a[j + 1] = a[j];
        --j;
      }
      a[j + 1] = x;
    }
    return;
  }
  /* LSD radix sort, 8-bit passes over the significant bits, ping-pong with tmp */
  uint32_t mx = 0;
  for (int64_t i = 0; i < len; ++i) mx = a[i] > mx ? a[i] : mx;
  int passes = 1;
  while (passes < 4 && (mx >> (8 * passes)) != 0) ++passes;
  uint32_t* src = a;
  uint32_t* dst = tmp;
  for (int shift = 0; shift < 8 * passes; shift += 8) {
    int64_t cnt[257];
    memset(cnt, 0, sizeof(cnt));
    for (int64_t i = 0; i < len; ++i) cnt[((src[i] >> shift) & 255u) + 1]++;
    for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
    for (int64_t i = 0; i < len; ++i) dst[cnt[(src[i] >> shift) & 255u]++] = src[i];
    uint32_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != a) memcpy(a, src, (size_t)len * sizeof(uint32_t));
}

/*
 * Symmetrize a list of (u,v) pairs, drop self-loops and duplicates, and
 * build a CSR with sorted rows.  Pairs with an endpoint >= n are dropped.
 * On success *row_off (n+1 int64) and *col (nnz uint32) are malloc'ed.
 */
static int gg_pairs_to_csr(uint64_t n, const uint32_t* pu, const uint32_t* pv, uint64_t npairs,
                           int64_t** row_off_out, uint32_t** col_out, uint64_t* nnz_out) {
  int64_t* cnt = (int64_t*)calloc(n + 1, sizeof(int64_t));
  if (!cnt) return -1;
  /* inside an enclosing parallel region (sg_gen_many) the loops below run on
   * one thread, so plain increments suffice */
  int serial = 0;
#ifdef _OPENMP
  serial = omp_in_parallel();
#else
  serial = 1;
#endif
  if (serial) {
    for (uint64_t i = 0; i < npairs; ++i) {
      uint32_t u = pu[i], v = pv[i];
      if (u == v || u >= n || v >= n) continue;
      cnt[u]++;
      cnt[v]++;
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)npairs; ++i) {
      uint32_t u = pu[i], v = pv[i];
      if (u == v || u >= n || v >= n) continue;
      __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
      __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    }
  }
  int64_t* off = (int64_t*)malloc((n + 1) * sizeof(int64_t));
  if (!off) {
    free(cnt);
    return -1;
  }
  off[0] = 0;
  for (uint64_t r = 0; r < n; ++r) off[r + 1] = off[r] + cnt[r];
  int64_t total = off[n];
  uint32_t* adj = (uint32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(uint32_t));
  if (!adj) {
    free(cnt);
    free(off);
    return -1;
  }
  /* cnt becomes the per-row cursor */
  memcpy(cnt, off, n * sizeof(int64_t));
  if (serial) {
    for (uint64_t i = 0; i < npairs; ++i) {
      uint32_t u = pu[i], v = pv[i];
      if (u == v || u >= n || v >= n) continue;
      adj[cnt[u]++] = v;
      adj[cnt[v]++] = u;
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)npairs; ++i) {
      uint32_t u = pu[i], v = pv[i];
      if (u == v || u >= n || v >= n) continue;
      int64_t a = __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
      int64_t b = __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
      adj[a] = v;
      adj[b] = u;
    }
  }
  /* sort + dedup every row in place; cnt[r] := deduplicated length */
#pragma omp parallel
  {
    int64_t tmp_cap = 0;
    uint32_t* tmp = NULL;
#pragma omp for schedule(dynamic, 1024)
    for (int64_t r = 0; r < (int64_t)n; ++r) {
      int64_t b = off[r], len = off[r + 1] - off[r];
      if (len > tmp_cap) {
        free(tmp);
        tmp_cap = len;
        tmp = (uint32_t*)malloc((size_t)tmp_cap * sizeof(uint32_t));
      }
      gg_sort_u32(adj + b, len, tmp);
      int64_t k = 0;
      for (int64_t i = 0; i < len; ++i)
        if (k == 0 || adj[b + i] != adj[b + k - 1]) adj[b + k++] = adj[b + i];
      cnt[r] = k;
    }
    free(tmp);
  }
  int64_t* ro = (int64_t*)malloc((n + 1) * sizeof(int64_t));
  if (!ro) {
    free(cnt);
    free(off);
    free(adj);
    return -1;
  }
  ro[0] = 0;
  for (uint64_t r = 0; r < n; ++r) ro[r + 1] = ro[r] + cnt[r];
  uint64_t nnz = (uint64_t)ro[n];
  uint32_t* col = (uint32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(uint32_t));
  if (!col) {
    free(cnt);
    free(off);
    free(adj);
    free(ro);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t r = 0; r < (int64_t)n; ++r)
    memcpy(col + ro[r], adj + off[r], (size_t)cnt[r] * sizeof(uint32_t));
  free(cnt);
  free(off);
  free(adj);
  *row_off_out = ro;
  *col_out = col;
  *nnz_out = nnz;
  return 0;
}

/* ------------------------------------------------------------ G(n,q) */

/*
 * Erdos-Renyi G(n,q): every unordered pair {u<v} is an edge independently
 * with probability q.  Row u's candidates v in (u, n) are visited with
 * geometric skips (Batagelj and Brandes, Phys. Rev. E 71, 2005), drawn from
 * the stream (seed, u).
 */
static int64_t gg_er_row(uint64_t n, double q, double lq, uint64_t seed, uint64_t u,
                         uint32_t* out /* may be NULL: count only */) {
  gg_rng r = gg_stream(seed, 1, u);
  int64_t k = 0;
  if (q <= 0.0) return 0;
  if (q >= 1.0) {
    for (uint64_t v = u + 1; v < n; ++v) {
      if (out) out[k] = (uint32_t)v;
      ++k;
    }
    return k;
  }
  uint64_t v = u;
  for (;;) {
    double x = gg_unit(&r);
    double skip = floor(log1p(-x) / lq); /* >= 0 */
    if (skip >= (double)(n - v)) break;
    v += 1 + (uint64_t)skip;
    if (v >= n) break;
    if (out) out[k] = (uint32_t)v;
    ++k;
  }
  return k;
}

int sg_gen_er(uint64_t n, double avg_degree, uint64_t seed, int64_t** row_off, uint32_t** col,
              uint64_t* nnz) {
  if (n < 1 || n > 0xffffffffull) return -2;
  double q = n > 1 ? avg_degree / (double)(n - 1) : 0.0;
  if (q > 1.0) q = 1.0;
  double lq = q < 1.0 ? log1p(-q) : 0.0;
  int64_t* cnt = (int64_t*)calloc(n + 1, sizeof(int64_t));
  if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t u = 0; u < (int64_t)n; ++u) cnt[u + 1] = gg_er_row(n, q, lq, seed, (uint64_t)u, NULL);
  for (uint64_t u = 0; u < n; ++u) cnt[u + 1] += cnt[u];
  uint64_t np = (uint64_t)cnt[n];
  uint32_t* pu = (uint32_t*)malloc((size_t)(np > 0 ? np : 1) * sizeof(uint32_t));
  uint32_t* pv = (uint32_t*)malloc((size_t)(np > 0 ? np : 1) * sizeof(uint32_t));
  if (!pu || !pv) {
    free(cnt);
    free(pu);
    free(pv);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t u = 0; u < (int64_t)n; ++u) {
    int64_t b = cnt[u];
    int64_t k = gg_er_row(n, q, lq, seed, (uint64_t)u, pv + b);
    for (int64_t i = 0; i < k; ++i) pu[b + i] = (uint32_t)u;
  }
  free(cnt);
  int rc = gg_pairs_to_csr(n, pu, pv, np, row_off, col, nnz);
  free(pu);
  free(pv);
  return rc;
}

/* -------------------------------------------------------------- R-MAT */

/* A seeded bijection of [0, 2^s): rounds of (odd multiply + add) mod 2^s and
 * a right xorshift, each of which is invertible on s-bit integers. */
typedef struct {
  uint64_t mul[4], add[4], mask;
  int sh;
} gg_perm;

static gg_perm gg_perm_make(int scale, uint64_t seed) {
  gg_perm p;
  gg_rng r = gg_stream(seed, 3, 0);
  p.mask = scale >= 64 ? ~0ull : ((1ull << scale) - 1);
  p.sh = (scale + 1) / 2;
  if (p.sh < 1) p.sh = 1;
  for (int i = 0; i < 4; ++i) {
    p.mul[i] = (gg_next(&r) | 1ull) & p.mask;
    if (p.mul[i] == 0) p.mul[i] = 1;
    p.add[i] = gg_next(&r) & p.mask;
  }
  return p;
}

static inline uint64_t gg_perm_apply(const gg_perm* p, uint64_t x) {
  for (int i = 0; i < 4; ++i) {
    x = (x * p->mul[i] + p->add[i]) & p->mask;
    x ^= x >> p->sh;
  }
  return x;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each of `samples` directed
 * samples descends `scale` levels of the adjacency matrix, picking quadrant
 * (0,0),(0,1),(1,0),(1,1) with probabilities a,b,c,d=1-a-b-c; no noise.  The
 * quadrant draw is an integer comparison of a 32-bit uniform against the
 * cumulative probabilities scaled to 2^32.  If `permute` is set, vertex ids
 * go through a seeded bijection of [0,2^scale) (as Graph500 does), and
 * endpoints >= n are rejected (n <= 2^scale).  Then symmetrize and dedup.
 */
int sg_gen_rmat(int scale, uint64_t n, uint64_t samples, double a, double b, double c, int permute,
                uint64_t seed, int64_t** row_off, uint32_t** col, uint64_t* nnz) {
  if (scale < 1 || scale > 32) return -2;
  uint64_t full = 1ull << scale;
  if (n == 0) n = full;
  if (n > full || n > 0xffffffffull) return -2;
  uint64_t ta = (uint64_t)floor(a * 4294967296.0);
  uint64_t tb = (uint64_t)floor((a + b) * 4294967296.0);
  uint64_t tc = (uint64_t)floor((a + b + c) * 4294967296.0);
  gg_perm perm = gg_perm_make(scale, seed);
  uint32_t* pu = (uint32_t*)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(uint32_t));
  uint32_t* pv = (uint32_t*)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(uint32_t));
  if (!pu || !pv) {
    free(pu);
    free(pv);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)samples; ++i) {
    gg_rng r = gg_stream(seed, 2, (uint64_t)i);
    uint64_t u = 0, v = 0, word = 0;
    for (int l = 0; l < scale; ++l) {
      if ((l & 1) == 0) word = gg_next(&r);
      uint64_t x = (l & 1) ? (word >> 32) : (word & 0xffffffffull);
      int bu, bv;
      if (x < ta) {
        bu = 0;
        bv = 0;
      } else if (x < tb) {
        bu = 0;
        bv = 1;
      } else if (x < tc) {
        bu = 1;
        bv = 0;
      } else {
        bu = 1;
        bv = 1;
      }
      u = (u << 1) | (uint64_t)bu;
      v = (v << 1) | (uint64_t)bv;
    }
    if (permute) {
      u = gg_perm_apply(&perm, u);
      v = gg_perm_apply(&perm, v);
    }
    /* endpoints >= n are dropped by gg_pairs_to_csr */
    pu[i] = u < n ? (uint32_t)u : 0xffffffffu;
    pv[i] = v < n ? (uint32_t)v : 0xffffffffu;
  }
  int rc = gg_pairs_to_csr(n, pu, pv, samples, row_off, col, nnz);
  free(pu);
  free(pv);
  return rc;
}

/* ------------------------------------------------------ many graphs */

/*
 * Generates `count` graphs at once, one graph per thread (the generators'
 * own parallel loops then run on one thread each), largest first.  Graph i
 * is G(n[i], d[i]/(n[i]-1)) with seed[i] if kind[i] == 0, else R-MAT at
 * scale[i] with n[i] vertices and samples[i] samples.  Output i is exactly
 * what the single-graph call returns.  Returns 0, or the first failing
 * graph's code (outputs of other graphs are still filled or NULL).
 */
int sg_gen_many(uint64_t count, const int32_t* kind, const uint64_t* n, const double* d,
                const uint64_t* seed, const int32_t* scale, const uint64_t* samples,
                int64_t** row_offs, uint32_t** cols, uint64_t* nnzs) {
  uint64_t* order = (uint64_t*)malloc((size_t)(count > 0 ? count : 1) * sizeof(uint64_t));
  double* work = (double*)malloc((size_t)(count > 0 ? count : 1) * sizeof(double));
  if (!order || !work) {
    free(order);
    free(work);
    return -1;
  }
  for (uint64_t i = 0; i < count; ++i) {
    order[i] = i;
    work[i] = (double)n[i] * (kind[i] == 0 ? d[i] : (double)samples[i] / (double)(n[i] ? n[i] : 1));
    row_offs[i] = NULL;
    cols[i] = NULL;
    nnzs[i] = 0;
  }
  /* largest first: insertion into a max-ordered list is fine for a few thousand */
  for (uint64_t i = 1; i < count; ++i) {
    uint64_t x = order[i];
    int64_t j = (int64_t)i - 1;
    while (j >= 0 && work[order[j]] < work[x]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = x;
  }
  int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < (int64_t)count; ++k) {
    const uint64_t i = order[k];
    int r = kind[i] == 0 ? sg_gen_er(n[i], d[i], seed[i], &row_offs[i], &cols[i], &nnzs[i])
                         : sg_gen_rmat(scale[i], n[i], samples[i], 0.57, 0.19, 0.19, 1, seed[i],
                                       &row_offs[i], &cols[i], &nnzs[i]);
    if (r != 0) {
#pragma omp critical
      if (rc == 0) rc = r;
    }
  }
  free(order);
  free(work);
  return rc;
}

/* ------------------------------------------------------ misc helpers */

/* Build a CSR from an explicit pair list (symmetrized, deduplicated). */
int sg_pairs_csr(uint64_t n, const uint32_t* pu, const uint32_t* pv, uint64_t npairs,
                 int64_t** row_off, uint32_t** col, uint64_t* nnz) {
  if (n > 0xffffffffull) return -2;
  return gg_pairs_to_csr(n, pu, pv, npairs, row_off, col, nnz);
}

/* Copy out and release buffers returned by the generators. */
void sg_copy_free(int64_t* row_off, uint32_t* col, uint64_t n, uint64_t nnz, int64_t* dst_off,
                  uint32_t* dst_col) {
  if (dst_off) memcpy(dst_off, row_off, (size_t)(n + 1) * sizeof(int64_t));
  if (dst_col && nnz) memcpy(dst_col, col, (size_t)nnz * sizeof(uint32_t));
  free(row_off);
  free(col);
}

int sg_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
