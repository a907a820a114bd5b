// Triangle listing with selection and deletion marks (Triangle p-1-Reduction,
// section 4.3: every triangle of the input graph runs kernel `p-1-reduction`
// once; a selected triangle deletes one uniformly chosen edge).
//
// Vertices are ranked by (degree, id) and every edge points from lower to
// higher rank.  A triangle y < x < w (in rank) is found exactly once, from
// its middle vertex x: the edge (y,x) is an in-edge of x, w lies in out(x)
// and in out(y) above x.  Work is organised over tiles of CSR entries: the
// rows of a tile are middle vertices, their backward entries are the
// in-edges, and their out-lists sit in an LDS hash keyed by (w, row).  Each
// in-edge (y,x) scans the part of out(y) ranked above x -- the suffix after
// x for a sorted row (binary search), the whole row for a short one -- and
// the scan items of all in-edges of a batch are spread over the lanes so
// that loads are contiguous.  Hits go to a per-wave queue and are hashed
// (Philox4x32-10 of the id-sorted triple) 64 at a time.
//
// Deletion marks: (x,w) lies in the tile's own out-lists and is collected
// in an LDS bitmap; (y,x) is a per-in-edge flag; (y,w) is a byte store into
// the global per-edge mark bytes over DAG positions (the first two are
// flushed there too).  Every mark sets a value to 1 and nothing is cleared,
// so the result does not depend on the order in which triangles are found.
//
// Variants (section 4.3), in the general instantiation of the kernel:
// Triangle p-2-Reduction marks the two edges other than the drawn one;
// Min-Count p-1-Reduction first runs a counting pass (its own instantiation:
// every triangle adds 1 to each of its edges where the probe finds it, with
// LDS counters for (y,x) and (x,w) and a global atomic for (y,w); no queue,
// no hash of the triple) and then marks, in each selected triangle, the edge
// of fewest triangles (ties: the drawn index among the tied edges).
//
// Edge-Once p-1-Reduction (section 4.3 with the conditions of section 6.2)
// runs in rounds.  Bids (pass 2 of this kernel): every selected triangle
// with no closed edge writes its priority, (Philox word 2, third vertex),
// into each of its three edges by an atomic minimum.  Acceptance (an
// edge-parallel kernel, no listing): the key on an edge names its holder
// triangle through the third vertex, and a triangle that holds the minimum
// on all three of its edges is considered -- it deletes its drawn edge and
// closes all three.  Triangles that share an edge with a considered one are
// decided against by that closed edge; an edge no undecided triangle bid on
// is closed between rounds.  The minimum of one edge compares triangles
// that differ only in their third vertex, so these per-edge keys order them
// as (word 2, a, b, c) does, and the rounds reach the set that the walk in
// that priority order reaches.  Closed in-edges are not scanned and closed
// out-list entries are not hashed, so later rounds list fewer triangles.
// Once the undecided triangles fit a list (kEoListPerEdge records per
// edge), the bidding pass that finds them appends them, and all later rounds
// run over the list (two small kernels) instead of listing triangles again;
// each of those rounds copies its bidders into a second list, which the
// next round reads, so a round costs in proportion to the undecided count.
#include <type_traits>

#include "slim_internal.h"

namespace slim {

#ifndef SLIM_TRI_BLOCK
#define SLIM_TRI_BLOCK 512
#endif
constexpr int kTB = SLIM_TRI_BLOCK;  // threads per block
constexpr int kTW = kTB / kWave;     // waves per block
constexpr int kTT = 1024;            // CSR entries per tile
constexpr int kTC = kTT / kWave;     // 64-entry chunks per tile
constexpr int kChunksPerWave = (kTC + kTW - 1) / kTW;
constexpr int kWavesPerEU = 2 * kTW / 4;  // two resident blocks per CU (LDS), four SIMDs
constexpr int kHashCap = 2048;       // out-list entries hashed per pass
constexpr int kBuckets = 2048;       // hash buckets of two slots (load <= 1/2)
constexpr int kBucketBits = 11;
constexpr int kQ = 128;              // per-wave hit queue (records)
#ifndef SLIM_TRI_UNROLL
#define SLIM_TRI_UNROLL 8
#endif
constexpr int kUnroll = SLIM_TRI_UNROLL;  // windows of 64 items whose loads are in flight together
constexpr uint32_t kEmpty = 0xffffffffu;
constexpr uint32_t kDead = 0xffffffffu;  // Edge-Once list record of a decided triangle

static_assert(kTC <= kWave && kHashCap / kWave <= kWave, "one wave scans the chunk sums and maxima");

// In-edges per batch (kB) of each instantiation: as many as two blocks per CU
// allow in LDS; the general and Edge-Once ones also keep per-in-edge counts
// or bids (larger batches cut the per-batch setup and barriers).
constexpr int kLdsPerBlock = 160 * 1024 / 2;
template <int kMode>
constexpr int kBatchOf = kMode == kModePlain ? 512 : (kMode == kModeEO ? 352 : 384);

template <int kB>
struct TriSmem {
  static_assert(kB <= kTB, "one thread per in-edge in the setup");
  uint32_t srow[kTT];  // row of each tile entry (after the max-scan)
  uint32_t cmax[kTC];
  uint16_t bw[kTT];    // local indices of the tile's backward entries, in order
  uint32_t fwd[kTT / 32];  // forward entries of the tile (edge ids come from the hash)
  uint4 hb[kBuckets + 1];     // two slots {w, tag}; tag = (position in range << 16) | row tag
  uint32_t xold[kHashCap];    // original id of each hashed out-list entry
  uint32_t xbits[kHashCap / 32 + 2];
  uint4 ie[kB];           // {scan begin, x rank, y old id, x old id}
  uint32_t ie_pre[kB + 1];
  uint32_t ie_e[kB];      // DAG position of (y,x) (kEmpty until found)
  uint4 ie_scan[kB];      // {scan begin - item base, hash tag, next in-edge start, 0}
  uint32_t ie_flag[(kB + 31) / 32];
  union {
    uint32_t dpos[kHashCap];  // row start offset of each hashed position
    uint2 queue[kTW][kQ];     // hit records {item, (in-edge << 16) | position in range}
  } u;
  uint32_t wsum[kTW];
  uint32_t cbase[kHashCap / kWave];  // per chunk: bw slots of the tile, or row offset maxima of the hashed range
  uint64_t cmask[kTC];
  uint32_t bcast[4];
  uint64_t red[2][kTW];
};

template <int kB>
struct TriSmemPlain {
  TriSmem<kB> s;
};
// LDS of the general instantiation: per-edge triangle counts of the hashed
// range and of the batch's in-edges (accumulated in the counting pass, loaded
// for the Min-Count selection).
template <int kB>
struct TriSmemGeneral {
  TriSmem<kB> s;
  uint32_t xcnt[kHashCap];
  uint32_t ie_cnt[kB];
};
// LDS of the Edge-Once instantiation: the smallest bid on each in-edge of
// the batch, written to the global minimum once per batch, and the smallest
// priority word bid on each hashed out-list entry in the current pass.
template <int kB>
struct TriSmemEO {
  TriSmem<kB> s;
  uint64_t ie_key[kB];
  uint32_t xmin[kHashCap];
};

// A key is (w, row tag) with row tag = 16 x (offset of the row's start in
// the hashed range), below 2^15; bucket addresses are byte offsets (16 B per
// bucket).  A slot's tag word holds (position in range << 16) | row tag, and
// bit 31 of a bucket's second tag word (kPassed) is set once an insertion
// found the bucket full and went on past it.
constexpr uint32_t kRowTag = 4;             // row tag = row offset << kRowTag
constexpr uint32_t kPassed = 0x80000000u;
constexpr uint32_t kQposMask = 0x7fffu;     // position in range, from tag >> 16
constexpr uint32_t kNoRow = 0xffffu;        // a row tag no key has

// Byte offset of the home bucket of key (w, row tag g), below 16 kBuckets:
// bits 21..31 of w * 0x9E3779B1 xor the row offset, times 16.
__device__ __forceinline__ uint32_t hhome(uint32_t w, uint32_t g) {
  return (((w * 0x9E3779B1u) >> (32 - kBucketBits - kRowTag)) ^ g) &
         ((kBuckets - 1) << kRowTag);
}

// Probe order: home buckets are 0 .. kBuckets-1; the walk goes on to the
// spare bucket kBuckets and then wraps to 0, so a home bucket and the next
// one are always adjacent in LDS.  b is a byte offset.
__device__ __forceinline__ uint32_t hnext(uint32_t b) {
  return b == (kBuckets << kRowTag) ? 0u : b + (1u << kRowTag);
}

__device__ __forceinline__ uint4 hread(const uint4* hb, uint32_t b) {
  return *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(hb) + b);
}

// Look up (w, row tag g).  Slots fill in probe order and are never removed,
// so the key lies past a bucket only if an insertion went on past it.
__device__ __forceinline__ bool hlookup(const uint4* hb, uint32_t w, uint32_t g,
                                        uint32_t& qpos) {
  uint32_t b = hhome(w, g);
  for (;;) {
    const uint4 e = hread(hb, b);
    if (e.x == w && (e.y & 0xffffu) == g) {
      qpos = (e.y >> 16) & kQposMask;
      return true;
    }
    if (e.z == w && (e.w & 0xffffu) == g) {
      qpos = (e.w >> 16) & kQposMask;
      return true;
    }
    if (!(e.w & kPassed)) return false;
    b = hnext(b);
  }
}

// First position in the sorted DAG range [lo, hi) whose rank id is >= x
// (the entry x itself in a valid input; hi if every entry is below x).  The
// fence samples of the line starts inside the range pick the one 128-byte
// line of dag_col that holds the answer, and the halving ends inside it: a
// search of a long row reads its samples (one or two lines) and one line of
// dag_col, instead of a new line for each of its first halvings.
__device__ __forceinline__ uint32_t dag_find(const TriArgs& a, uint32_t lo, uint32_t hi,
                                             uint32_t x) {
  static_assert(kFenceStep == 32, "line starts are multiples of 32 positions");
  // line starts 32q inside [lo, hi): q in [qa, qe)
  const uint32_t qa = (lo >> 5) + ((lo & 31u) != 0), qe = (hi >> 5) + ((hi & 31u) != 0);
  if (qa < qe) {
    uint32_t l = qa, h = qe;  // first q whose line starts above x
    while (l < h) {
      const uint32_t mid = l + ((h - l) >> 1);
      if (a.fence[mid] <= x)
        l = mid + 1;
      else
        h = mid;
    }
    if (l > qa) lo = (l - 1) << 5;  // the line of the last start at or below x
    const uint64_t lend = (uint64_t)l << 5;
    if (lend < hi) hi = (uint32_t)lend;
  }
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (a.dag_col[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row of every entry of the tile [j0, j0 + kTT): srow[i] after the scan.
template <int kB>
__device__ void tri_tile_rows(const int64_t* row_off, int64_t j0, uint32_t lo, uint32_t hi,
                              TriSmem<kB>& S) {
  const int t = threadIdx.x, w = t / kWave, lane = lane_id();
  for (int i = t; i < kTT; i += kTB) S.srow[i] = 0;
  __syncthreads();
  if (t == 0) S.srow[0] = lo > 0 ? lo - 1 : 0;
  __syncthreads();
  for (uint64_t r = lo + (uint64_t)t; r < hi; r += kTB) {
    const int64_t b = row_off[r], e = row_off[r + 1];
    const int64_t s = b - j0;
    if (e > b && s >= 0 && s < kTT) S.srow[s] = r;
  }
  __syncthreads();
  for (int c = w; c < kTC; c += kTW) {
    const uint32_t v = wave_incl_max(S.srow[c * kWave + lane]);
    S.srow[c * kWave + lane] = v;
    if (lane == kWave - 1) S.cmax[c] = v;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t v = lane < kTC ? S.cmax[lane] : 0;
    const uint32_t incl = wave_incl_max(v);
    uint32_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0;
    if (lane < kTC) S.cmax[lane] = excl;
  }
  __syncthreads();
  for (int i = t; i < kTT; i += kTB) {
    const uint32_t a = S.srow[i], b = S.cmax[i >> 6];
    S.srow[i] = a > b ? a : b;
  }
  __syncthreads();
}

struct TriCtx {
  TriArgs a;
  uint32_t* xcnt;    // general instantiation only: per-edge counts of the hashed range
  uint32_t* ie_cnt;  //   and of the batch's in-edges
  uint64_t* ie_key;  // Edge-Once instantiation only
  uint32_t* xmin;    // Edge-Once instantiation only
  uint32_t cap;   // out-list entries hashed per pass (<= kHashCap)
  int64_t j0;
  uint32_t D0;    // first DAG position of the hashed range
  uint32_t hlen;  // number of hashed entries
  uint64_t thr;   // the tile's graph: selection threshold, Philox key, first vertex
  uint32_t k0, k1, vb;
  uint32_t op;    // the tile's graph's operation
  bool eo_later;  // an Edge-Once pass after the first bids: eids are known, closed edges skipped
  bool eo_append; // an Edge-Once bidding pass that also lists the bidding triangles
  uint64_t wcur;  // Edge-Once list slots reserved by this wave: next free one
  uint32_t wleft; //   and how many are left (the same in every lane of the wave)
  uint32_t achunk;  // slots a wave reserves at a time
  uint64_t n_tri, n_sel;
};

// Hash the out-list entries [D0, D0 + len) under key (w, row tag); the row
// start offset comes from dpos (all rows of the tile) or is 0 (one row).
template <int kB>
__device__ void tri_build_hash(TriCtx& C, TriSmem<kB>& S, uint32_t len, bool use_dpos) {
  for (int i = threadIdx.x; i < kBuckets + 1; i += kTB)
    S.hb[i] = make_uint4(kEmpty, 0u, kEmpty, 0u);
  for (int i = threadIdx.x; i < kHashCap / 32 + 2; i += kTB) S.xbits[i] = 0;
  __syncthreads();
  uint32_t* hw = reinterpret_cast<uint32_t*>(S.hb);
  const bool skip_closed = C.eo_later;
  for (uint32_t q = threadIdx.x; q < len; q += kTB) {
    const uint32_t w = C.a.dag_col[C.D0 + q];
    S.xold[q] = C.a.order[w];
    if (C.xmin) C.xmin[q] = 0xffffffffu;
    // Edge-Once rounds after the first pass: a closed edge {x,w} decides
    // every triangle on it, so it is left out of the hash
    if (skip_closed && bit_get(C.a.closed, C.D0 + q)) continue;
    const uint32_t g = (use_dpos ? S.u.dpos[q] : 0u) << kRowTag;
    uint32_t b = hhome(w, g);
    for (;;) {
      uint32_t* s = hw + b / 4;
      // tags are ORed in: an insertion passing the bucket may set kPassed
      // in the second tag word at the same time
      if (atomicCAS(&s[0], kEmpty, w) == kEmpty) {
        atomicOr(&s[1], (q << 16) | g);
        break;
      }
      if (atomicCAS(&s[2], kEmpty, w) == kEmpty) {
        atomicOr(&s[3], (q << 16) | g);
        break;
      }
      atomicOr(&s[3], kPassed);
      b = hnext(b);
    }
    // counts exist only for Min-Count graphs: loaded for their selection
    // pass, zeroed for their counting pass (other operations never read them)
    if (C.xcnt) C.xcnt[q] = C.a.pass == 1 && C.op == SLIM_OP_MCTR ? C.a.tcount[C.D0 + q] : 0u;
  }
  C.hlen = len;
  __syncthreads();
}

template <int kB>
__device__ void tri_flush_xbits(TriCtx& C, TriSmem<kB>& S) {
  __syncthreads();
  if (C.xcnt && C.a.pass == 0) {  // counting pass: add the (x,w) counts of the range
    for (uint32_t q = threadIdx.x; q < C.hlen; q += kTB) {
      const uint32_t v = C.xcnt[q];
      if (v) atomicAdd(C.a.tcount + C.D0 + q, v);
    }
  } else {
    const uint32_t nwords = (C.D0 % 32 + C.hlen + 31) / 32;
    const uint32_t base = C.D0 / 32;
    for (uint32_t i = threadIdx.x; i < nwords; i += kTB)
      for (uint32_t v = S.xbits[i]; v; v &= v - 1) mark_set(C.a.marks, (base + i) * 32u + __builtin_ctz(v));
  }
  __syncthreads();
}

// Forward entries among tile entries [ia, ib): their edge is in out(x) of the
// entry's own row, so the DAG position comes from the hash (a miss means the
// entry lies in another pass of a split row).
template <int kB>
__device__ void tri_forward_eids(TriCtx& C, TriSmem<kB>& S, uint32_t ia, uint32_t ib,
                                 bool all_rows) {
  if (C.hlen == 0) return;
  for (uint32_t i = ia + threadIdx.x; i < ib; i += kTB) {
    if (!(S.fwd[i >> 5] & (1u << (i & 31)))) continue;
    const uint64_t j = (uint64_t)C.j0 + i;
    const uint32_t w = C.a.rcol[j];
    const uint32_t g = all_rows ? (C.a.fstart[S.srow[i]] - C.D0) << kRowTag : 0u;
    uint32_t qpos;
    if (hlookup(S.hb, w, g, qpos)) C.a.eid[j] = C.D0 + qpos;
  }
}

// Marks the edge of triangle (y,x,w) that does not contain vertex `excl`
// (union ids: c = y, u0 = x, ow = w).
template <int kB>
__device__ __forceinline__ void tri_mark(uint8_t* marks, TriSmem<kB>& S, uint32_t excl, uint32_t c,
                                         uint32_t ow, uint32_t k, uint32_t qpos, uint32_t D0,
                                         uint32_t p_yw) {
  if (excl == ow) {  // edge {y,x}: flag of the in-edge
    atomicOr(&S.ie_flag[k >> 5], 1u << (k & 31));
  } else if (excl == c) {  // edge {x,w}: position qpos of the hashed range
    const uint32_t bit = D0 % 32 + qpos;
    atomicOr(&S.xbits[bit >> 5], 1u << (bit & 31));
  } else {  // edge {y,w}: a byte store (nothing waits on it)
    mark_set(marks, p_yw);
  }
}

// Edge-Once bid: lowers *p to key; the plain load skips the atomic when the
// edge already holds a smaller key (values only decrease within a pass).
__device__ __forceinline__ void eo_bid(uint64_t* p, uint64_t key) {
  if (key < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    __hip_atomic_fetch_min(p, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Edge-Once drain of the queued hits q[head .. head + cnt) (cnt <= 64): a
// selected triangle with no closed edge bids its per-edge keys.  In the
// bidding pass that starts the triangle list, every bidding triangle is
// also appended to the list (one counter atomic per wave).  Returns 1 in
// lanes that bid.
template <int kB>
__device__ __forceinline__ uint32_t tri_drain_eo(TriCtx& C, TriSmem<kB>& S, const uint2* q,
                                                 uint32_t head, uint32_t cnt) {
  const uint32_t lane = lane_id();
  uint32_t res = 0;
  bool app = false;
  uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = ra;
  if (lane < cnt) {
    const uint2 rec = q[(head + lane) % kQ];
    const uint32_t k = rec.y >> 16, qpos = rec.y & kQposMask;
    const uint4 ie = S.ie[k];
    const uint32_t p_yw = ie.x + (rec.x - S.ie_pre[k]);
    const uint32_t ow = S.xold[qpos];
    const uint32_t c = ie.z, u0 = ie.w;
    uint32_t t0 = c, t1 = u0, t2 = ow;
    sort3(t0, t1, t2);  // union ids of one graph: the order of its local ids
    const uint4 wr = philox4(t0 - C.vb, t1 - C.vb, t2 - C.vb, 0u, C.k0, C.k1);
    // the in-edge and the hashed entry are open (closed ones are neither
    // scanned nor hashed); {y,w} is read here
    const bool open = (uint64_t)wr.x < C.thr && !(C.eo_later && bit_get(C.a.closed, p_yw));
    if (open) {
      // per-edge keys (word 2, third vertex): {y,x} -> w, {x,w} -> y, {y,w} -> x
      const uint64_t hi = (uint64_t)wr.z << 32;
      const uint32_t e_yx = S.ie_e[k], e_xw = C.D0 + qpos;
      const uint32_t lw = ow - C.vb, ly = c - C.vb, lx = u0 - C.vb;
      const uint64_t k_yx = hi | lw, k_xw = hi | ly, k_yw = hi | lx;
      uint64_t* mk = C.a.minkey;
      const uint32_t kk = __umulhi(wr.y, 3u);  // edge kk of ({t0,t1}, {t0,t2}, {t1,t2})
      const uint32_t excl = kk == 0 ? t2 : (kk == 1 ? t1 : t0);
      atomicMin((unsigned long long*)&C.ie_key[k], (unsigned long long)k_yx);  // LDS
      // {x,w} lies in the hashed range: a bid whose priority word is above
      // the smallest one this pass has bid on the entry cannot hold the
      // minimum (that one went to the global key), so only the others bid
      if (wr.z <= atomicMin(&C.xmin[qpos], wr.z)) eo_bid(mk + e_xw, k_xw);
      eo_bid(mk + p_yw, k_yw);
      res = 1;
      app = true;
      ra = make_uint4(e_yx, e_xw, p_yw, excl == ow ? e_yx : (excl == c ? e_xw : p_yw));
      rb = make_uint4(wr.z, lw, ly, lx);
    }
  }
  if (C.eo_append) {  // the same in every lane of the block
    // slots come from the wave's reserved run first; the rest from a new run
    // of max(rest, achunk) slots, taken with one atomic on the list counter
    const uint64_t mask = __ballot(app);
    if (mask) {
      const uint32_t n = __popcll(mask), r = __popcll(mask & lanemask_lt());
      const uint32_t take0 = n < C.wleft ? n : C.wleft;
      const uint64_t base0 = C.wcur;
      uint64_t base1 = 0;
      if (n > take0) {
        const uint32_t need = n - take0, run = need > C.achunk ? need : C.achunk;
        unsigned long long nb = 0;
        if (lane == 0) nb = atomicAdd((unsigned long long*)C.a.eo_list_cnt, (unsigned long long)run);
        base1 = __shfl(nb, 0, kWave);
        C.wcur = base1 + need;
        C.wleft = run - need;
      } else {
        C.wcur += n;
        C.wleft -= n;
      }
      const uint64_t idx = r < take0 ? base0 + r : base1 + (r - take0);
      if (app && idx < C.a.eo_cap) {
        C.a.eo_list[2 * idx] = ra;
        C.a.eo_list[2 * idx + 1] = rb;
      }
    }
  }
  return res;
}

// Hash, select and mark the queued hits q[head .. head + cnt) (cnt <= 64);
// one lane per hit.  Returns 1 in lanes whose triangle was selected.
template <int kMode, int kB>
__device__ __forceinline__ uint32_t tri_drain(TriCtx& C, TriSmem<kB>* Sp, const uint2* q,
                                              uint32_t head, uint32_t cnt) {
  constexpr bool kGeneral = kMode == kModeGeneral, kEO = kMode == kModeEO;
  if constexpr (kEO) return tri_drain_eo(C, *Sp, q, head, cnt);
  TriSmem<kB>& S = *Sp;
  const uint32_t lane = lane_id();
  uint32_t sel = 0;
  if (lane < cnt) {
    const uint2 rec = q[(head + lane) % kQ];
    const uint32_t k = rec.y >> 16, qpos = rec.y & kQposMask;
    const uint4 ie = S.ie[k];
    const uint32_t p_yw = ie.x + (rec.x - S.ie_pre[k]);
    const uint32_t ow = S.xold[qpos];
    const uint32_t c = ie.z, u0 = ie.w;
    uint32_t t0 = c, t1 = u0, t2 = ow;
    sort3(t0, t1, t2);  // union ids of one graph: the order of its local ids
    const uint4 wr = philox4(t0 - C.vb, t1 - C.vb, t2 - C.vb, 0u, C.k0, C.k1);
    const uint32_t w0 = wr.x, w1 = wr.y;
    if ((uint64_t)w0 < C.thr) {
      sel = 1;
      // edge e of ({t0,t1}, {t0,t2}, {t1,t2}) is the one without excl[e]
      const uint32_t excl[3] = {t2, t1, t0};
      if constexpr (!kGeneral) {
        tri_mark(C.a.marks, S, excl[__umulhi(w1, 3u)], c, ow, k, qpos, C.D0, p_yw);
      } else if (C.op == SLIM_OP_MCTR) {
        uint32_t t[3];
#pragma unroll
        for (int e = 0; e < 3; ++e)
          t[e] = excl[e] == ow ? C.ie_cnt[k]
                               : (excl[e] == c ? C.xcnt[qpos] : C.a.tcount[p_yw]);
        const uint32_t tmin = min(t[0], min(t[1], t[2]));
        const uint32_t nt = (t[0] == tmin) + (t[1] == tmin) + (t[2] == tmin);
        uint32_t pick = __umulhi(w1, nt), e = 0;
        for (; e < 3; ++e) {
          if (t[e] != tmin) continue;
          if (pick == 0) break;
          --pick;
        }
        tri_mark(C.a.marks, S, excl[e], c, ow, k, qpos, C.D0, p_yw);
      } else {
        const uint32_t kk = __umulhi(w1, 3u);
#pragma unroll
        for (int e = 0; e < 3; ++e)
          if ((C.op == SLIM_OP_TR2) ? (uint32_t)e != kk : (uint32_t)e == kk)
            tri_mark(C.a.marks, S, excl[e], c, ow, k, qpos, C.D0, p_yw);
      }
    }
  }
  return sel;
}

// Process the in-edges bw[b0, b1) of the tile against the current hash.
template <int kMode, int kB>
__device__ void tri_batch(TriCtx& C, TriSmem<kB>& S, uint32_t b0, uint32_t b1, bool all_rows) {
  constexpr bool kGeneral = kMode == kModeGeneral, kCount = kMode == kModeCount;
  const int tid = threadIdx.x;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t lane = lane_id();
  const uint32_t nin = b1 - b0;
  // ---- setup: one thread per in-edge (y,x); x is found in sorted out(y) by
  // binary search, and the items are the entries of out(y) after it
  uint32_t cnt = 0, bmp = 0, xtag = 0;
  if ((uint32_t)tid < nin) {
    const uint32_t i = S.bw[b0 + tid];
    const uint64_t j = (uint64_t)C.j0 + i;
    const uint32_t r = S.srow[i];
    const uint32_t c = C.a.col[j];
    const uint32_t y = C.a.rcol[j];
    const uint32_t x = C.a.rank[r];
    const uint2 yr = C.a.dag_rng[y];
    const uint32_t fs = C.a.fstart[r], fe = C.a.fstart[r + 1];
    uint32_t e;
    bool closed = false;
    if (C.eo_later) {  // found by the first Edge-Once pass
      e = C.a.eid[j];
      closed = bit_get(C.a.closed, e);
    } else {
      e = dag_find(C.a, yr.x, yr.y, x);  // dag_col[e] == x
      C.a.eid[j] = e;
    }
    // out(x) empty: no triangle, no scan (e == yr.y only for inputs that
    // break the CSR contract: then nothing is scanned either); a closed
    // in-edge of an Edge-Once round is not scanned
    const uint32_t beg = fe > fs && e < yr.y && !closed ? e + 1 : yr.y;
    cnt = yr.y - beg;
    xtag = all_rows ? (fs - C.D0) << kRowTag : 0u;
    S.ie[tid] = make_uint4(beg, x, c, r);
    S.ie_e[tid] = e;
    if (kGeneral) C.ie_cnt[tid] = C.op == SLIM_OP_MCTR ? C.a.tcount[e] : 0u;
    if (kCount) C.ie_cnt[tid] = 0u;
    bmp = beg;
  }
  if ((uint32_t)tid < (kB + 31) / 32) S.ie_flag[tid] = 0;
  if (C.ie_key && (uint32_t)tid < nin) C.ie_key[tid] = ~0ull;
  {  // block exclusive scan of cnt into ie_pre; scan records {beg - pre, tag, next start}
    const uint64_t incl = wave_incl_sum64(cnt);
    if (lane == kWave - 1) S.wsum[w] = (uint32_t)incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int i = 0; i < kTW; ++i) {
      if ((uint32_t)i < w) before += S.wsum[i];
      all += S.wsum[i];
    }
    const uint32_t pre = before + (uint32_t)incl - cnt;
    if ((uint32_t)tid < nin) {
      S.ie_pre[tid] = pre;
      S.ie_scan[tid] = make_uint4(bmp - pre, xtag, pre + cnt, 0u);
    }
    if (tid == 0) S.ie_pre[nin] = all;
    __syncthreads();
  }
  const uint32_t W = __builtin_amdgcn_readfirstlane(S.ie_pre[nin]);
  // ---- items: wave w takes the contiguous range [ws, we).  The current
  // in-edge's fields stay in scalar registers; a window of 64 items crosses
  // an in-edge boundary only now and then (a short scalar loop).
  const uint32_t ws = (uint32_t)(((uint64_t)W * w) / kTW);
  const uint32_t we = (uint32_t)(((uint64_t)W * (w + 1)) / kTW);
  uint2* q = S.u.queue[w];
  uint32_t qhead = 0, qcnt = 0;
  uint32_t kcur = 0;
  if (ws < we) {  // in-edge holding item ws: last k with ie_pre[k] <= ws
    uint32_t lo = 0, hi = nin;
    while (hi - lo > 1) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (S.ie_pre[mid] <= ws)
        lo = mid;
      else
        hi = mid;
    }
    kcur = lo;
  }
  kcur = __builtin_amdgcn_readfirstlane(kcur);
  uint32_t c_bmp, c_tag, c_nxt;  // scan begin - item base, hash tag, next in-edge start
  auto fetch = [&](uint32_t k) {
    const uint4 r = S.ie_scan[k];
    c_bmp = __builtin_amdgcn_readfirstlane(r.x);
    c_tag = __builtin_amdgcn_readfirstlane(r.y);
    c_nxt = __builtin_amdgcn_readfirstlane(r.z);
  };
  fetch(kcur);
  for (uint32_t wb = ws; wb < we; wb += kWave * kUnroll) {
    uint32_t kk[kUnroll], xb[kUnroll], wv[kUnroll], ad[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t base = wb + u * kWave;
      const uint32_t t = base + lane;
      uint32_t k = kcur, g = c_tag, p = c_bmp + t;  // p: DAG position of the item (edge {y,w})
      const uint32_t lim = base + kWave < we ? base + kWave : we;
      while (c_nxt < lim) {  // the next in-edge starts inside this window
        const uint32_t bound = c_nxt;
        ++kcur;
        fetch(kcur);
        const bool after = t >= bound;
        k = after ? kcur : k;
        p = after ? c_bmp + t : p;
        g = after ? c_tag : g;
      }
      // a lane past the range gets row tag kNoRow, which no hashed key has
      // (row tags are multiples of 16): it never hits
      kk[u] = k;
      xb[u] = t < we ? g : kNoRow;
      ad[u] = t < we ? p : 0u;
      wv[u] = C.a.dag_col[ad[u]];
    }
    // Probe window by window: the home bucket and the next one (four slots,
    // read together); a key can only sit further on if an insertion went on
    // past the second one (its kPassed bit).  The
    // SIMDs issue vector instructions in most cycles of this loop, so the
    // probe is written for few of them: one compare per slot key, the row
    // tag of the first slot holding w, and the rare cases (the same w in
    // another row of the tile, two full buckets) as divergent branches,
    // which the exec mask skips when no lane takes them.
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t bku = hhome(wv[u], xb[u]);
      const uint4 e = hread(S.hb, bku);
      const uint4 f = hread(S.hb, bku + (1u << kRowTag));  // adjacent: the spare bucket follows the last
      const uint32_t t = wb + u * kWave + lane, wq = wv[u], g = xb[u];
      const bool k0 = e.x == wq, k1 = e.z == wq, k2 = f.x == wq;
      uint32_t tsel = f.w;
      tsel = k2 ? f.y : tsel;
      tsel = k1 ? e.w : tsel;
      tsel = k0 ? e.y : tsel;
      const bool kany = (k0 | k1 | k2) || f.z == wq;
      const bool rowok = (tsel & 0xffffu) == g;
      bool hit = kany & rowok;
      uint32_t qpos = tsel >> 16;  // kPassed may ride along in bit 15: masked where it is used
      bool more = !kany & ((int32_t)f.w < 0);
      if (kany & !hit) {  // w is hashed for another row too: check all four slots
        const bool m0 = k0 & ((e.y & 0xffffu) == g);
        const bool m1 = k1 & ((e.w & 0xffffu) == g);
        const bool m2 = k2 & ((f.y & 0xffffu) == g);
        const bool m3 = (f.z == wq) & ((f.w & 0xffffu) == g);
        hit = m0 | m1 | m2 | m3;
        qpos = (m0 ? e.y : m1 ? e.w : m2 ? f.y : f.w) >> 16;
        more = !hit & ((int32_t)f.w < 0);
      }
      uint32_t bkt = bku + (1u << kRowTag);
      while (more) {  // an insertion went on past both buckets: keep probing (rare)
        bkt = hnext(bkt);
        const uint4 h = hread(S.hb, bkt);
        const bool n0 = (h.x == wq) & ((h.y & 0xffffu) == g);
        const bool n1 = (h.z == wq) & ((h.w & 0xffffu) == g);
        hit = n0 | n1;
        qpos = (n0 ? h.y : h.w) >> 16;
        more = !(n0 | n1) & ((int32_t)h.w < 0);
      }
      if constexpr (kCount) {  // one more triangle on each of its three edges
        if (hit) {
          atomicAdd(&C.xcnt[qpos & kQposMask], 1u);
          atomicAdd(C.a.tcount + ad[u], 1u);
        }
        // {y,x}: the hits of one in-edge add together (a window rarely
        // holds more than one or two in-edges)
        uint64_t rem = __ballot(hit);
        while (rem) {
          const int src = __builtin_ctzll(rem);
          const uint32_t ks = __shfl(kk[u], src, kWave);
          const uint64_t same = __ballot(hit && kk[u] == ks);
          if ((int)lane == src) atomicAdd(&C.ie_cnt[ks], (uint32_t)__popcll(same));
          rem &= ~same;
        }
        continue;
      }
      const uint64_t bal = __builtin_amdgcn_ballot_w64(hit);
      if (bal) {
        const uint32_t before = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (hit) q[(qhead + qcnt + before) % kQ] = make_uint2(t, (kk[u] << 16) | qpos);
        qcnt += __popcll(bal);
        if (qcnt >= (uint32_t)kWave) {
          wave_sync();
          C.n_sel += tri_drain<kMode, kB>(C, &S, q, qhead, kWave);
          C.n_tri += 1;
          qhead = (qhead + kWave) % kQ;
          qcnt -= kWave;
        }
      }
    }
  }
  if (qcnt) {
    wave_sync();
    C.n_sel += tri_drain<kMode, kB>(C, &S, q, qhead, qcnt);
    C.n_tri += lane < qcnt ? 1 : 0;
  }
  __syncthreads();
  // ---- finish: (y,x) marks, or the (y,x) counts of the counting pass
  if (kCount) {
    if ((uint32_t)tid < nin && C.ie_cnt[tid]) atomicAdd(C.a.tcount + S.ie_e[tid], C.ie_cnt[tid]);
  } else if ((uint32_t)tid < nin && (S.ie_flag[tid >> 5] & (1u << (tid & 31)))) {
    mark_set(C.a.marks, S.ie_e[tid]);
  }
  if (C.ie_key && (uint32_t)tid < nin && C.ie_key[tid] != ~0ull)  // the batch's {y,x} bids
    eo_bid(C.a.minkey + S.ie_e[tid], C.ie_key[tid]);
  __syncthreads();
}

// Adds the block's triangle and selection counts to graph g's counters.
// Edge-Once bids add the undecided triangles to the round's counter (and,
// in the first round, T and the selected count to the graph's counters);
// acceptance passes report nothing.
template <int kB>
__device__ void tri_flush_counts(TriCtx& C, TriSmem<kB>& S, uint32_t g) {
  const int tid = threadIdx.x, w = tid / kWave;
  const uint64_t s0 = wave_sum64(C.n_tri), s1 = wave_sum64(C.n_sel);
  const bool first = C.a.pass < 2 || (C.a.pass == 2 && C.a.round == 1);
  if (lane_id() == 0) {
    S.red[0][w] = s0;
    S.red[1][w] = s1;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t t0 = 0, t1 = 0;
    for (int i = 0; i < kTW; ++i) {
      t0 += S.red[0][i];
      t1 += S.red[1][i];
    }
    if (first && t0) atomicAdd((unsigned long long*)&C.a.counters[2 * g], (unsigned long long)t0);
    if (first && t1)
      atomicAdd((unsigned long long*)&C.a.counters[2 * g + 1], (unsigned long long)t1);
    if (C.a.pass == 2 && t1)
      atomicAdd((unsigned long long*)&C.a.eo_und[C.a.round], (unsigned long long)t1);
  }
  __syncthreads();
  C.n_tri = 0;
  C.n_sel = 0;
}

// Persistent blocks take tiles in increasing order from a counter, so the
// graph of a block's tiles never decreases: counts are flushed when it
// changes and at the end.
template <int kMode>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(kWavesPerEU))) void k_triangles(
    TriArgs a, uint32_t* tile_ctr, uint32_t cap) {
  constexpr bool kGeneral = kMode == kModeGeneral, kEO = kMode == kModeEO;
  constexpr bool kCount = kMode == kModeCount;
  constexpr int kB = kBatchOf<kMode>;
  using Smem = std::conditional_t<kGeneral || kCount, TriSmemGeneral<kB>,
                                  std::conditional_t<kEO, TriSmemEO<kB>, TriSmemPlain<kB>>>;
  static_assert(sizeof(Smem) <= kLdsPerBlock, "two blocks per CU share the LDS");
  __shared__ Smem SS;
  TriSmem<kB>& S = SS.s;
  TriCtx C;
  C.a = a;
  if constexpr (kGeneral || kCount) {
    C.xcnt = SS.xcnt;
    C.ie_cnt = SS.ie_cnt;
  } else {
    C.xcnt = nullptr;
    C.ie_cnt = nullptr;
  }
  if constexpr (kEO) {
    C.ie_key = SS.ie_key;
    C.xmin = SS.xmin;
  } else {
    C.ie_key = nullptr;
    C.xmin = nullptr;
  }
  C.cap = cap;
  C.op = 0;
  C.n_tri = 0;
  C.n_sel = 0;
  C.thr = 0;
  C.k0 = C.k1 = C.vb = 0;
  C.eo_later = kEO && a.round > 1;
  C.eo_append = false;
  // Edge-Once rounds end once a bidding pass finds no undecided triangle:
  // bids of round r stop if round r-1 had none, acceptance if round r has
  // none.  Once the undecided triangles may fit the list (round r-1 had at
  // most eo_list_try percent of its capacity), the bidding pass of round r also
  // lists them; if they fit, later rounds run on the list instead of listing
  // triangles again, else the list is dropped at the start of round r+1.
  if (kEO) {
    if (a.round > 1 && a.eo_und[a.round - 1] == 0) return;
    const uint32_t listed = a.eo_state[0];
    if (listed != 0 && listed < a.round) return;
    // every wave may leave up to achunk reserved slots unused (marked dead
    // at the end); they count against the capacity like the triangles
    const uint64_t waves = (uint64_t)gridDim.x * kTW;
    const uint64_t ch = a.eo_cap / (8 * waves);
    C.achunk = (uint32_t)(ch < 256 ? ch : 256);
    C.wcur = 0;
    C.wleft = 0;
    // (another block of this pass may already have recorded the round)
    C.eo_append = a.round >= 2 && (listed == 0 || listed == a.round) &&
                  a.eo_und[a.round - 1] * 100 <= (uint64_t)a.eo_list_try * a.eo_cap;
    if (C.eo_append && threadIdx.x == 0) a.eo_state[0] = a.round;
  }
  const int tid = threadIdx.x, w = tid / kWave;
  const uint32_t lane = lane_id();
  const uint64_t ntiles = a.ntiles;
  uint32_t gcur = 0xffffffffu;
  for (;;) {
    if (tid == 0) S.bcast[0] = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint64_t t = S.bcast[0];
    __syncthreads();
    if (t >= ntiles) break;
    const TileRec R = a.recs[t];
    if (R.span == 0) continue;  // a graph without edges
    const uint32_t gop = a.gd[R.g].op;
    // tiles of graphs that list no triangles are skipped; the counting pass
    // visits Min-Count graphs only, the Edge-Once passes Edge-Once graphs only
    if (!op_lists_triangles(gop)) continue;
    if (kEO ? gop != SLIM_OP_EOTR
            : (kCount ? gop != SLIM_OP_MCTR : gop == SLIM_OP_EOTR))
      continue;
    if (R.g != gcur) {
      // the counting pass reports no triangle or selection counts
      if (gcur != 0xffffffffu && !kCount) tri_flush_counts(C, S, gcur);
      gcur = R.g;
      const GDesc& G = a.gd[gcur];
      C.thr = G.thr;
      C.k0 = G.k0;
      C.k1 = G.k1;
      C.vb = (uint32_t)G.vb;
      C.op = G.op;
    }
    // Edge-Once: a tile lists the same triangles in every pass, so one that
    // found no undecided triangle in a bidding pass has none later either
    if (kEO && C.eo_later && a.eo_live[t] + 1u < a.round) continue;
    const uint64_t sel0 = C.n_sel;
    const int64_t j0 = R.j0;
    const uint32_t span = R.span;
    C.j0 = j0;
    tri_tile_rows(a.row_off, j0, R.lo, R.hi, S);
    // ---- backward entries (the in-edges of the tile's rows), in CSR order
    uint32_t fb = 0;
    for (int k = 0; k < kChunksPerWave; ++k) {
      const int c = w + k * kTW;
      if (c >= kTC) break;
      const uint32_t i = c * kWave + lane;
      bool f = false, g = false;
      if (i < span) {
        const uint32_t rc = a.rcol[j0 + i], rr = a.rank[S.srow[i]];
        f = rc < rr;
        g = rc > rr;
      }
      const uint64_t m = __ballot(f);
      const uint64_t mf = __ballot(g);
      if (lane == 0) {
        S.cmask[c] = m;
        S.fwd[2 * c] = (uint32_t)mf;
        S.fwd[2 * c + 1] = (uint32_t)(mf >> 32);
      }
      if (f) fb |= 1u << k;
    }
    __syncthreads();
    if (w == 0) {
      const uint32_t v = lane < kTC ? __popcll(S.cmask[lane]) : 0;
      const uint64_t incl = wave_incl_sum64(v);
      if (lane < kTC) S.cbase[lane] = (uint32_t)(incl - v);
      if (lane == kWave - 1) S.bcast[1] = (uint32_t)incl;
    }
    __syncthreads();
    for (int k = 0; k < kChunksPerWave; ++k) {
      if (fb & (1u << k)) {
        const int c = w + k * kTW;
        S.bw[S.cbase[c] + __popcll(S.cmask[c] & lanemask_lt())] = (uint16_t)(c * kWave + lane);
      }
    }
    const uint32_t nbw = S.bcast[1];
    __syncthreads();
    const uint32_t r_lo = S.srow[0], r_hi = S.srow[span - 1];
    const uint32_t D0 = a.fstart[r_lo], D1 = a.fstart[r_hi + 1];
    const bool all_rows = D1 - D0 <= C.cap;
    if (all_rows) {
      // ---- all rows of the tile share one hash: row start offset per position
      const uint32_t len = D1 - D0;
      for (uint32_t i = tid; i < len; i += kTB) S.u.dpos[i] = 0;
      __syncthreads();
      for (uint64_t r = r_lo + (uint64_t)tid; r <= r_hi; r += kTB) {
        const uint32_t fs = a.fstart[r], fe = a.fstart[r + 1];
        if (fe > fs) S.u.dpos[fs - D0] = fs - D0;
      }
      __syncthreads();
      const uint32_t nc = (len + kWave - 1) / kWave;
      for (uint32_t c = w; c < nc; c += kTW) {  // max-scan: chunk scans, then carry
        const uint32_t i = c * kWave + lane;
        const uint32_t v = wave_incl_max(i < len ? S.u.dpos[i] : 0u);
        if (i < len) S.u.dpos[i] = v;
        if (lane == kWave - 1) S.cbase[c] = v;
      }
      __syncthreads();
      if (w == 0) {
        const uint32_t v = lane < nc ? S.cbase[lane] : 0;
        const uint32_t incl = wave_incl_max(v);
        uint32_t excl = __shfl_up(incl, 1, kWave);
        if (lane == 0) excl = 0;
        if (lane < nc) S.cbase[lane] = excl;
      }
      __syncthreads();
      for (uint32_t i = tid; i < len; i += kTB) {
        const uint32_t v = S.u.dpos[i], cb = S.cbase[i >> 6];
        S.u.dpos[i] = v > cb ? v : cb;
      }
      __syncthreads();
    }
    // ---- passes: the whole tile (all_rows), or each (row, out-list chunk)
    // with its in-edges and forward entries; the hashed range is [pD0, pD0+plen)
    uint32_t r = r_lo, cur = 0, cb = 0, xe = 0, bh = 0, ea = 0, eb = 0;
    bool row_open = false, done = false;
    while (!done) {
      uint32_t pD0, plen, pb0, pb1, pfa, pfb;
      if (all_rows) {
        pD0 = D0;
        plen = D1 - D0;
        pb0 = 0;
        pb1 = nbw;
        pfa = 0;
        pfb = span;
        done = true;
      } else {
        if (!row_open) {  // find the next row with entries in the tile
          bool found = false;
          for (; r <= r_hi; ++r) {
            const int64_t rb = a.row_off[r], re = a.row_off[r + 1];
            ea = (uint32_t)((rb > j0 ? rb : j0) - j0);
            eb = (uint32_t)((re < j0 + (int64_t)span ? re : j0 + (int64_t)span) - j0);
            if (eb <= ea) continue;
            if (tid == 0) {  // first bw index at or past the end of row r in the tile
              uint32_t lo = cur, hi = nbw;
              while (lo < hi) {
                const uint32_t mid = lo + ((hi - lo) >> 1);
                if ((uint32_t)S.bw[mid] < eb)
                  lo = mid + 1;
                else
                  hi = mid;
              }
              S.bcast[2] = lo;
            }
            __syncthreads();
            bh = S.bcast[2];
            __syncthreads();
            cb = a.fstart[r];
            xe = a.fstart[r + 1];
            if (xe > cb || bh > cur) {
              found = true;
              break;
            }
            cur = bh;
          }
          if (!found) break;
          row_open = true;
        }
        pD0 = cb;
        plen = xe - cb < C.cap ? xe - cb : C.cap;
        pb0 = cur;
        pb1 = bh;
        pfa = ea;
        pfb = eb;
        cb += C.cap;
        if (cb >= xe) {  // last chunk of this row
          row_open = false;
          cur = bh;
          ++r;
        }
      }
      C.D0 = pD0;
      tri_build_hash(C, S, plen, all_rows);
      if (!C.eo_later) tri_forward_eids(C, S, pfa, pfb, all_rows);
      for (uint32_t b0 = pb0; b0 < pb1; b0 += kB)
        tri_batch<kMode, kB>(C, S, b0, b0 + kB < pb1 ? b0 + kB : pb1, all_rows);
      tri_flush_xbits(C, S);
    }
    if (kEO) {  // record the round in which the tile still bid
      if (tid == 0) S.bcast[3] = 0;
      __syncthreads();
      if (C.n_sel != sel0) S.bcast[3] = 1;
      __syncthreads();
      if (tid == 0 && S.bcast[3]) a.eo_live[t] = a.round;
    }
  }
  if (gcur != 0xffffffffu && !kCount) tri_flush_counts(C, S, gcur);
  if (kEO && C.eo_append)  // the wave's unused reserved slots become dead records
    for (uint32_t i = lane; i < C.wleft; i += kWave)
      if (C.wcur + i < a.eo_cap)
        reinterpret_cast<uint32_t*>(a.eo_list + 2 * (C.wcur + i))[0] = kDead;
}

// ---- Edge-Once rounds on the triangle lists: records {e_yx, e_xw, e_yw,
// e_del} {word 2, third vertex of each of the three edges}.  In list 0 a
// reserved slot that stayed unused has e_yx = kDead.  Round r after the
// listing round L bids from list (r - L - 1) mod 2 and copies each triangle
// that bids (none of its edges closed) into the other list; a triangle whose
// edge closed is decided and dropped, so each round reads only the last
// round's bidders.
constexpr int kListBlock = 256;

// The listing round's bidders did not fit the list (the slots taken,
// unused reserved ones included, pass its capacity).
__device__ __forceinline__ bool eo_list_overflow(const TriArgs& a) {
  return a.eo_list_cnt[0] > a.eo_cap;
}

// Bids on the list start the round after the listing round, acceptance on
// the list in the listing round itself (unless the list overflowed).
__device__ __forceinline__ bool eo_listed_round(const TriArgs& a, bool accept) {
  const uint32_t listed = a.eo_state[0];
  return listed != 0 &&
         (listed < a.round || (accept && listed == a.round && !eo_list_overflow(a)));
}

__global__ void k_eo_round_start(TriArgs a) {
  const uint32_t listed = a.eo_state[0];
  if (listed != 0 && listed + 1 == a.round && eo_list_overflow(a)) {
    a.eo_state[0] = 0;
    a.eo_list_cnt[0] = 0;
    a.eo_list_cnt[1] = 0;
  }
}

// Clears the bids that the previous round's bidders placed: they are the
// records of the list this round bids from (all of them bid on their three
// edges; a dead slot of the listing round's list bid nowhere).
__global__ __launch_bounds__(kListBlock) void k_eo_list_clear(TriArgs a) {
  if (a.eo_und[a.round - 1] == 0) return;
  const uint32_t listed = a.eo_state[0];
  if (listed == 0 || listed >= a.round) return;
  const uint32_t src = (a.round - listed - 1) & 1u;
  uint64_t n = a.eo_list_cnt[src];
  if (n > kEoListClearMax) return;  // k_eo_clear_bids swept every edge
  if (n > a.eo_cap) n = a.eo_cap;
  const uint4* list = a.eo_list + (uint64_t)src * 2 * a.eo_cap;
  for (uint64_t i = blockIdx.x * (uint64_t)kListBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kListBlock) {
    const uint4 r0 = list[2 * i];
    if (r0.x == kDead) continue;
    a.minkey[r0.x] = ~0ull;
    a.minkey[r0.y] = ~0ull;
    a.minkey[r0.z] = ~0ull;
  }
}

// Records a wave takes at a time: it counts the ones that will bid, reserves
// that many slots of the other list with one atomic, then bids and copies
// them (one atomic per 64 records on the shared counter serialized the
// kernel).
constexpr uint32_t kListSpan = 16 * kWave;

__device__ __forceinline__ bool eo_list_live(const TriArgs& a, const uint4& r0) {
  return r0.x != kDead && !bit_get(a.closed, r0.x) && !bit_get(a.closed, r0.y) &&
         !bit_get(a.closed, r0.z);
}

__global__ __launch_bounds__(kListBlock) void k_eo_list_bid(TriArgs a) {
  if (!eo_listed_round(a, false) || a.eo_und[a.round - 1] == 0) return;
  __shared__ uint64_t red[kListBlock / kWave];
  const uint32_t src = (a.round - a.eo_state[0] - 1) & 1u, dst = src ^ 1u;
  const uint4* from = a.eo_list + (uint64_t)src * 2 * a.eo_cap;
  uint4* to = a.eo_list + (uint64_t)dst * 2 * a.eo_cap;
  uint64_t n = a.eo_list_cnt[src];
  if (n > a.eo_cap) n = a.eo_cap;
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (kListBlock / kWave);
  uint64_t und = 0;
  for (uint64_t b = (blockIdx.x * (uint64_t)(kListBlock / kWave) + threadIdx.x / kWave) * kListSpan;
       b < n; b += waves * kListSpan) {
    const uint64_t e = b + kListSpan < n ? b + kListSpan : n;
    uint64_t cnt = 0;
    for (uint64_t i = b + lane; i < e; i += kWave) cnt += eo_list_live(a, from[2 * i]);
    cnt = wave_sum64(cnt);
    if (cnt == 0) continue;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long*)&a.eo_list_cnt[dst], (unsigned long long)cnt);
    base = __shfl(base, 0, kWave);
    // the same records pass the same test again (this kernel changes no
    // closed bit), so exactly cnt slots from base are written; the first
    // lane has the lowest index, so it is in every iteration another lane is
    for (uint64_t i = b + lane; i < e; i += kWave) {
      const uint4 r0 = from[2 * i];
      const bool live = eo_list_live(a, r0);
      const uint64_t mask = __ballot(live);
      if (live) {
        const uint4 r1 = from[2 * i + 1];
        const uint64_t hi = (uint64_t)r1.x << 32;
        eo_bid(a.minkey + r0.x, hi | r1.y);
        eo_bid(a.minkey + r0.y, hi | r1.z);
        eo_bid(a.minkey + r0.z, hi | r1.w);
        ++und;
        const uint64_t j = base + __popcll(mask & lanemask_lt());
        if (j < a.eo_cap) {  // j < n <= eo_cap: at most every source record bids
          to[2 * j] = r0;
          to[2 * j + 1] = r1;
        }
      }
      base += __popcll(mask);
    }
  }
  const uint64_t t = wave_sum64(und);
  if (lane == 0) red[threadIdx.x / kWave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s = 0;
    for (int i = 0; i < kListBlock / kWave; ++i) s += red[i];
    if (s) atomicAdd((unsigned long long*)&a.eo_und[a.round], (unsigned long long)s);
  }
}

__global__ __launch_bounds__(kListBlock) void k_eo_list_accept(TriArgs a) {
  if (!eo_listed_round(a, true)) return;
  const uint32_t listed = a.eo_state[0];
  // the list this round's bids came from has been read in full: clear its
  // count for the next round, which copies into it
  const uint32_t src = (a.round - listed - 1) & 1u;
  if (a.round > listed && blockIdx.x == 0 && threadIdx.x == 0) a.eo_list_cnt[src] = 0;
  if (a.eo_und[a.round] == 0) return;
  const uint32_t cur = a.round == listed ? 0u : src ^ 1u;
  const uint4* list = a.eo_list + (uint64_t)cur * 2 * a.eo_cap;
  uint64_t n = a.eo_list_cnt[cur];
  if (n > a.eo_cap) n = a.eo_cap;
  for (uint64_t i = blockIdx.x * (uint64_t)kListBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kListBlock) {
    const uint4 r0 = list[2 * i];
    if (r0.x == kDead) continue;
    const uint4 r1 = list[2 * i + 1];
    const uint64_t hi = (uint64_t)r1.x << 32;
    if (a.minkey[r0.x] != (hi | r1.y) || a.minkey[r0.y] != (hi | r1.z) ||
        a.minkey[r0.z] != (hi | r1.w))
      continue;
    bit_set(a.closed, r0.x);
    bit_set(a.closed, r0.y);
    bit_set(a.closed, r0.z);
    mark_set(a.marks, r0.w);
  }
}

// Acceptance of an Edge-Once round without a list: the key on DAG edge
// {a,b} (a's row) names its holder triangle {a,b,w} by the third vertex w.
// The edge facing the holder's largest id checks the holder's keys on the
// other two edges (binary searches in the DAG rows of their lower-ranked
// ends); if it holds all three minima the triangle is considered: its three
// edges close and its drawn edge k is marked.  A wave takes 64 consecutive
// vertices, whose DAG rows are one contiguous range: the lanes stride over
// it (coalesced key reads) and find each position's row among the 64 row
// starts by a search over the lanes.
__device__ __forceinline__ uint32_t dag_pos(const TriArgs& a, uint32_t ru, uint32_t rv) {
  const uint32_t lo_r = ru < rv ? ru : rv, hi_r = ru < rv ? rv : ru;
  const uint2 rg = a.dag_rng[lo_r];
  const uint32_t lo = dag_find(a, rg.x, rg.y, hi_r);
  return lo < rg.y && a.dag_col[lo] == hi_r ? lo : kDead;
}

__global__ __launch_bounds__(kListBlock) void k_eo_accept_edges(TriArgs a, uint64_t n) {
  const uint32_t listed = a.eo_state[0];
  const bool on_list = listed != 0 && listed <= a.round &&
                       !(listed == a.round && eo_list_overflow(a));
  if (on_list || a.eo_und[a.round] == 0) return;
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (kListBlock / kWave);
  for (uint64_t g = blockIdx.x * (uint64_t)(kListBlock / kWave) + threadIdx.x / kWave;
       g * kWave < n; g += waves) {
    const uint64_t v0 = g * kWave;
    const uint64_t vend = v0 + kWave < n ? v0 + kWave : n;
    const uint32_t pend = a.fstart[vend];
    const uint32_t fs = v0 + lane < vend ? a.fstart[v0 + lane] : pend;  // row start per lane
    const uint32_t pbeg = __shfl(fs, 0, kWave);
    // 64-bit positions: with m near 2^32 a 32-bit base + 64 could wrap
    for (uint64_t base = pbeg; base < pend; base += kWave) {
      const uint64_t p = base + lane;
      uint32_t own = 0;  // last lane whose row starts at or before p
#pragma unroll
      for (uint32_t step = kWave / 2; step > 0; step >>= 1) {
        const uint32_t cand = own + step;
        if (__shfl(fs, (int)cand, kWave) <= p) own = cand;
      }
      if (p >= pend) continue;
      const uint32_t pos = (uint32_t)p;  // < pend <= 2^32 - 1
      const uint64_t mk = a.minkey[pos];
      if (mk == ~0ull) continue;
      const uint32_t v = (uint32_t)(v0 + own);
      uint32_t lo = 0, hi = a.gcount;  // the vertex's graph: last with vb <= v
      while (hi - lo > 1) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a.gd[mid].vb <= v)
          lo = mid;
        else
          hi = mid;
      }
      const GDesc& G = a.gd[lo];
      const uint32_t vb = (uint32_t)G.vb;
      const uint32_t rb = a.dag_col[pos];
      const uint32_t la = v - vb, lb = a.order[rb] - vb, lw = (uint32_t)mk;
      if (!(lw > la && lw > lb)) continue;  // the edge facing the largest id decides
      const uint64_t hk = mk & 0xffffffff00000000ull;
      const uint32_t rw = a.rank[vb + lw];
      const uint32_t p_aw = dag_pos(a, a.rank[v], rw), p_bw = dag_pos(a, rb, rw);
      if (p_aw == kDead || p_bw == kDead) continue;  // only for inputs breaking the contract
      if (a.minkey[p_aw] != (hk | lb) || a.minkey[p_bw] != (hk | la)) continue;
      // considered: edge k of ({t0,t1}, {t0,t2}, {t1,t2}), t2 = lw the largest
      const uint32_t t0 = la < lb ? la : lb, t1 = la < lb ? lb : la;
      const uint4 wr = philox4(t0, t1, lw, 0u, G.k0, G.k1);
      const uint32_t kk = __umulhi(wr.y, 3u);
      const uint32_t p_t0w = la < lb ? p_aw : p_bw, p_t1w = la < lb ? p_bw : p_aw;
      bit_set(a.closed, pos);
      bit_set(a.closed, p_aw);
      bit_set(a.closed, p_bw);
      mark_set(a.marks, kk == 0 ? pos : (kk == 1 ? p_t0w : p_t1w));
    }
  }
}

void eo_accept_edges(const TriArgs& a, uint64_t n, int num_cu, hipStream_t s) {
  const unsigned blocks = (unsigned)(num_cu > 0 ? num_cu * 8 : 2048);
  hipLaunchKernelGGL(k_eo_accept_edges, dim3(blocks), dim3(kListBlock), 0, s, a, n);
}

void eo_round_start(const TriArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_eo_round_start, dim3(1), dim3(1), 0, s, a);
}

void eo_list_clear(const TriArgs& a, int num_cu, hipStream_t s) {
  const unsigned blocks = (unsigned)(num_cu > 0 ? num_cu * 8 : 2048);
  hipLaunchKernelGGL(k_eo_list_clear, dim3(blocks), dim3(kListBlock), 0, s, a);
}

void eo_list_round(const TriArgs& a, int num_cu, hipStream_t s) {
  const unsigned blocks = (unsigned)(num_cu > 0 ? num_cu * 8 : 2048);
  hipLaunchKernelGGL(k_eo_list_bid, dim3(blocks), dim3(kListBlock), 0, s, a);
  hipLaunchKernelGGL(k_eo_list_accept, dim3(blocks), dim3(kListBlock), 0, s, a);
}

uint64_t tri_tile_max() { return kTT; }

void triangles(const TriArgs& a, int mode, uint32_t* tile_ctr, int num_cu,
               int blocks_per_cu, int chunk, hipStream_t s) {
  uint64_t blocks = (uint64_t)num_cu * blocks_per_cu;
  if (blocks > a.ntiles) blocks = a.ntiles;
  if (blocks < 1) blocks = 1;
  fill_u32(tile_ctr, 1, 0, s);
  uint32_t cap = (uint32_t)chunk;
  if (cap > (uint32_t)kHashCap) cap = kHashCap;
  if (mode == kModeGeneral)
    hipLaunchKernelGGL(k_triangles<kModeGeneral>, dim3((unsigned)blocks), dim3(kTB), 0, s, a,
                       tile_ctr, cap);
  else if (mode == kModeCount)
    hipLaunchKernelGGL(k_triangles<kModeCount>, dim3((unsigned)blocks), dim3(kTB), 0, s, a,
                       tile_ctr, cap);
  else if (mode == kModeEO)
    hipLaunchKernelGGL(k_triangles<kModeEO>, dim3((unsigned)blocks), dim3(kTB), 0, s, a,
                       tile_ctr, cap);
  else
    hipLaunchKernelGGL(k_triangles<kModePlain>, dim3((unsigned)blocks), dim3(kTB), 0, s, a,
                       tile_ctr, cap);
}

}  // namespace slim
