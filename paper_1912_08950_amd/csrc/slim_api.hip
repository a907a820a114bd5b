// C ABI of libslim (declared in include/slim.h): argument checks, workspace
// carving and the launch sequence of a graph set on the caller's stream --
// one graph for slim_triangle_reduce / slim_edge_sample, many for a batch
// (gathered into a union CSR, captured once into a HIP graph and replayed).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "slim_batch.h"
#include "slim_internal.h"

namespace slim {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return SLIM_OK;
}

int hip_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SLIM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

const char* last_error() { return g_err.c_str(); }

namespace {

constexpr uint64_t kAlign = 256;

struct Carve {
  uint64_t off = 0;
  template <class T>
  uint64_t take(uint64_t count) {
    uint64_t o = off;
    uint64_t bytes = count * sizeof(T);
    off += (bytes + kAlign - 1) / kAlign * kAlign;
    return o;
  }
};

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

template <class T>
T* at(void* base, uint64_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

}  // namespace

uint64_t threshold(double p) {
  if (p >= 1.0) return uint64_t(1) << 32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

int check_p(double p) {
  if (!(p >= 0.0 && p <= 1.0)) return fail(SLIM_EINVAL, "p must lie in [0, 1], got %g", p);
  return SLIM_OK;
}

int check_param(int op, double p) {
  if (op == SLIM_OP_SPECTRAL) {
    if (!(p >= 0.0)) return fail(SLIM_EINVAL, "upsilon must be >= 0, got %g", p);
    return SLIM_OK;
  }
  return check_p(p);
}

// 8-bit radix passes that order degrees up to maxdeg.
int radix_passes(uint64_t maxdeg) {
  int bits = 0;
  while (bits < 64 && (maxdeg >> bits) != 0) ++bits;
  int passes = (bits + 7) / 8;
  return passes < 1 ? 1 : passes;
}

uint64_t tiles_of(uint64_t ne, uint64_t tile) {
  const uint64_t t = ceil_div(ne, tile);
  return t < 1 ? 1 : t;
}

SetShape single_shape(uint64_t n, uint64_t nnz, int op) {
  SetShape S;
  S.count = 1;
  S.N = n;
  S.NNZ = nnz;
  S.gathered = false;
  S.has_tr = op_lists_triangles((uint32_t)op);
  S.has_eo = op == SLIM_OP_EOTR;
  S.has_list = S.has_tr && !S.has_eo;
  S.general = op == SLIM_OP_TR2 || op == SLIM_OP_MCTR;
  S.has_mc = op == SLIM_OP_MCTR;
  S.n_c = tiles_of(nnz, kTile);
  S.n_u = S.n_c;
  for (int i = 0; i < 3; ++i) S.n_tri[i] = tiles_of(nnz, kTriTileMin << i);
  S.nvt = S.net = 0;
  uint64_t maxdeg = n > 0 ? n - 1 : 0;
  if (nnz < maxdeg) maxdeg = nnz;
  S.passes = radix_passes(maxdeg);
  return S;
}

SetLayout set_layout(const SetShape& S) {
  SetLayout L{};
  // header, packed: gd[count+1] (the last is the union), t0c, t0t [count+1],
  // t0u[2], vt0, et0 [count+1]; a one-graph set's first four fit 256 bytes
  const uint64_t cnt1 = (uint64_t)S.count + 1;
  L.gd = 0;
  L.t0c = L.gd + sizeof(GDesc) * cnt1;
  L.t0t = L.t0c + 8 * cnt1;
  L.t0u = L.t0t + 8 * cnt1;
  L.vt0 = L.t0u + 16;
  L.et0 = L.vt0 + 8 * cnt1;
  L.hdr_bytes = L.et0 + 8 * cnt1;
  Carve c;
  c.off = (L.hdr_bytes + kAlign - 1) / kAlign * kAlign;
  if (S.gathered) {
    L.urow = c.take<int64_t>(S.N + 1);
    L.ucol = c.take<uint32_t>(S.NNZ);
  }
  L.recs_c = c.take<TileRec>(S.n_c);
  const uint64_t nt = std::max(S.n_c, S.n_u);
  L.tile_cnt = c.take<uint32_t>(nt + 1);
  L.tile_base = c.take<uint64_t>(nt + 1);
  L.masks = c.take<uint64_t>(nt * (uint64_t)kChunks);
  uint64_t st = scan_tmp_elems(nt);
  if (S.has_tr) {
    const uint64_t n = S.N, m = S.NNZ / 2;
    const uint64_t hist = sort_hist_elems(n);
    st = std::max(st, scan_tmp_elems(hist));
    L.recs_u = S.gathered ? c.take<TileRec>(S.n_u) : L.recs_c;
    L.recs_t = c.take<TileRec>(S.n_tri[0]);
    L.ka = c.take<uint32_t>(n);
    L.va = c.take<uint32_t>(n);
    L.kb = c.take<uint32_t>(n);
    L.vb = c.take<uint32_t>(n);
    L.rank = c.take<uint32_t>(n);
    L.rcol = c.take<uint32_t>(S.NNZ);
    L.hist = c.take<uint32_t>(hist);
    L.hist_scan = c.take<uint64_t>(hist + 1);
    L.fstart = c.take<uint32_t>(n + 1);
    L.dag_rng = c.take<uint2>(n);
    L.dag_col = c.take<uint32_t>(m);
    L.fence = c.take<uint32_t>(ceil_div(m, kFenceStep) + 1);
    L.eid = c.take<uint32_t>(S.NNZ);
    L.del = c.take<uint32_t>(ceil_div(m, 32) + 1);
    L.marks = c.take<uint32_t>(ceil_div(m, 4) + 1);  // one byte per edge, filled by words
    L.counters = c.take<uint64_t>(2 * (uint64_t)S.count);
    L.sort_lists = c.take<uint32_t>(3 * n);
    L.sort_counts = c.take<uint32_t>(4);
    L.tri_ctr = c.take<uint32_t>(4);
    if (S.has_mc) L.tcount = c.take<uint32_t>(m);
    if (S.has_eo) {
      L.minkey = c.take<uint64_t>(m);
      L.closed = c.take<uint32_t>(ceil_div(m, 32) + 1);
      L.eo_und = c.take<uint64_t>(kEoMaxRounds + 1);
      L.eo_live = c.take<uint32_t>(S.n_tri[0]);
      L.eo_list = c.take<uint4>(2 * 2 * kEoListPerEdge * m);  // two lists
      L.eo_misc = c.take<uint64_t>(3);
    }
  }
  L.scan_tmp = c.take<uint64_t>(st + 1);
  L.total = c.off;
  return L;
}

// The union descriptor (index `count` of the set's table) that makes the
// orientation write the DAG into the workspace.
GDesc union_desc(const SetShape& S, const SetLayout& L, void* ws) {
  GDesc u{};
  u.vb = 0;
  u.nv = S.N;
  u.eb = 0;
  u.ne = S.NNZ;
  u.cap = S.NNZ / 2;
  u.op = 0;
  u.out_row = at<uint32_t>(ws, L.fstart);
  u.out_col = at<uint32_t>(ws, L.dag_col);
  return u;
}

// ---------------------------------------------------------- profiler
// Phase timing with HIP events on the call's stream (slim_profile_*).
struct Profiler {
  std::mutex mu;
  bool on = false;
  struct Ph {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
  };
  std::vector<Ph> ph;
  size_t used = 0;
};

Profiler& prof() {
  static Profiler p;
  return p;
}

void prof_reset() {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  P.used = 0;
}

void prof_begin(bool on, const char* name, hipStream_t s) {
  if (!on) return;
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.on) return;
  if (P.used == P.ph.size()) {
    Profiler::Ph p;
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    P.ph.push_back(p);
  }
  P.ph[P.used].name = name;
  (void)hipEventRecord(P.ph[P.used].a, s);
}

void prof_end(bool on, hipStream_t s) {
  if (!on) return;
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.on || P.used >= P.ph.size()) return;
  (void)hipEventRecord(P.ph[P.used].b, s);
  ++P.used;
}

// ------------------------------------------------------ the pipeline
// Edge-Once rounds r0..r1 of a set (launches after the last busy round
// return at once).
void eo_rounds(const SetShape& S, const SetLayout& L, const Tuning& knobs, int num_cu, void* ws,
               TriArgs a, uint32_t r0, uint32_t r1, hipStream_t s) {
  a.minkey = at<uint64_t>(ws, L.minkey);
  a.closed = at<uint32_t>(ws, L.closed);
  a.eo_und = at<uint64_t>(ws, L.eo_und);
  a.eo_live = at<uint32_t>(ws, L.eo_live);
  a.eo_list = at<uint4>(ws, L.eo_list);
  a.eo_list_cnt = at<uint64_t>(ws, L.eo_misc);
  a.eo_state = reinterpret_cast<uint32_t*>(at<uint64_t>(ws, L.eo_misc) + 2);
  a.eo_cap = kEoListPerEdge * (S.NNZ / 2);
  a.eo_list_try = (uint32_t)knobs.eo_list_try;
  a.gcount = S.count;
  for (uint32_t r = r0; r <= r1; ++r) {
    a.round = r;
    eo_round_start(a, s);
    eo_clear_bids(a.minkey, a.closed, S.NNZ / 2, a.eo_und, a.eo_state, a.eo_list_cnt, r, s);
    eo_list_clear(a, num_cu, s);
    a.pass = 2;
    triangles(a, kModeEO, at<uint32_t>(ws, L.tri_ctr), num_cu, knobs.tri_blocks_per_cu,
              knobs.tri_chunk, s);
    eo_accept_edges(a, S.N, num_cu, s);
    eo_list_round(a, num_cu, s);
  }
}

// The triangle kernel's arguments for a set whose DAG is in the workspace.
TriArgs tri_args(const SetShape& S, const SetLayout& L, const Tuning& knobs, void* ws,
                 const int64_t* row_off, const uint32_t* col, const uint32_t* order) {
  TriArgs a{};
  a.row_off = row_off;
  a.col = col;
  a.rank = at<uint32_t>(ws, L.rank);
  a.rcol = at<uint32_t>(ws, L.rcol);
  a.order = order;
  a.dag_rng = at<uint2>(ws, L.dag_rng);
  a.fstart = at<uint32_t>(ws, L.fstart);
  a.dag_col = at<uint32_t>(ws, L.dag_col);
  a.fence = at<uint32_t>(ws, L.fence);
  a.eid = at<uint32_t>(ws, L.eid);
  a.marks = at<uint8_t>(ws, L.marks);
  a.counters = at<uint64_t>(ws, L.counters);
  a.gd = at<GDesc>(ws, L.gd);
  a.recs = at<TileRec>(ws, L.recs_t);
  a.ntiles = S.n_t(knobs.tri_tile);
  a.tcount = S.has_mc ? at<uint32_t>(ws, L.tcount) : nullptr;
  return a;
}
// Enqueues every phase of a set whose header (descriptors and tile
// prefixes) is already in the workspace.  `row_off`/`col` are the caller's
// CSR for a single graph; a gathered set builds its union in the workspace.
void run_set(const SetShape& S, const SetLayout& L, const Tuning& knobs, int num_cu, void* ws,
             const int64_t* row_off, const uint32_t* col, hipStream_t s, bool profile) {
  const GDesc* gd = at<GDesc>(ws, L.gd);
  const uint64_t* t0c = at<uint64_t>(ws, L.t0c);
  uint32_t* tile_cnt = at<uint32_t>(ws, L.tile_cnt);
  uint64_t* tile_base = at<uint64_t>(ws, L.tile_base);
  uint64_t* scan_tmp = at<uint64_t>(ws, L.scan_tmp);
  TileRec* recs_c = at<TileRec>(ws, L.recs_c);
  const bool tr = S.has_tr && S.NNZ > 0;
  prof_begin(profile, tr ? "rank" : "sample", s);
  if (S.gathered) {
    int64_t* urow = at<int64_t>(ws, L.urow);
    uint32_t* ucol = at<uint32_t>(ws, L.ucol);
    gather(gd, S.count, at<uint64_t>(ws, L.vt0), at<uint64_t>(ws, L.et0), S.nvt, S.net, S.N,
           S.NNZ, urow, ucol, s);
    row_off = urow;
    col = ucol;
  }
  tile_recs(row_off, gd, t0c, S.count, S.n_c, kTile, recs_c, s);
  uint32_t* eid = nullptr;
  uint32_t* del = nullptr;
  uint64_t* counters = nullptr;
  if (tr) {
    uint32_t* rank = at<uint32_t>(ws, L.rank);
    uint32_t* order = nullptr;
    degree_rank(row_off, S.N, S.passes, at<uint32_t>(ws, L.ka), at<uint32_t>(ws, L.va),
                at<uint32_t>(ws, L.kb), at<uint32_t>(ws, L.vb), at<uint32_t>(ws, L.hist),
                at<uint64_t>(ws, L.hist_scan), scan_tmp, &order, rank, s);
    prof_end(profile, s);
    prof_begin(profile, "orient", s);
    const GDesc* gu = gd + S.count;
    const uint64_t* t0u = S.gathered ? at<uint64_t>(ws, L.t0u) : t0c;
    TileRec* recs_u = at<TileRec>(ws, L.recs_u);
    if (S.gathered) tile_recs(row_off, gu, t0u, 1, S.n_u, kTile, recs_u, s);
    uint32_t* fstart = at<uint32_t>(ws, L.fstart);
    uint32_t* dag_col = at<uint32_t>(ws, L.dag_col);
    uint2* dag_rng = at<uint2>(ws, L.dag_rng);
    uint32_t* rcol = at<uint32_t>(ws, L.rcol);
    orient(row_off, col, rank, rcol, gu, t0u, recs_u, S.n_u, tile_cnt, at<uint64_t>(ws, L.masks),
           tile_base, scan_tmp, s);
    dag_ranges(order, fstart, S.N, dag_rng, s);
    sort_rows(dag_rng, S.N, dag_col, at<uint32_t>(ws, L.sort_lists),
              at<uint32_t>(ws, L.sort_counts), num_cu, s);
    uint32_t* fence = at<uint32_t>(ws, L.fence);
    fence_samples(dag_col, S.NNZ / 2, fence, s);
    eid = at<uint32_t>(ws, L.eid);
    del = at<uint32_t>(ws, L.del);
    counters = at<uint64_t>(ws, L.counters);
    TileRec* recs_t = at<TileRec>(ws, L.recs_t);
    const uint64_t n_t = S.n_t(knobs.tri_tile);
    tile_recs(row_off, gd, at<uint64_t>(ws, L.t0t), S.count, n_t, (uint64_t)knobs.tri_tile,
              recs_t, s);
    uint8_t* marks = at<uint8_t>(ws, L.marks);
    fill_u32(reinterpret_cast<uint32_t*>(marks), ceil_div(S.NNZ / 2, 4) + 1, 0, s);
    fill_u32(reinterpret_cast<uint32_t*>(counters), 4 * (uint64_t)S.count, 0, s);
    prof_end(profile, s);
    prof_begin(profile, "triangles", s);
    TriArgs a{};
    a.row_off = row_off;
    a.col = col;
    a.rank = rank;
    a.rcol = rcol;
    a.order = order;
    a.dag_rng = dag_rng;
    a.fstart = fstart;
    a.dag_col = dag_col;
    a.fence = fence;
    a.eid = eid;
    a.marks = marks;
    a.counters = counters;
    a.gd = gd;
    a.recs = recs_t;
    a.ntiles = n_t;
    a.tcount = S.has_mc ? at<uint32_t>(ws, L.tcount) : nullptr;
    a.round = 0;
    if (S.has_mc) {  // Min-Count: per-edge triangle counts first
      fill_u32(a.tcount, S.NNZ / 2, 0, s);
      a.pass = 0;
      triangles(a, kModeCount, at<uint32_t>(ws, L.tri_ctr), num_cu, knobs.tri_blocks_per_cu,
                knobs.tri_chunk, s);
    }
    if (S.has_list) {
      a.pass = 1;
      triangles(a, S.general ? kModeGeneral : kModePlain, at<uint32_t>(ws, L.tri_ctr), num_cu,
                knobs.tri_blocks_per_cu, knobs.tri_chunk, s);
    }
    prof_end(profile, s);
    if (S.has_eo) {
      prof_begin(profile, "eo_rounds", s);
      fill_u32(at<uint32_t>(ws, L.closed), ceil_div(S.NNZ / 2, 32) + 1, 0, s);
      fill_u32(reinterpret_cast<uint32_t*>(at<uint64_t>(ws, L.eo_und)), 2 * (kEoMaxRounds + 1),
               0, s);
      fill_u32(at<uint32_t>(ws, L.eo_live), S.n_t(knobs.tri_tile), 0, s);
      fill_u32(reinterpret_cast<uint32_t*>(at<uint64_t>(ws, L.eo_misc)), 6, 0, s);
      eo_rounds(S, L, knobs, num_cu, ws, a, 1, (uint32_t)knobs.eo_rounds, s);
      prof_end(profile, s);
    }
    prof_begin(profile, "compact", s);
    pack_marks(marks, del, S.NNZ / 2, s);
  }
  compact_out(row_off, col, eid, del, S.NNZ / 2, gd, t0c, recs_c, S.n_c, tile_cnt,
              at<uint64_t>(ws, L.masks), tile_base,
              scan_tmp, s);
  write_stats(gd, S.count, t0c, counters, tile_base, s);
  prof_end(profile, s);
}

int eo_finish(const SetShape& S, const SetLayout& L, const Tuning& knobs, int num_cu, void* ws,
              const int64_t* row_off, const uint32_t* col, hipStream_t s) {
  if (!S.has_eo || S.NNZ == 0) return SLIM_OK;
  if (S.gathered) {
    row_off = at<int64_t>(ws, L.urow);
    col = at<uint32_t>(ws, L.ucol);
  }
  const uint64_t* und = at<uint64_t>(ws, L.eo_und);
  const uint32_t step = (uint32_t)knobs.eo_rounds;
  uint32_t last = step;
  bool more = false;
  for (;;) {
    uint64_t u = 0;
    if (hipMemcpyAsync(&u, und + last, sizeof(u), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(SLIM_EDEVICE, "Edge-Once round counter: %s",
                  hipGetErrorString(hipGetLastError()));
    if (u == 0) break;
    if (last + step > kEoMaxRounds)
      return fail(SLIM_EDEVICE, "Edge-Once: undecided triangles after %u rounds", last);
    const uint32_t* order = at<uint32_t>(ws, S.passes % 2 ? L.vb : L.va);
    eo_rounds(S, L, knobs, num_cu, ws, tri_args(S, L, knobs, ws, row_off, col, order), last + 1,
              last + step, s);
    last += step;
    more = true;
  }
  if (more) {  // the first compaction saw the marks of the first rounds only
    const GDesc* gd = at<GDesc>(ws, L.gd);
    const uint64_t* t0c = at<uint64_t>(ws, L.t0c);
    uint64_t* tile_base = at<uint64_t>(ws, L.tile_base);
    pack_marks(at<uint8_t>(ws, L.marks), at<uint32_t>(ws, L.del), S.NNZ / 2, s);
    compact_out(row_off, col, at<uint32_t>(ws, L.eid), at<uint32_t>(ws, L.del), S.NNZ / 2, gd,
                t0c, at<TileRec>(ws, L.recs_c), S.n_c, at<uint32_t>(ws, L.tile_cnt),
                at<uint64_t>(ws, L.masks), tile_base,
                at<uint64_t>(ws, L.scan_tmp), s);
    write_stats(gd, S.count, t0c, at<uint64_t>(ws, L.counters), tile_base, s);
  }
  return SLIM_OK;
}

// ----------------------------------------------------------- tuning
bool tune_apply(Tuning& t, const char* key, int64_t value) {
  const std::string k(key);
  if (k == "tri_chunk") {
    if (value < 32 || value > 2048) return false;
    t.tri_chunk = (int)value;
  } else if (k == "tri_blocks_per_cu") {
    if (value < 1 || value > 64) return false;
    t.tri_blocks_per_cu = (int)value;
  } else if (k == "tri_tile") {
    if (value < (int64_t)kTriTileMin || value > (int64_t)tri_tile_max() ||
        (value & (value - 1)) != 0)
      return false;
    t.tri_tile = (int)value;
  } else if (k == "eo_rounds") {
    if (value < 1 || value > 64) return false;
    t.eo_rounds = (int)value;
  } else if (k == "eo_list_try") {
    if (value < 0 || value > 100000) return false;
    t.eo_list_try = (int)value;
  } else {
    return false;
  }
  return true;
}

bool tune_read(const Tuning& t, const char* key, int64_t* value) {
  const std::string k(key);
  if (k == "tri_chunk")
    *value = t.tri_chunk;
  else if (k == "tri_blocks_per_cu")
    *value = t.tri_blocks_per_cu;
  else if (k == "tri_tile")
    *value = t.tri_tile;
  else if (k == "eo_rounds")
    *value = t.eo_rounds;
  else if (k == "eo_list_try")
    *value = t.eo_list_try;
  else
    return false;
  return true;
}

Tuning& tuning() {
  static Tuning t;
  return t;
}

std::mutex& tuning_mutex() {
  static std::mutex m;
  return m;
}

}  // namespace slim

using namespace slim;

namespace {

int check_call(const slim_graph* g, int op, double p, void* ws, uint64_t ws_bytes, uint64_t need,
               int64_t* out_ro, uint32_t* out_col) {
  if (!g) return fail(SLIM_EINVAL, "graph handle is NULL");
  if (check_param(op, p)) return SLIM_EINVAL;
  if (!out_ro) return fail(SLIM_EINVAL, "d_out_row_off is NULL");
  if (g->nnz && !out_col) return fail(SLIM_EINVAL, "d_out_col is NULL");
  if (ws_bytes < need)
    return fail(SLIM_ENOMEM, "workspace has %llu bytes, %llu needed",
                (unsigned long long)ws_bytes, (unsigned long long)need);
  if (need && !ws) return fail(SLIM_EINVAL, "d_ws is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(SLIM_EINVAL, "d_ws must be %llu-byte aligned", (unsigned long long)kAlign);
  return SLIM_OK;
}

// The header of a one-graph set, written by one small kernel.
struct SingleHdr {
  GDesc gd[2];
  uint64_t t0c[2];
  uint64_t t0t[2];
  uint64_t t0u[2];
};
static_assert(sizeof(SingleHdr) <= 512, "one put_bytes launch");
static_assert(sizeof(GDesc) == 120, "descriptor size");

int single_op(int op, const slim_graph* g, double p, uint64_t seed, void* ws, uint64_t ws_bytes,
              int64_t* out_ro, uint32_t* out_col, float* out_w, slim_stats_t* stats,
              hipStream_t s, bool profile = true) {
  if (!op_valid(op)) return fail(SLIM_EINVAL, "unknown op %d", op);
  const bool tr = op_lists_triangles((uint32_t)op);
  const char* what = op == SLIM_OP_TR         ? "slim_triangle_reduce"
                     : op == SLIM_OP_ES       ? "slim_edge_sample"
                     : op == SLIM_OP_SPECTRAL ? "slim_spectral_sparsify"
                                              : "slim_compress";
  const SetShape S = g ? single_shape(g->n, g->nnz, op) : SetShape{};
  const uint64_t need = g && g->nnz ? set_layout(S).total : 0;
  if (int rc = check_call(g, op, p, ws, ws_bytes, need, out_ro, out_col)) return rc;
  (void)hipGetLastError();
  if (profile) prof_reset();
  if (g->nnz == 0) {
    prof_begin(profile, tr ? "compact" : "sample", s);
    fill_i64(out_ro, g->n + 1, 0, s);
    if (stats) {
      slim_stats_t st{g->n, 0, 0, 0, 0, 0};
      put_bytes(stats, &st, sizeof(st), s);
    }
    prof_end(profile, s);
    return hip_check(what);
  }
  Tuning knobs;
  {
    std::lock_guard<std::mutex> lk(tuning_mutex());
    knobs = tuning();
  }
  const SetLayout L = set_layout(S);
  SingleHdr h{};
  GDesc& d = h.gd[0];
  d.vb = 0;
  d.nv = g->n;
  d.eb = 0;
  d.ne = g->nnz;
  d.thr = op == SLIM_OP_SPECTRAL ? 0 : threshold(p);
  d.ups = op == SLIM_OP_SPECTRAL ? p : 0.0;
  d.k0 = (uint32_t)seed;
  d.k1 = (uint32_t)(seed >> 32);
  d.op = (uint32_t)op;
  d.cap = g->nnz;
  d.in_row = g->row_off;
  d.in_col = g->col;
  d.out_row = out_ro;
  d.out_col = out_col;
  d.out_w = out_w;
  d.stats = stats;
  h.gd[1] = union_desc(S, L, ws);
  h.t0c[0] = 0;
  h.t0c[1] = S.n_c;
  h.t0t[0] = 0;
  h.t0t[1] = S.n_t(knobs.tri_tile);
  h.t0u[0] = 0;
  h.t0u[1] = S.n_u;
  // the packed header of a one-graph set starts with exactly these arrays
  static_assert(offsetof(SingleHdr, t0c) == 2 * sizeof(GDesc), "layout");
  if (L.t0c != offsetof(SingleHdr, t0c) || L.t0t != offsetof(SingleHdr, t0t) ||
      L.t0u != offsetof(SingleHdr, t0u))
    return fail(SLIM_EDEVICE, "internal: set header layout");
  put_bytes(at<char>(ws, L.gd), &h, sizeof(h), s);
  run_set(S, L, knobs, g->num_cu, ws, g->row_off, g->col, s, profile);
  if (int rc = hip_check(what)) return rc;
  if (int rc = eo_finish(S, L, knobs, g->num_cu, ws, g->row_off, g->col, s)) return rc;
  return hip_check(what);
}

// ------------------------------------------ the entry point that allocates nothing
// The workspace of slim_triangle_reduce_noalloc: a device array of fixed size
// that every GPU the library runs on holds until the process ends.  In host
// code `scratch` names only a host-side stand-in; its device address on the
// current device comes from hipGetSymbolAddress, taken once per device and
// kept, and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[SLIM_NOALLOC_WS_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SLIM_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SLIM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SLIM_OK;
}

}  // namespace

extern "C" {

const char* slim_last_error(void) { return last_error(); }

const char* slim_strerror(int code) {
  switch (code) {
    case SLIM_OK: return "SLIM_OK";
    case SLIM_EINVAL: return "SLIM_EINVAL";
    case SLIM_ENOMEM: return "SLIM_ENOMEM";
    case SLIM_EBUDGET: return "SLIM_EBUDGET";
    case SLIM_EDEVICE: return "SLIM_EDEVICE";
    case SLIM_EAGAIN: return "SLIM_EAGAIN";
    default: return "SLIM_E(unknown)";
  }
}

int slim_version(void) { return 200; }

int slim_load_csr(const int64_t* d_row_off, const uint32_t* d_col, uint64_t n, uint64_t nnz,
                  uint32_t flags, void* stream, slim_graph_t** out) {
  if (!out) return fail(SLIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_row_off) return fail(SLIM_EINVAL, "d_row_off is NULL");
  if (nnz && !d_col) return fail(SLIM_EINVAL, "d_col is NULL");
  if (n > 0xffffffffull) return fail(SLIM_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
  if (nnz % 2) return fail(SLIM_EINVAL, "nnz = %llu is odd (CSR must be symmetric)",
                           (unsigned long long)nnz);
  if (nnz / 2 > 0xffffffffull) return fail(SLIM_EINVAL, "m = nnz/2 exceeds 2^32-1");
  if (n == 0 && nnz) return fail(SLIM_EINVAL, "n = 0 with nnz > 0");
  if (flags & ~SLIM_VALIDATE) return fail(SLIM_EINVAL, "unknown flags 0x%x", flags);
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SLIM_EDEVICE, "hipGetDevice failed");
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(SLIM_EDEVICE, "cannot query the CU count");
  if (flags & SLIM_VALIDATE) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t ntiles = tiles_of(nnz, kTile);
    // err word, then a one-graph set header and its tile records
    const uint64_t hdr = 256, recs_off = 2 * hdr;
    const uint64_t bytes = recs_off + sizeof(TileRec) * ntiles;
    char* buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess)
      return fail(SLIM_EDEVICE, "validation buffer allocation failed");
    uint32_t* err = reinterpret_cast<uint32_t*>(buf);
    GDesc* gd = reinterpret_cast<GDesc*>(buf + hdr);
    uint64_t* t0 = reinterpret_cast<uint64_t*>(buf + hdr + sizeof(GDesc));
    TileRec* recs = reinterpret_cast<TileRec*>(buf + recs_off);
    uint32_t h_err = 0;
    fill_u32(err, 1, 0, s);
    validate_offsets(d_row_off, n, nnz, err, s);
    hipError_t e = hipMemcpyAsync(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && h_err == 0 && nnz) {
      struct {
        GDesc d;
        uint64_t t0[2];
      } h{};
      h.d.nv = n;
      h.d.ne = nnz;
      h.t0[1] = ntiles;
      put_bytes(gd, &h, sizeof(h), s);
      tile_recs(d_row_off, gd, t0, 1, ntiles, kTile, recs, s);
      validate_entries(d_row_off, d_col, n, recs, ntiles, err, s);
      e = hipMemcpyAsync(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(SLIM_EDEVICE, "validation: %s", hipGetErrorString(e));
    if (h_err) {
      const char* what = (h_err & 1)    ? "row offsets are not monotone from 0 to nnz"
                         : (h_err & 2)  ? "a column id is >= n"
                         : (h_err & 4)  ? "a self-loop"
                         : (h_err & 8)  ? "a row is not strictly increasing"
                                        : "an edge is missing its reverse copy";
      return fail(SLIM_EINVAL, "invalid CSR: %s", what);
    }
  }
  slim_graph* g = new (std::nothrow) slim_graph{d_row_off, d_col, n, nnz, dev, cu};
  if (!g) return fail(SLIM_ENOMEM, "out of host memory");
  *out = g;
  return ok();
}

void slim_graph_free(slim_graph_t* g) { delete g; }

int slim_workspace_size(const slim_graph_t* g, int op, uint64_t* bytes) {
  if (!g || !bytes) return fail(SLIM_EINVAL, "NULL argument");
  if (!op_valid(op)) return fail(SLIM_EINVAL, "unknown op %d", op);
  *bytes = g->nnz ? set_layout(single_shape(g->n, g->nnz, op)).total : 0;
  return ok();
}

int slim_triangle_reduce(const slim_graph_t* g, double p, uint64_t seed, void* d_ws,
                         uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                         slim_stats_t* d_stats, void* stream) {
  return single_op(SLIM_OP_TR, g, p, seed, d_ws, ws_bytes, d_out_row_off, d_out_col, nullptr,
                   d_stats,
                   static_cast<hipStream_t>(stream));
}

int slim_compress(const slim_graph_t* g, int op, double p, uint64_t seed, void* d_ws,
                  uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                  slim_stats_t* d_stats, void* stream) {
  return single_op(op, g, p, seed, d_ws, ws_bytes, d_out_row_off, d_out_col, nullptr, d_stats,
                   static_cast<hipStream_t>(stream));
}

int slim_edge_sample(const slim_graph_t* g, double p, uint64_t seed, void* d_ws,
                     uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                     slim_stats_t* d_stats, void* stream) {
  return single_op(SLIM_OP_ES, g, p, seed, d_ws, ws_bytes, d_out_row_off, d_out_col, nullptr,
                   d_stats,
                   static_cast<hipStream_t>(stream));
}

int slim_spectral_sparsify(const slim_graph_t* g, double upsilon, uint64_t seed, void* d_ws,
                           uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                           float* d_out_weight, slim_stats_t* d_stats, void* stream) {
  return single_op(SLIM_OP_SPECTRAL, g, upsilon, seed, d_ws, ws_bytes, d_out_row_off, d_out_col,
                   d_out_weight, d_stats, static_cast<hipStream_t>(stream));
}

int slim_triangle_reduce_noalloc(const slim_graph_t* g, double p, uint64_t seed,
                                 int64_t* d_out_row_off, uint32_t* d_out_col,
                                 slim_stats_t* d_stats, void* stream) {
  if (!g) return fail(SLIM_EINVAL, "graph handle is NULL");
  if (check_p(p)) return SLIM_EINVAL;
  const uint64_t need =
      g->nnz ? set_layout(single_shape(g->n, g->nnz, SLIM_OP_TR)).total : 0;
  if (need > SLIM_NOALLOC_WS_BYTES)
    return fail(SLIM_ENOMEM,
                "slim_triangle_reduce_noalloc: the graph needs %llu bytes of workspace, the "
                "static workspace holds %llu (use slim_triangle_reduce with a caller workspace)",
                (unsigned long long)need, (unsigned long long)SLIM_NOALLOC_WS_BYTES);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SLIM_EDEVICE, "hipGetDevice failed");
  if (dev != g->device)
    return fail(SLIM_EINVAL, "the graph lives on device %d, current device is %d", g->device, dev);
  void* ws = nullptr;
  if (int rc = scratch_address(dev, &ws)) return rc;
  return single_op(SLIM_OP_TR, g, p, seed, ws, SLIM_NOALLOC_WS_BYTES, d_out_row_off, d_out_col,
                   nullptr, d_stats, static_cast<hipStream_t>(stream), false);
}

int slim_profile_enable(int on) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  P.on = on != 0;
  P.used = 0;
  return ok();
}

int slim_profile_read(slim_phase_t* out, int max, int* count) {
  if (!count || (max > 0 && !out)) return fail(SLIM_EINVAL, "NULL argument");
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  *count = (int)P.used;
  for (size_t i = 0; i < P.used && (int)i < max; ++i) {
    hipError_t e = hipEventSynchronize(P.ph[i].b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, P.ph[i].a, P.ph[i].b);
    if (e != hipSuccess) return fail(SLIM_EDEVICE, "profile: %s", hipGetErrorString(e));
    std::memset(out[i].name, 0, sizeof(out[i].name));
    std::strncpy(out[i].name, P.ph[i].name.c_str(), sizeof(out[i].name) - 1);
    out[i].ms = ms;
  }
  return ok();
}

int slim_tune_set(const char* key, int64_t value) {
  if (!key) return fail(SLIM_EINVAL, "key is NULL");
  std::lock_guard<std::mutex> lk(tuning_mutex());
  if (!tune_apply(tuning(), key, value))
    return fail(SLIM_EINVAL, "unknown knob '%s' or value %lld out of range", key,
                (long long)value);
  return ok();
}

int slim_tune_get(const char* key, int64_t* value) {
  if (!key || !value) return fail(SLIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(tuning_mutex());
  if (!tune_read(tuning(), key, value)) return fail(SLIM_EINVAL, "unknown knob '%s'", key);
  return ok();
}

}  // extern "C"
