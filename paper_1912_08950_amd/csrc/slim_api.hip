// C ABI of libslim (declared in include/slim.h): argument checks, workspace
// carving and the launch sequence of each operation on the caller's stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "slim_internal.h"

struct slim_graph {
  const int64_t* row_off;
  const uint32_t* col;
  uint64_t n;
  uint64_t nnz;
  int device;
  int num_cu;
};

namespace {

thread_local std::string g_err;

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

struct Common {
  uint64_t ntiles;
  uint64_t tile_lo, tile_cnt, tile_base, scan_tmp;
};

struct TrLayout : Common {
  uint64_t ka, va, kb, vb, rank, hist, hist_scan;
  uint64_t fstart, dag_rng, dag_col, eid, del, counters;
  uint64_t sort_lists, sort_counts, tri_tlo, tri_ctr;
  uint64_t total;
  int passes;
};

struct EsLayout : Common {
  uint64_t total;
};

int radix_passes(uint64_t n, uint64_t nnz) {
  uint64_t maxdeg = n > 0 ? n - 1 : 0;
  if (nnz < maxdeg) maxdeg = nnz;
  int bits = 0;
  while (bits < 64 && (maxdeg >> bits) != 0) ++bits;
  int passes = (bits + 7) / 8;
  return passes < 1 ? 1 : passes;
}

TrLayout tr_layout(uint64_t n, uint64_t nnz) {
  TrLayout L{};
  Carve c;
  const uint64_t m = nnz / 2;
  L.ntiles = ceil_div(nnz, slim::kTile);
  L.passes = radix_passes(n, nnz);
  const uint64_t hist = slim::sort_hist_elems(n);
  uint64_t st = slim::scan_tmp_elems(hist);
  uint64_t st2 = slim::scan_tmp_elems(L.ntiles);
  if (st2 > st) st = st2;
  L.ka = c.take<uint32_t>(n);
  L.va = c.take<uint32_t>(n);
  L.kb = c.take<uint32_t>(n);
  L.vb = c.take<uint32_t>(n);
  L.rank = c.take<uint32_t>(n);
  L.hist = c.take<uint32_t>(hist);
  L.hist_scan = c.take<uint64_t>(hist + 1);
  L.scan_tmp = c.take<uint64_t>(st + 1);
  L.tile_lo = c.take<uint32_t>(L.ntiles + 1);
  L.tile_cnt = c.take<uint32_t>(L.ntiles + 1);
  L.tile_base = c.take<uint64_t>(L.ntiles + 1);
  L.fstart = c.take<uint32_t>(n + 1);
  L.dag_rng = c.take<uint2>(n);
  L.dag_col = c.take<uint32_t>(m);
  L.eid = c.take<uint32_t>(nnz);
  L.del = c.take<uint32_t>(ceil_div(m, 32) + 1);
  L.counters = c.take<uint64_t>(4);
  L.sort_lists = c.take<uint32_t>(3 * n);
  L.sort_counts = c.take<uint32_t>(4);
  L.tri_tlo = c.take<uint32_t>(slim::tri_tiles(nnz) + 1);
  L.tri_ctr = c.take<uint32_t>(4);
  L.total = c.off;
  return L;
}

EsLayout es_layout(uint64_t nnz) {
  EsLayout L{};
  Carve c;
  L.ntiles = ceil_div(nnz, slim::kTile);
  L.scan_tmp = c.take<uint64_t>(slim::scan_tmp_elems(L.ntiles) + 1);
  L.tile_lo = c.take<uint32_t>(L.ntiles + 1);
  L.tile_cnt = c.take<uint32_t>(L.ntiles + 1);
  L.tile_base = c.take<uint64_t>(L.ntiles + 1);
  L.total = c.off;
  return L;
}

template <class T>
T* at(void* base, uint64_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int check_p(double p) {
  if (!(p >= 0.0 && p <= 1.0)) return fail(SLIM_EINVAL, "p must lie in [0, 1], got %g", p);
  return SLIM_OK;
}

uint64_t threshold(double p) {
  if (p >= 1.0) return uint64_t(1) << 32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

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

void prof_begin(const char* name, hipStream_t s) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.on) return;
  if (P.used == P.ph.size()) {
    Profiler::Ph p;
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    P.ph.push_back(p);
  }
  P.ph[P.used].name = name;
  hipEventRecord(P.ph[P.used].a, s);
}

void prof_end(hipStream_t s) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.on || P.used >= P.ph.size()) return;
  hipEventRecord(P.ph[P.used].b, s);
  ++P.used;
}

int check_call(const slim_graph* g, double p, void* ws, uint64_t ws_bytes, uint64_t need,
               int64_t* out_ro, uint32_t* out_col) {
  if (!g) return fail(SLIM_EINVAL, "graph handle is NULL");
  if (check_p(p)) return SLIM_EINVAL;
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

}  // namespace

extern "C" {

const char* slim_last_error(void) { return g_err.c_str(); }

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

int slim_version(void) { return 100; }

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
    const uint64_t ntiles = ceil_div(nnz, slim::kTile);
    uint32_t* buf = nullptr;
    if (hipMalloc(&buf, sizeof(uint32_t) * (ntiles + 2)) != hipSuccess)
      return fail(SLIM_EDEVICE, "validation buffer allocation failed");
    uint32_t* err = buf;
    uint32_t* tile_lo = buf + 1;
    uint32_t h_err = 0;
    slim::fill_u32(err, 1, 0, s);
    slim::validate_offsets(d_row_off, n, nnz, err, s);
    hipError_t e = hipMemcpyAsync(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && h_err == 0 && nnz) {
      slim::tile_lo_build(d_row_off, n, nnz, ntiles, tile_lo, s);
      slim::validate_entries(d_row_off, d_col, n, nnz, ntiles, tile_lo, err, s);
      e = hipMemcpyAsync(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    hipFree(buf);
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
  if (op == SLIM_OP_TR)
    *bytes = g->nnz ? tr_layout(g->n, g->nnz).total : 0;
  else if (op == SLIM_OP_ES)
    *bytes = g->nnz ? es_layout(g->nnz).total : 0;
  else
    return fail(SLIM_EINVAL, "unknown op %d", op);
  return ok();
}

int slim_triangle_reduce(const slim_graph_t* g, double p, uint64_t seed, void* d_ws,
                         uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                         slim_stats_t* d_stats, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t need = g && g->nnz ? tr_layout(g->n, g->nnz).total : 0;
  if (int rc = check_call(g, p, d_ws, ws_bytes, need, d_out_row_off, d_out_col)) return rc;
  (void)hipGetLastError();
  const uint64_t n = g->n, nnz = g->nnz;
  if (nnz == 0) {
    slim::fill_i64(d_out_row_off, n + 1, 0, s);
    slim::write_stats(n, 0, nullptr, nullptr, d_stats, s);
    return hip_check("slim_triangle_reduce");
  }
  const TrLayout L = tr_layout(n, nnz);
  prof_reset();
  prof_begin("rank", s);
  uint32_t* rank = at<uint32_t>(d_ws, L.rank);
  uint32_t* order = nullptr;
  uint64_t* scan_tmp = at<uint64_t>(d_ws, L.scan_tmp);
  slim::degree_rank(g->row_off, n, L.passes, at<uint32_t>(d_ws, L.ka), at<uint32_t>(d_ws, L.va),
                    at<uint32_t>(d_ws, L.kb), at<uint32_t>(d_ws, L.vb),
                    at<uint32_t>(d_ws, L.hist), at<uint64_t>(d_ws, L.hist_scan), scan_tmp,
                    &order, rank, s);
  prof_end(s);
  prof_begin("orient", s);
  uint32_t* tile_lo = at<uint32_t>(d_ws, L.tile_lo);
  uint32_t* tile_cnt = at<uint32_t>(d_ws, L.tile_cnt);
  uint64_t* tile_base = at<uint64_t>(d_ws, L.tile_base);
  uint32_t* fstart = at<uint32_t>(d_ws, L.fstart);
  uint32_t* dag_col = at<uint32_t>(d_ws, L.dag_col);
  uint32_t* eid = at<uint32_t>(d_ws, L.eid);
  uint32_t* del = at<uint32_t>(d_ws, L.del);
  uint64_t* counters = at<uint64_t>(d_ws, L.counters);
  uint2* dag_rng = at<uint2>(d_ws, L.dag_rng);
  slim::tile_lo_build(g->row_off, n, nnz, L.ntiles, tile_lo, s);
  slim::orient(g->row_off, g->col, rank, n, nnz, L.ntiles, tile_lo, tile_cnt, tile_base, scan_tmp,
               dag_col, eid, fstart, s);
  slim::dag_ranges(order, fstart, n, dag_rng, s);
  slim::sort_rows(dag_rng, n, dag_col, at<uint32_t>(d_ws, L.sort_lists),
                  at<uint32_t>(d_ws, L.sort_counts), g->num_cu, s);
  uint32_t* tri_tlo = at<uint32_t>(d_ws, L.tri_tlo);
  slim::tile_lo_build(g->row_off, n, nnz, slim::tri_tiles(nnz), tri_tlo, s,
                      slim::tri_tile_entries());
  slim::fill_u32(del, ceil_div(nnz / 2, 32) + 1, 0, s);
  slim::fill_u32(reinterpret_cast<uint32_t*>(counters), 8, 0, s);
  prof_end(s);
  slim::TriArgs a;
  a.row_off = g->row_off;
  a.col = g->col;
  a.rank = rank;
  a.order = order;
  a.dag_rng = dag_rng;
  a.fstart = fstart;
  a.dag_col = dag_col;
  a.eid = eid;
  a.del = del;
  a.counters = counters;
  a.n = n;
  a.nnz = nnz;
  a.thr = threshold(p);
  a.k0 = (uint32_t)seed;
  a.k1 = (uint32_t)(seed >> 32);
  prof_begin("triangles", s);
  slim::triangles(a, tri_tlo, at<uint32_t>(d_ws, L.tri_ctr), g->num_cu, s);
  prof_end(s);
  prof_begin("compact", s);
  slim::compact_tr(g->row_off, g->col, eid, del, n, nnz, L.ntiles, tile_lo, tile_cnt, tile_base,
                   scan_tmp, d_out_col, d_out_row_off, s);
  slim::write_stats(n, nnz, counters, tile_base + L.ntiles, d_stats, s);
  prof_end(s);
  return hip_check("slim_triangle_reduce");
}

int slim_edge_sample(const slim_graph_t* g, double p, uint64_t seed, void* d_ws,
                     uint64_t ws_bytes, int64_t* d_out_row_off, uint32_t* d_out_col,
                     slim_stats_t* d_stats, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t need = g && g->nnz ? es_layout(g->nnz).total : 0;
  if (int rc = check_call(g, p, d_ws, ws_bytes, need, d_out_row_off, d_out_col)) return rc;
  (void)hipGetLastError();
  const uint64_t n = g->n, nnz = g->nnz;
  if (nnz == 0) {
    slim::fill_i64(d_out_row_off, n + 1, 0, s);
    slim::write_stats(n, 0, nullptr, nullptr, d_stats, s);
    return hip_check("slim_edge_sample");
  }
  const EsLayout L = es_layout(nnz);
  prof_reset();
  prof_begin("sample", s);
  uint32_t* tile_lo = at<uint32_t>(d_ws, L.tile_lo);
  uint64_t* tile_base = at<uint64_t>(d_ws, L.tile_base);
  slim::tile_lo_build(g->row_off, n, nnz, L.ntiles, tile_lo, s);
  slim::compact_es(g->row_off, g->col, threshold(p), seed, n, nnz, L.ntiles, tile_lo,
                   at<uint32_t>(d_ws, L.tile_cnt), tile_base, at<uint64_t>(d_ws, L.scan_tmp),
                   d_out_col, d_out_row_off, s);
  slim::write_stats(n, nnz, nullptr, tile_base + L.ntiles, d_stats, s);
  prof_end(s);
  return hip_check("slim_edge_sample");
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
  slim::Tuning& t = slim::tuning();
  std::string k(key);
  if (k == "tri_chunk") {
    if (value < 32 || value > 2048) return fail(SLIM_EINVAL, "tri_chunk must lie in [32, 2048]");
    t.tri_chunk = (int)value;
  } else if (k == "tri_blocks_per_cu") {
    if (value < 1 || value > 64) return fail(SLIM_EINVAL, "tri_blocks_per_cu must lie in [1, 64]");
    t.tri_blocks_per_cu = (int)value;
  } else {
    return fail(SLIM_EINVAL, "unknown knob '%s'", key);
  }
  return ok();
}

int slim_tune_get(const char* key, int64_t* value) {
  if (!key || !value) return fail(SLIM_EINVAL, "NULL argument");
  const slim::Tuning& t = slim::tuning();
  std::string k(key);
  if (k == "tri_chunk")
    *value = t.tri_chunk;
  else if (k == "tri_blocks_per_cu")
    *value = t.tri_blocks_per_cu;
  else
    return fail(SLIM_EINVAL, "unknown knob '%s'", key);
  return ok();
}

}  // extern "C"

namespace slim {
Tuning& tuning() {
  static Tuning t;
  return t;
}
}  // namespace slim
