// Batches (slim_batch_*): many graphs as one graph set.  The host builds
// the set header (per-graph descriptors and tile prefixes), a run refreshes
// it in the workspace with one copy when it changed, and the launch sequence
// of the set is captured once into a HIP graph and replayed.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "slim_batch.h"

using namespace slim;

namespace slim {

int plan_set(const std::vector<GDesc>& graphs, SetPlan& P) {
  const uint32_t count = (uint32_t)graphs.size();
  P.gd.assign(count + 1, GDesc{});
  P.t0c.assign(count + 1, 0);
  P.vt0.assign(count + 1, 0);
  P.et0.assign(count + 1, 0);
  P.ne.assign(count, 0);
  SetShape& S = P.shape;
  S = SetShape{};
  S.count = count;
  S.gathered = true;
  uint64_t N = 0, NNZ = 0, maxdeg = 0;
  for (uint32_t g = 0; g < count; ++g) {
    GDesc d = graphs[g];
    d.vb = N;
    d.eb = NNZ;
    d.cap = d.ne;
    P.gd[g] = d;
    P.ne[g] = d.ne;
    P.t0c[g] = S.n_c;
    P.vt0[g] = S.nvt;
    P.et0[g] = S.net;
    S.n_c += tiles_of(d.ne, kTile);
    for (int i = 0; i < 3; ++i) S.n_tri[i] += tiles_of(d.ne, kTriTileMin << i);
    S.nvt += (d.nv + kTile - 1) / kTile;
    S.net += (d.ne + kTile - 1) / kTile;
    if (op_lists_triangles(d.op)) S.has_tr = true;
    if (d.op == SLIM_OP_TR2 || d.op == SLIM_OP_MCTR) S.general = true;
    if (d.op == SLIM_OP_MCTR) S.has_mc = true;
    if (d.op == SLIM_OP_EOTR)
      S.has_eo = true;
    else if (op_lists_triangles(d.op))
      S.has_list = true;
    uint64_t md = d.nv > 0 ? d.nv - 1 : 0;
    if (d.ne < md) md = d.ne;
    if (md > maxdeg) maxdeg = md;
    N += d.nv;
    NNZ += d.ne;
  }
  P.t0c[count] = S.n_c;
  P.vt0[count] = S.nvt;
  P.et0[count] = S.net;
  if (N > 0xffffffffull || NNZ / 2 > 0xffffffffull)
    return fail(SLIM_EINVAL, "set union too large: n = %llu, m = %llu (limit 2^32-1 each)",
                (unsigned long long)N, (unsigned long long)(NNZ / 2));
  S.N = N;
  S.NNZ = NNZ;
  S.n_u = tiles_of(NNZ, kTile);
  S.passes = radix_passes(maxdeg);
  return SLIM_OK;
}

void fill_header(const SetPlan& P, const SetLayout& L, const Tuning& knobs, void* ws,
                 std::vector<char>& hdr) {
  const uint32_t cnt = P.shape.count;
  hdr.assign(L.hdr_bytes, 0);
  char* h = hdr.data();
  GDesc* gd = reinterpret_cast<GDesc*>(h + L.gd);
  for (uint32_t g = 0; g < cnt; ++g) gd[g] = P.gd[g];
  gd[cnt] = union_desc(P.shape, L, ws);
  uint64_t* t0c = reinterpret_cast<uint64_t*>(h + L.t0c);
  uint64_t* t0t = reinterpret_cast<uint64_t*>(h + L.t0t);
  uint64_t* t0u = reinterpret_cast<uint64_t*>(h + L.t0u);
  uint64_t* vt0 = reinterpret_cast<uint64_t*>(h + L.vt0);
  uint64_t* et0 = reinterpret_cast<uint64_t*>(h + L.et0);
  uint64_t acc = 0;
  for (uint32_t g = 0; g <= cnt; ++g) {
    t0c[g] = P.t0c[g];
    vt0[g] = P.vt0[g];
    et0[g] = P.et0[g];
    t0t[g] = acc;
    if (g < cnt) acc += tiles_of(P.ne[g], (uint64_t)knobs.tri_tile);
  }
  t0u[0] = 0;
  t0u[1] = P.shape.n_u;
}

}  // namespace slim

struct slim_batch {
  int device = 0;
  int num_cu = 0;
  uint32_t count = 0;
  SetPlan plan;
  SetLayout layout{};
  Tuning knobs;
  bool use_graph = true;
  bool verbose = false;  // the tuner reports each candidate on stderr
  // header upload
  std::vector<char> hdr;
  void* pinned = nullptr;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  // per-graph stats of the most recent run (device, one record per graph),
  // and the event that marks the end of that run
  slim_stats_t* dstats = nullptr;
  hipEvent_t run_done = nullptr;
  bool ran = false;
  // captured launch sequence
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* cap_ws = nullptr;
  Tuning cap_knobs;
};

namespace {

bool same_knobs(const Tuning& a, const Tuning& b) {
  return a.tri_chunk == b.tri_chunk && a.tri_blocks_per_cu == b.tri_blocks_per_cu &&
         a.tri_tile == b.tri_tile && a.eo_rounds == b.eo_rounds;
}

void drop_graph(slim_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap_ws = nullptr;
}

// Fills the host copy of the set header for workspace `ws` and outputs.
void build_header(slim_batch* b, void* ws, const slim_out_t* outs) {
  for (uint32_t g = 0; g < b->count; ++g) {
    b->plan.gd[g].out_row = outs[g].row_off;
    b->plan.gd[g].out_col = outs[g].col;
    b->plan.gd[g].stats = outs[g].stats;
    b->plan.gd[g].out_w = outs[g].weight;
  }
  fill_header(b->plan, b->layout, b->knobs, ws, b->hdr);
  // the union descriptor carries the batch's own per-graph stats array
  reinterpret_cast<GDesc*>(b->hdr.data() + b->layout.gd)[b->count].stats = b->dstats;
}

int check_run(const slim_batch* b, void* ws, uint64_t ws_bytes, const slim_out_t* outs) {
  if (!b) return fail(SLIM_EINVAL, "batch is NULL");
  if (!outs) return fail(SLIM_EINVAL, "outs is NULL");
  if (ws_bytes < b->layout.total)
    return fail(SLIM_ENOMEM, "workspace has %llu bytes, %llu needed",
                (unsigned long long)ws_bytes, (unsigned long long)b->layout.total);
  if (!ws) return fail(SLIM_EINVAL, "d_ws is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SLIM_EINVAL, "d_ws must be 256-byte aligned");
  for (uint32_t g = 0; g < b->count; ++g) {
    if (!outs[g].row_off) return fail(SLIM_EINVAL, "outs[%u].row_off is NULL", g);
    if (b->plan.gd[g].ne && !outs[g].col) return fail(SLIM_EINVAL, "outs[%u].col is NULL", g);
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return fail(SLIM_EINVAL, "the batch lives on device %d, current device is %d", b->device, dev);
  return SLIM_OK;
}

int run(slim_batch* b, void* ws, uint64_t ws_bytes, const slim_out_t* outs, hipStream_t s) {
  if (int rc = check_run(b, ws, ws_bytes, outs)) return rc;
  (void)hipGetLastError();
  build_header(b, ws, outs);
  const size_t hb = b->hdr.size();
  // The header is uploaded on every run: between two runs of this batch the
  // workspace may have served another call, which writes its own header at
  // the same place.
  // The pinned buffer may still feed the previous upload.
  if (b->upload_pending && hipEventSynchronize(b->upload_done) != hipSuccess)
    return fail(SLIM_EDEVICE, "batch header: previous upload failed");
  std::memcpy(b->pinned, b->hdr.data(), hb);
  if (hipMemcpyAsync(ws, b->pinned, hb, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventRecord(b->upload_done, s) != hipSuccess)
    return fail(SLIM_EDEVICE, "batch header upload failed");
  b->upload_pending = true;
  auto finish = [&]() -> int {
    if (hipEventRecord(b->run_done, s) != hipSuccess)
      return fail(SLIM_EDEVICE, "slim_batch_run: event record failed");
    b->ran = true;
    return hip_check("slim_batch_run");
  };
  if (!b->use_graph) {  // direct launches: phases are timed when profiling is on
    prof_reset();
    run_set(b->plan.shape, b->layout, b->knobs, b->num_cu, ws, nullptr, nullptr, s, true);
    if (int rc = hip_check("slim_batch_run")) return rc;
    if (int rc = eo_finish(b->plan.shape, b->layout, b->knobs, b->num_cu, ws, nullptr, nullptr, s))
      return rc;
    return finish();
  }
  if (!b->exec || b->cap_ws != ws || !same_knobs(b->cap_knobs, b->knobs)) {
    drop_graph(b);
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
      return fail(SLIM_EDEVICE, "hipStreamBeginCapture failed");
    run_set(b->plan.shape, b->layout, b->knobs, b->num_cu, ws, nullptr, nullptr, b->cap_stream, false);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &gr);
    if (e != hipSuccess || !gr) {
      (void)hipGetLastError();
      return fail(SLIM_EDEVICE, "capture of the batch failed: %s", hipGetErrorString(e));
    }
    b->graph = gr;
    e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      b->exec = nullptr;
      drop_graph(b);
      return fail(SLIM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->cap_ws = ws;
    b->cap_knobs = b->knobs;
  }
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return fail(SLIM_EDEVICE, "hipGraphLaunch failed");
  // Edge-Once rounds past the captured ones run as direct launches
  if (int rc = eo_finish(b->plan.shape, b->layout, b->knobs, b->num_cu, ws, nullptr, nullptr, s))
    return rc;
  return finish();
}

std::string tune_key(const slim_batch* b) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, b->device);
  std::ostringstream k;
  k << prop.gcnArchName << ":" << b->num_cu << ":" << b->count << ":" << b->plan.shape.N << ":"
    << b->plan.shape.NNZ << ":" << (b->plan.shape.has_tr ? "tr" : "es");
  std::string s = k.str();
  for (char& c : s)
    if (c == ' ' || c == '\t' || c == '\n') c = '_';
  return s;
}

bool tune_lookup(const char* path, const std::string& key, Tuning& t) {
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // the last matching line wins
    std::istringstream is(line);
    std::string k;
    if (!(is >> k) || k != key) continue;
    Tuning c = t;
    std::string kv;
    bool good = true;
    while (is >> kv) {
      const size_t eq = kv.find('=');
      if (eq == std::string::npos) {
        good = false;
        break;
      }
      const std::string name = kv.substr(0, eq);
      const long long v = std::atoll(kv.c_str() + eq + 1);
      if (!tune_apply(c, name.c_str(), v)) good = false;
    }
    if (good) {
      t = c;
      found = true;
    }
  }
  return found;
}

}  // namespace

extern "C" {

int slim_batch_create(const slim_graph_t* const* graphs, const slim_job_params_t* jobs,
                      uint32_t count, slim_batch_t** out) {
  if (!out) return fail(SLIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!graphs || !jobs) return fail(SLIM_EINVAL, "graphs or jobs is NULL");
  if (count == 0) return fail(SLIM_EINVAL, "a batch needs at least one graph");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SLIM_EDEVICE, "hipGetDevice failed");
  std::vector<GDesc> gs(count);
  int num_cu = 0;
  for (uint32_t g = 0; g < count; ++g) {
    const slim_graph* G = graphs[g];
    const slim_job_params_t& J = jobs[g];
    if (!G) return fail(SLIM_EINVAL, "graphs[%u] is NULL", g);
    if (G->device != dev)
      return fail(SLIM_EINVAL, "graphs[%u] lives on device %d, not %d", g, G->device, dev);
    if (!op_valid(J.op) || J.pad != 0)
      return fail(SLIM_EINVAL, "jobs[%u]: bad op %d", g, J.op);
    if (check_param(J.op, J.p)) return SLIM_EINVAL;
    num_cu = G->num_cu;
    GDesc& d = gs[g];
    d.nv = G->n;
    d.ne = G->nnz;
    d.thr = J.op == SLIM_OP_SPECTRAL ? 0 : threshold(J.p);
    d.ups = J.op == SLIM_OP_SPECTRAL ? J.p : 0.0;
    d.k0 = (uint32_t)J.seed;
    d.k1 = (uint32_t)(J.seed >> 32);
    d.op = (uint32_t)J.op;
    d.in_row = G->row_off;
    d.in_col = G->col;
  }
  slim_batch* b = new (std::nothrow) slim_batch;
  if (!b) return fail(SLIM_ENOMEM, "out of host memory");
  b->device = dev;
  b->num_cu = num_cu;
  b->count = count;
  if (int rc = plan_set(gs, b->plan)) {
    delete b;
    return rc;
  }
  const SetShape& S = b->plan.shape;
  b->layout = set_layout(S);
  {
    std::lock_guard<std::mutex> lk(tuning_mutex());
    b->knobs = tuning();
  }
  if (hipHostMalloc(&b->pinned, b->layout.hdr_bytes, hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&b->dstats, sizeof(slim_stats_t) * count) != hipSuccess ||
      hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->run_done, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    slim_batch_free(b);
    return fail(SLIM_EDEVICE, "batch: host buffer, event or stream creation failed");
  }
  *out = b;
  return ok();
}

int slim_batch_workspace_size(const slim_batch_t* b, uint64_t* bytes) {
  if (!b || !bytes) return fail(SLIM_EINVAL, "NULL argument");
  *bytes = b->layout.total;
  return ok();
}

int slim_batch_run(slim_batch_t* b, void* d_ws, uint64_t ws_bytes, const slim_out_t* outs,
                   void* stream) {
  return run(b, d_ws, ws_bytes, outs, static_cast<hipStream_t>(stream));
}

int slim_batch_set(slim_batch_t* b, const char* key, int64_t value) {
  if (!b || !key) return fail(SLIM_EINVAL, "NULL argument");
  if (std::strcmp(key, "use_graph") == 0 || std::strcmp(key, "verbose") == 0) {
    if (value != 0 && value != 1) return fail(SLIM_EINVAL, "%s must be 0 or 1", key);
    (key[0] == 'u' ? b->use_graph : b->verbose) = value != 0;
    return ok();
  }
  if (!tune_apply(b->knobs, key, value))
    return fail(SLIM_EINVAL, "unknown knob '%s' or value %lld out of range", key,
                (long long)value);
  return ok();
}

int slim_batch_get(const slim_batch_t* b, const char* key, int64_t* value) {
  if (!b || !key || !value) return fail(SLIM_EINVAL, "NULL argument");
  if (std::strcmp(key, "use_graph") == 0 || std::strcmp(key, "verbose") == 0) {
    *value = (key[0] == 'u' ? b->use_graph : b->verbose) ? 1 : 0;
    return ok();
  }
  if (!tune_read(b->knobs, key, value)) return fail(SLIM_EINVAL, "unknown knob '%s'", key);
  return ok();
}

int slim_batch_tune(slim_batch_t* b, void* d_ws, uint64_t ws_bytes, const slim_out_t* outs,
                    const char* cache_path, void* stream) {
  if (int rc = check_run(b, d_ws, ws_bytes, outs)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string key = tune_key(b);
  if (cache_path && tune_lookup(cache_path, key, b->knobs)) {
    if (int rc = run(b, d_ws, ws_bytes, outs, s)) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(SLIM_EDEVICE, "tune: sync failed");
    return ok();
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SLIM_EDEVICE, "tune: event creation failed");
  // best of two timed replays after one untimed run (which captures)
  auto time_cfg = [&](const Tuning& t, float* ms) -> int {
    b->knobs = t;
    if (int rc = run(b, d_ws, ws_bytes, outs, s)) return rc;
    float best = 1e30f;
    for (int r = 0; r < 2; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) return fail(SLIM_EDEVICE, "tune: event");
      if (int rc = run(b, d_ws, ws_bytes, outs, s)) return rc;
      float x = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&x, e0, e1) != hipSuccess)
        return fail(SLIM_EDEVICE, "tune: timing failed");
      if (x < best) best = x;
    }
    *ms = best;
    if (b->verbose) {
      std::fprintf(stderr, "[slim tune] tri_tile=%d tri_blocks_per_cu=%d tri_chunk=%d: %.3f ms\n",
                   t.tri_tile, t.tri_blocks_per_cu, t.tri_chunk, best);
      std::fflush(stderr);
    }
    return SLIM_OK;
  };
  Tuning best = b->knobs;
  float best_ms = 0.f;
  int rc = SLIM_OK;
  if (b->plan.shape.has_tr && b->plan.shape.NNZ > 0) {
    rc = time_cfg(best, &best_ms);
    const int tiles[] = {1024, 512, 256};
    const int bpcs[] = {1, 2, 3, 4};
    const int chunks[] = {2048, 1024, 512};
    for (int dim = 0; dim < 3 && rc == SLIM_OK; ++dim) {
      const int* vals = dim == 0 ? tiles : dim == 1 ? bpcs : chunks;
      const int nv = dim == 1 ? 4 : 3;
      for (int i = 0; i < nv && rc == SLIM_OK; ++i) {
        Tuning c = best;
        if (dim == 0) c.tri_tile = vals[i];
        if (dim == 1) c.tri_blocks_per_cu = vals[i];
        if (dim == 2) c.tri_chunk = vals[i];
        if (same_knobs(c, best)) continue;
        float ms = 0.f;
        rc = time_cfg(c, &ms);
        if (rc == SLIM_OK && ms < best_ms) {
          best = c;
          best_ms = ms;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SLIM_OK) return rc;
  b->knobs = best;
  if ((rc = run(b, d_ws, ws_bytes, outs, s)) != SLIM_OK) return rc;
  if (hipStreamSynchronize(s) != hipSuccess) return fail(SLIM_EDEVICE, "tune: sync failed");
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    if (!f) return fail(SLIM_EINVAL, "cannot append to tuning cache '%s'", cache_path);
    f << key << " tri_tile=" << best.tri_tile << " tri_blocks_per_cu=" << best.tri_blocks_per_cu
      << " tri_chunk=" << best.tri_chunk << "\n";
  }
  return ok();
}

int slim_batch_stats(slim_batch_t* b, slim_stats_t* per_graph) {
  if (!b || !per_graph) return fail(SLIM_EINVAL, "NULL argument");
  if (!b->ran) return fail(SLIM_EINVAL, "slim_batch_stats: the batch has not run yet");
  if (hipEventSynchronize(b->run_done) != hipSuccess ||
      hipMemcpy(per_graph, b->dstats, sizeof(slim_stats_t) * b->count, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return fail(SLIM_EDEVICE, "slim_batch_stats: %s", hipGetErrorString(hipGetLastError()));
  return ok();
}

void slim_batch_free(slim_batch_t* b) {
  if (!b) return;
  drop_graph(b);
  if (b->upload_done) {
    (void)hipEventSynchronize(b->upload_done);
    (void)hipEventDestroy(b->upload_done);
  }
  if (b->run_done) {
    (void)hipEventSynchronize(b->run_done);
    (void)hipEventDestroy(b->run_done);
  }
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->dstats) (void)hipFree(b->dstats);
  delete b;
}

}  // extern "C"
