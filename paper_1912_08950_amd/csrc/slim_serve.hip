// Serving (slim_serve_*): jobs are admitted against an HBM budget and run in
// batches that workers form continuously, each worker on its own stream.
// A batch is a graph set like slim_batch's (same planning, header and launch
// sequence), launched directly: its composition is new every time, so there
// is nothing to replay.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "slim_batch.h"

using namespace slim;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Size classes: powers of two up to 1 MiB, then eight classes per doubling
// (at most 9% above the request), so that blocks are reused across batches
// of similar size.
uint64_t size_class(uint64_t bytes) {
  if (bytes <= 256) return 256;
  if (bytes <= (1u << 20)) {
    uint64_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  int top = 63 - __builtin_clzll(bytes);
  const uint64_t step = (uint64_t(1) << top) / 8;
  return (bytes + step - 1) / step * step;
}

// Sub-allocating device allocator.  Device memory is taken from the runtime
// in chunks (kChunk bytes, or one request's size if larger) and carved into
// ranges best fit; freed ranges coalesce with their free neighbours.  In
// steady serving no hipMalloc or hipFree is called (hipFree waits for the
// whole device, which would stall every worker).  A chunk is returned to the
// runtime only when it is entirely free and a new chunk would pass `cap`.
// A range's size travels with it: alloc returns it in *got, free takes it
// back.
class Arena {
 public:
  static constexpr uint64_t kChunk = uint64_t(2) << 30;
  static constexpr uint64_t kAlignB = 4096;
  void set_cap(uint64_t cap) { cap_ = cap; }
  void* alloc(uint64_t bytes, uint64_t* got) {
    const uint64_t c = (std::max<uint64_t>(bytes, 1) + kAlignB - 1) / kAlignB * kAlignB;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = by_size_.lower_bound(c);
    if (it == by_size_.end()) {
      if (!grow(c)) return nullptr;
      it = by_size_.lower_bound(c);
      if (it == by_size_.end()) return nullptr;
    }
    const Range r = it->second;
    const uint64_t len = it->first;
    by_size_.erase(it);
    by_off_.erase(r);
    if (len > c) insert_free(Range{r.chunk, r.off + c}, len - c);
    chunks_[r.chunk].used += c;
    *got = c;
    return chunks_[r.chunk].base + r.off;
  }
  void free(void* p, uint64_t size) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    char* q = static_cast<char*>(p);
    auto ci = by_base_.upper_bound(q);  // the chunk holding q: last base <= q
    if (ci == by_base_.begin()) return;
    --ci;
    const uint32_t k = ci->second;
    chunks_[k].used -= size;
    uint64_t off = (uint64_t)(q - chunks_[k].base), len = size;
    auto nx = by_off_.lower_bound(Range{k, off});
    if (nx != by_off_.end() && nx->first.chunk == k && nx->first.off == off + len) {
      len += nx->second;  // merge with the next free range
      erase_size(nx->first, nx->second);
      nx = by_off_.erase(nx);
    }
    if (nx != by_off_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first.chunk == k && pv->first.off + pv->second == off) {
        off = pv->first.off;  // merge with the previous free range
        len += pv->second;
        erase_size(pv->first, pv->second);
        by_off_.erase(pv);
      }
    }
    insert_free(Range{k, off}, len);
  }
  void release_all() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& ch : chunks_)
      if (ch.base) (void)hipFree(ch.base);
    chunks_.clear();
    by_size_.clear();
    by_off_.clear();
    by_base_.clear();
    total_ = 0;
  }

 private:
  struct Range {
    uint32_t chunk;
    uint64_t off;
    bool operator<(const Range& o) const {
      return chunk != o.chunk ? chunk < o.chunk : off < o.off;
    }
  };
  struct Chunk {
    char* base = nullptr;
    uint64_t size = 0, used = 0;
  };
  void insert_free(Range r, uint64_t len) {
    by_off_.emplace(r, len);
    by_size_.emplace(len, r);
  }
  void erase_size(Range r, uint64_t len) {
    auto rg = by_size_.equal_range(len);
    for (auto i = rg.first; i != rg.second; ++i)
      if (i->second.chunk == r.chunk && i->second.off == r.off) {
        by_size_.erase(i);
        return;
      }
  }
  // A new chunk for a request of c bytes; entirely free chunks go back to
  // the runtime first if the new one would pass the cap.
  bool grow(uint64_t c) {
    const uint64_t sz = c > kChunk ? c : kChunk;
    for (uint32_t k = 0; total_ + sz > cap_ && k < chunks_.size(); ++k) {
      Chunk& ch = chunks_[k];
      if (!ch.base || ch.used != 0) continue;
      erase_size(Range{k, 0}, ch.size);
      by_off_.erase(Range{k, 0});
      by_base_.erase(ch.base);
      (void)hipFree(ch.base);
      total_ -= ch.size;
      ch = Chunk{};
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    uint32_t k = 0;
    while (k < chunks_.size() && chunks_[k].base) ++k;  // reuse a returned slot
    if (k == chunks_.size()) chunks_.emplace_back();
    chunks_[k].base = static_cast<char*>(p);
    chunks_[k].size = sz;
    chunks_[k].used = 0;
    by_base_.emplace(chunks_[k].base, k);
    total_ += sz;
    insert_free(Range{k, 0}, sz);
    return true;
  }

  std::mutex mu_;
  std::vector<Chunk> chunks_;
  std::multimap<uint64_t, Range> by_size_;  // free ranges by length
  std::map<Range, uint64_t> by_off_;        // free ranges by position
  std::map<char*, uint32_t> by_base_;       // chunk by base address
  uint64_t total_ = 0, cap_ = 0;
};

enum State { kQueued, kReady, kRunning, kDone };

struct Job {
  uint64_t ticket = 0;
  slim_job_t spec{};
  State state = kQueued;
  int status = SLIM_OK;
  uint64_t res_out = 0, res_in = 0, res_ws = 0;  // reserved bytes
  void* in_row = nullptr;  // device buffers and the arena block sizes behind them
  void* in_col = nullptr;
  void* out_row = nullptr;
  void* out_col = nullptr;
  uint64_t sz_in_row = 0, sz_in_col = 0, sz_out_row = 0, sz_out_col = 0;
  slim_stats_t stats{};
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct Worker {
  hipStream_t stream = nullptr;
  void* pin_hdr = nullptr;
  uint64_t pin_hdr_bytes = 0;
  void* pin_stats = nullptr;
  uint64_t pin_stats_bytes = 0;
  std::thread th;
};

uint64_t ws_estimate(const slim_job_t& j) {
  std::vector<GDesc> one(1);
  one[0].nv = j.n;
  one[0].ne = j.nnz;
  one[0].op = (uint32_t)j.op;
  SetPlan P;
  if (plan_set(one, P) != SLIM_OK) return ~uint64_t(0);
  const uint64_t est = set_layout(P.shape).total + 256 + sizeof(slim_stats_t);
  return size_class(est + est / 10);
}

}  // namespace

struct slim_server {
  slim_serve_cfg_t cfg{};
  int device = 0;
  int num_cu = 0;
  Tuning knobs;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending, ready;
  std::deque<uint64_t> finished;  // completion order, consumed by slim_serve_next
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_ticket = 1;
  uint64_t in_use = 0, peak = 0;
  uint32_t slots = 0, running = 0;
  bool stop = false;
  std::vector<Worker> workers;
  // statistics since the last reset
  std::vector<double> lat;
  uint64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, batches = 0, batch_jobs = 0;
  double t_first = -1, t_last = 0, edges = 0;
};

namespace {

void admit(slim_server* S) {
  while (!S->pending.empty()) {
    Job* j = S->jobs[S->pending.front()].get();
    const uint64_t r = j->res_out + j->res_in + j->res_ws;
    if (S->slots >= S->cfg.max_slots || S->in_use + r > S->cfg.hbm_budget_bytes) break;
    S->pending.pop_front();
    S->in_use += r;
    S->peak = std::max(S->peak, S->in_use);
    ++S->slots;
    j->state = kReady;
    S->ready.push_back(j->ticket);
  }
}

bool grow_pinned(void** p, uint64_t* have, uint64_t need) {
  if (*have >= need) return true;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *have = 0;
  const uint64_t sz = std::max<uint64_t>(need, 4096) * 2;
  if (hipHostMalloc(p, sz, hipHostMallocDefault) != hipSuccess) {
    *p = nullptr;
    return false;
  }
  *have = sz;
  return true;
}

// Runs one batch to completion on the worker's stream; returns the status.
int run_batch(slim_server* S, Worker& W, const std::vector<Job*>& batch) {
  hipStream_t s = W.stream;
  const uint32_t cnt = (uint32_t)batch.size();
  // An error after the first upload was enqueued waits for the stream before
  // it returns: the caller hands the jobs' blocks back to the arena, and a
  // copy still in flight must not write into a block another batch reuses.
  auto bail = [&](int rc) {
    (void)hipStreamSynchronize(s);
    return rc;
  };
  std::vector<GDesc> gs(cnt);
  for (uint32_t i = 0; i < cnt; ++i) {
    Job* j = batch[i];
    const slim_job_t& J = j->spec;
    j->out_row = S->arena.alloc(8 * (J.n + 1), &j->sz_out_row);
    j->out_col = J.nnz ? S->arena.alloc(4 * J.nnz, &j->sz_out_col) : nullptr;
    if (!j->out_row || (J.nnz && !j->out_col))
      return bail(fail(SLIM_EDEVICE, "serve: out of device memory"));
    const int64_t* in_row = J.row_off;
    const uint32_t* in_col = J.col;
    if (J.where == SLIM_HOST) {
      j->in_row = S->arena.alloc(8 * (J.n + 1), &j->sz_in_row);
      j->in_col = J.nnz ? S->arena.alloc(4 * J.nnz, &j->sz_in_col) : nullptr;
      if (!j->in_row || (J.nnz && !j->in_col))
        return bail(fail(SLIM_EDEVICE, "serve: out of device memory"));
      if (hipMemcpyAsync(j->in_row, J.row_off, 8 * (J.n + 1), hipMemcpyHostToDevice, s) !=
              hipSuccess ||
          (J.nnz && hipMemcpyAsync(j->in_col, J.col, 4 * J.nnz, hipMemcpyHostToDevice, s) !=
                        hipSuccess))
        return bail(fail(SLIM_EDEVICE, "serve: input upload failed"));
      in_row = static_cast<const int64_t*>(j->in_row);
      in_col = static_cast<const uint32_t*>(j->in_col);
    }
    GDesc& d = gs[i];
    d.nv = J.n;
    d.ne = J.nnz;
    d.thr = J.op == SLIM_OP_SPECTRAL ? 0 : threshold(J.p);
    d.ups = J.op == SLIM_OP_SPECTRAL ? J.p : 0.0;
    d.k0 = (uint32_t)J.seed;
    d.k1 = (uint32_t)(J.seed >> 32);
    d.op = (uint32_t)J.op;
    d.in_row = in_row;
    d.in_col = in_col;
    d.out_row = j->out_row;
    d.out_col = static_cast<uint32_t*>(j->out_col);
  }
  SetPlan P;
  if (int rc = plan_set(gs, P)) return bail(rc);
  const SetLayout L = set_layout(P.shape);
  const uint64_t stats_off = L.total;
  const uint64_t ws_bytes = L.total + sizeof(slim_stats_t) * cnt;
  uint64_t ws_got = 0;
  void* ws = S->arena.alloc(ws_bytes, &ws_got);
  if (!ws) return bail(fail(SLIM_EDEVICE, "serve: out of device memory (workspace)"));
  slim_stats_t* dstats = reinterpret_cast<slim_stats_t*>(static_cast<char*>(ws) + stats_off);
  for (uint32_t i = 0; i < cnt; ++i) P.gd[i].stats = dstats + i;
  std::vector<char> hdr;
  fill_header(P, L, S->knobs, ws, hdr);
  int rc = SLIM_OK;
  if (!grow_pinned(&W.pin_hdr, &W.pin_hdr_bytes, hdr.size()) ||
      !grow_pinned(&W.pin_stats, &W.pin_stats_bytes, sizeof(slim_stats_t) * cnt)) {
    rc = fail(SLIM_EDEVICE, "serve: pinned buffer allocation failed");
  } else {
    std::memcpy(W.pin_hdr, hdr.data(), hdr.size());
    if (hipMemcpyAsync(ws, W.pin_hdr, hdr.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = fail(SLIM_EDEVICE, "serve: header upload failed");
    } else {
      (void)hipGetLastError();
      run_set(P.shape, L, S->knobs, S->num_cu, ws, nullptr, nullptr, s, false);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess && eo_finish(P.shape, L, S->knobs, S->num_cu, ws, nullptr, nullptr, s))
        e = hipErrorUnknown;
      if (e == hipSuccess)
        e = hipMemcpyAsync(W.pin_stats, dstats, sizeof(slim_stats_t) * cnt,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = fail(SLIM_EDEVICE, "serve: batch failed: %s", hipGetErrorString(e));
    }
  }
  if (rc == SLIM_OK)
    for (uint32_t i = 0; i < cnt; ++i)
      batch[i]->stats = static_cast<const slim_stats_t*>(W.pin_stats)[i];
  (void)hipStreamSynchronize(s);  // nothing may still use ws or the pinned buffers
  S->arena.free(ws, ws_got);
  return rc;
}

void free_inputs(slim_server* S, Job* j) {
  S->arena.free(j->in_row, j->sz_in_row);
  S->arena.free(j->in_col, j->sz_in_col);
  j->in_row = j->in_col = nullptr;
}

void free_outputs(slim_server* S, Job* j) {
  S->arena.free(j->out_row, j->sz_out_row);
  S->arena.free(j->out_col, j->sz_out_col);
  j->out_row = j->out_col = nullptr;
}

void worker_main(slim_server* S, int wi) {
  (void)hipSetDevice(S->device);
  Worker& W = S->workers[wi];
  for (;;) {
    std::vector<Job*> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->ready.empty(); });
      if (S->stop) break;
      uint64_t N = 0, NNZ = 0;
      const double t = now_ms();
      while (!S->ready.empty() && batch.size() < S->cfg.max_batch) {
        Job* j = S->jobs[S->ready.front()].get();
        // Edge-Once jobs batch only with each other: their per-edge arrays
        // span the whole union, which the other jobs' reservations do not
        // cover, and their rounds end with host checks
        if (!batch.empty() &&
            (N + j->spec.n > 0xffffffffull || (NNZ + j->spec.nnz) / 2 > 0xffffffffull ||
             (j->spec.op == SLIM_OP_EOTR) != (batch[0]->spec.op == SLIM_OP_EOTR)))
          break;
        S->ready.pop_front();
        j->state = kRunning;
        j->t_start = t;
        N += j->spec.n;
        NNZ += j->spec.nnz;
        batch.push_back(j);
      }
      S->running += (uint32_t)batch.size();
    }
    const int rc = run_batch(S, W, batch);
    const double t = now_ms();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      ++S->batches;
      S->batch_jobs += batch.size();
      for (Job* j : batch) {
        free_inputs(S, j);
        if (rc != SLIM_OK) free_outputs(S, j);
        S->in_use -= j->res_ws + j->res_in;
        j->res_ws = j->res_in = 0;
        j->status = rc;
        j->state = kDone;
        j->t_done = t;
        S->finished.push_back(j->ticket);
        if (rc == SLIM_OK) {
          ++S->completed;
          S->lat.push_back(t - j->t_submit);
          S->edges += (double)(j->spec.nnz / 2);
        } else {
          ++S->failed;
        }
      }
      S->t_last = t;
      S->running -= (uint32_t)batch.size();
      admit(S);
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
}

void fill_result(const Job* j, slim_result_t* r) {
  std::memset(r, 0, sizeof(*r));
  r->status = j->status;
  r->row_off = static_cast<const int64_t*>(j->out_row);
  r->col = static_cast<const uint32_t*>(j->out_col);
  r->n = j->spec.n;
  r->stats = j->stats;
  r->queue_ms = j->t_start - j->t_submit;
  r->latency_ms = j->t_done - j->t_submit;
}

}  // namespace

extern "C" {

int slim_serve_create(const slim_serve_cfg_t* cfg, slim_server_t** out) {
  if (!out) return fail(SLIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(SLIM_EINVAL, "cfg is NULL");
  if (cfg->hbm_budget_bytes == 0 || cfg->pad != 0)
    return fail(SLIM_EINVAL, "cfg: hbm_budget_bytes must be > 0 and pad 0");
  if (cfg->n_streams > 16) return fail(SLIM_EINVAL, "cfg: n_streams must be <= 16");
  slim_server* S = new (std::nothrow) slim_server;
  if (!S) return fail(SLIM_ENOMEM, "out of host memory");
  S->cfg = *cfg;
  if (!S->cfg.max_slots) S->cfg.max_slots = 65536;
  if (!S->cfg.n_streams) S->cfg.n_streams = 2;
  if (!S->cfg.max_batch) S->cfg.max_batch = 4096;
  if (hipGetDevice(&S->device) != hipSuccess ||
      hipDeviceGetAttribute(&S->num_cu, hipDeviceAttributeMultiprocessorCount, S->device) !=
          hipSuccess) {
    delete S;
    return fail(SLIM_EDEVICE, "serve: device query failed");
  }
  {
    std::lock_guard<std::mutex> lk(tuning_mutex());
    S->knobs = tuning();
  }
  S->arena.set_cap(S->cfg.hbm_budget_bytes + S->cfg.hbm_budget_bytes / 8);
  S->workers.resize(S->cfg.n_streams);
  // pinned staging sized for the largest batch up front: growing it later
  // would free pinned memory, which waits for the device
  SetShape big;
  big.count = std::min<uint32_t>(S->cfg.max_batch, 65536);
  const uint64_t hdr_max = set_layout(big).hdr_bytes;
  for (auto& W : S->workers) {
    if (hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking) != hipSuccess ||
        !grow_pinned(&W.pin_hdr, &W.pin_hdr_bytes, hdr_max) ||
        !grow_pinned(&W.pin_stats, &W.pin_stats_bytes, sizeof(slim_stats_t) * big.count)) {
      for (auto& V : S->workers) {
        if (V.stream) (void)hipStreamDestroy(V.stream);
        if (V.pin_hdr) (void)hipHostFree(V.pin_hdr);
        if (V.pin_stats) (void)hipHostFree(V.pin_stats);
      }
      delete S;
      return fail(SLIM_EDEVICE, "serve: stream or pinned buffer creation failed");
    }
  }
  for (int i = 0; i < (int)S->workers.size(); ++i)
    S->workers[i].th = std::thread(worker_main, S, i);
  *out = S;
  return ok();
}

int slim_serve_submit(slim_server_t* S, const slim_job_t* job, uint64_t* ticket) {
  if (!S || !job || !ticket) return fail(SLIM_EINVAL, "NULL argument");
  const slim_job_t& J = *job;
  if (!op_valid(J.op) || J.pad || J.pad2)
    return fail(SLIM_EINVAL, "job: bad op %d", J.op);
  if (check_param(J.op, J.p)) return SLIM_EINVAL;
  if (J.where != SLIM_HOST && J.where != SLIM_DEVICE)
    return fail(SLIM_EINVAL, "job: where must be SLIM_HOST or SLIM_DEVICE");
  if (!J.row_off || (J.nnz && !J.col)) return fail(SLIM_EINVAL, "job: NULL CSR array");
  if (J.n > 0xffffffffull || J.nnz % 2 || J.nnz / 2 > 0xffffffffull || (J.n == 0 && J.nnz))
    return fail(SLIM_EINVAL, "job: n = %llu, nnz = %llu out of range", (unsigned long long)J.n,
                (unsigned long long)J.nnz);
  auto j = std::make_unique<Job>();
  j->spec = J;
  j->res_out = size_class(8 * (J.n + 1)) + (J.nnz ? size_class(4 * J.nnz) : 0);
  j->res_in = J.where == SLIM_HOST ? size_class(8 * (J.n + 1)) + (J.nnz ? size_class(4 * J.nnz) : 0)
                                   : 0;
  j->res_ws = ws_estimate(J);
  const uint64_t r = j->res_out + j->res_in + j->res_ws;
  if (r > S->cfg.hbm_budget_bytes)
    return fail(SLIM_EBUDGET, "job needs %llu bytes of device memory, budget is %llu",
                (unsigned long long)r, (unsigned long long)S->cfg.hbm_budget_bytes);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    j->ticket = S->next_ticket++;
    j->t_submit = now_ms();
    if (S->t_first < 0) S->t_first = j->t_submit;
    *ticket = j->ticket;
    S->pending.push_back(j->ticket);
    S->jobs.emplace(j->ticket, std::move(j));
    ++S->submitted;
    admit(S);
  }
  S->cv_work.notify_one();
  return ok();
}

int slim_serve_poll(slim_server_t* S, uint64_t ticket, slim_result_t* res) {
  if (!S || !res) return fail(SLIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return fail(SLIM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second->state != kDone) return SLIM_EAGAIN;
  fill_result(it->second.get(), res);
  return ok();
}

int slim_serve_wait(slim_server_t* S, uint64_t ticket, slim_result_t* res) {
  if (!S || !res) return fail(SLIM_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end())
      return fail(SLIM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state == kDone) {
      fill_result(it->second.get(), res);
      return ok();
    }
    if (S->stop) return fail(SLIM_EINVAL, "server is shutting down");
    S->cv_done.wait(lk);
  }
}

int slim_serve_next(slim_server_t* S, int64_t timeout_ms, uint64_t* ticket, slim_result_t* res) {
  if (!S || !ticket || !res) return fail(SLIM_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  const auto deadline =
      std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
  for (;;) {
    while (!S->finished.empty()) {
      const uint64_t t = S->finished.front();
      S->finished.pop_front();
      auto it = S->jobs.find(t);
      if (it == S->jobs.end()) continue;  // released before it was taken here
      *ticket = t;
      fill_result(it->second.get(), res);
      return ok();
    }
    if (S->stop) return fail(SLIM_EINVAL, "server is shutting down");
    if (timeout_ms == 0) return SLIM_EAGAIN;
    if (timeout_ms < 0) {
      S->cv_done.wait(lk);
    } else if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout &&
               S->finished.empty()) {
      return SLIM_EAGAIN;
    }
  }
}

int slim_serve_cancel(slim_server_t* S, uint64_t ticket) {
  if (!S) return fail(SLIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return fail(SLIM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Job* j = it->second.get();
  if (j->state == kQueued) {
    S->pending.erase(std::find(S->pending.begin(), S->pending.end(), ticket));
  } else if (j->state == kReady) {
    S->ready.erase(std::find(S->ready.begin(), S->ready.end(), ticket));
    S->in_use -= j->res_out + j->res_in + j->res_ws;
    --S->slots;
  } else {
    return SLIM_EAGAIN;
  }
  ++S->cancelled;
  S->jobs.erase(it);
  admit(S);
  S->cv_work.notify_all();
  return ok();
}

int slim_serve_copy(slim_server_t* S, uint64_t ticket, int64_t* row_off, uint32_t* col) {
  if (!S || !row_off) return fail(SLIM_EINVAL, "NULL argument");
  const void* src_row = nullptr;
  const void* src_col = nullptr;
  uint64_t n = 0, nnz_out = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end())
      return fail(SLIM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Job* j = it->second.get();
    if (j->state != kDone) return SLIM_EAGAIN;
    if (j->status != SLIM_OK) return fail(j->status, "the job failed");
    src_row = j->out_row;
    src_col = j->out_col;
    n = j->spec.n;
    nnz_out = 2 * j->stats.m_out;
  }
  if (nnz_out && !col) return fail(SLIM_EINVAL, "col is NULL");
  (void)hipSetDevice(S->device);
  if (hipMemcpy(row_off, src_row, 8 * (n + 1), hipMemcpyDefault) != hipSuccess ||
      (nnz_out && hipMemcpy(col, src_col, 4 * nnz_out, hipMemcpyDefault) != hipSuccess))
    return fail(SLIM_EDEVICE, "serve: result copy failed");
  return ok();
}

int slim_result_release(slim_server_t* S, uint64_t ticket) {
  if (!S) return fail(SLIM_EINVAL, "NULL argument");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end())
      return fail(SLIM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Job* j = it->second.get();
    if (j->state != kDone) return fail(SLIM_EAGAIN, "job %llu is not finished",
                                       (unsigned long long)ticket);
    free_outputs(S, j);
    S->in_use -= j->res_out;
    --S->slots;
    S->jobs.erase(it);
    admit(S);
  }
  S->cv_work.notify_all();
  return ok();
}

int slim_serve_stats(slim_server_t* S, slim_serve_stats_t* o) {
  if (!S || !o) return fail(SLIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(o, 0, sizeof(*o));
  o->submitted = S->submitted;
  o->completed = S->completed;
  o->failed = S->failed;
  o->cancelled = S->cancelled;
  o->queued = S->pending.size() + S->ready.size();
  o->running = S->running;
  o->batches = S->batches;
  o->mean_batch_jobs = S->batches ? (double)S->batch_jobs / (double)S->batches : 0.0;
  if (!S->lat.empty()) {
    std::vector<double> v = S->lat;
    auto pct = [&](double q) {
      const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * v.size()) - 1);
      std::nth_element(v.begin(), v.begin() + k, v.end());
      return v[k];
    };
    o->p50_ms = pct(0.50);
    o->p99_ms = pct(0.99);
    double sum = 0, mx = 0;
    for (double x : S->lat) {
      sum += x;
      mx = std::max(mx, x);
    }
    o->mean_ms = sum / (double)S->lat.size();
    o->max_ms = mx;
    const double span = (S->t_last - S->t_first) * 1e-3;
    if (span > 0) {
      o->jobs_per_s = (double)S->completed / span;
      o->edges_per_s = S->edges / span;
    }
  }
  o->hbm_in_use = S->in_use;
  o->hbm_peak = S->peak;
  o->hbm_budget = S->cfg.hbm_budget_bytes;
  return ok();
}

int slim_serve_reset_stats(slim_server_t* S) {
  if (!S) return fail(SLIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  S->lat.clear();
  S->submitted = S->completed = S->failed = S->cancelled = S->batches = S->batch_jobs = 0;
  S->t_first = -1;
  S->t_last = 0;
  S->edges = 0;
  S->peak = S->in_use;
  return ok();
}

void slim_serve_destroy(slim_server_t* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  for (auto& W : S->workers)
    if (W.th.joinable()) W.th.join();
  (void)hipSetDevice(S->device);
  for (auto& kv : S->jobs) {
    free_inputs(S, kv.second.get());
    free_outputs(S, kv.second.get());
  }
  S->jobs.clear();
  S->arena.release_all();
  for (auto& W : S->workers) {
    if (W.stream) (void)hipStreamDestroy(W.stream);
    if (W.pin_hdr) (void)hipHostFree(W.pin_hdr);
    if (W.pin_stats) (void)hipHostFree(W.pin_stats);
  }
  delete S;
}

}  // extern "C"
