// Served mode: operator sessions admitted into one HBM arena and run on lanes
// (a host thread and a stream each), each session's apply captured once as a
// HIP graph and replayed.  The kernels are those of sbie_apply, launched in the
// same order on the same data layout, so a session's results are bitwise those
// of a plain apply, alone or in the mix.  With batching a lane may hold several
// sessions of one operator, precision and order and run their applies together
// (apply_laplace_batch: one near and one far launch for all of them), again
// bitwise as their plain applies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "sbie_internal.h"

namespace sbie {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over one device allocation; freed ranges coalesce with
// their neighbours.  Offsets and lengths are multiples of kAlign.
struct Arena {
  char* base = nullptr;
  size_t size = 0, in_use = 0, peak = 0;
  std::map<size_t, size_t> free_ranges;  // offset -> length

  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, start = it->first + bytes;
      free_ranges.erase(it);
      if (rest) free_ranges.emplace(start, rest);
      in_use += bytes;
      peak = std::max(peak, in_use);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_ranges.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_ranges.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_ranges.erase(nx);
    }
    if (it != free_ranges.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_ranges.erase(it);
      }
    }
    in_use -= bytes;
  }
};

struct Job {
  const double* din = nullptr;
  double* dout = nullptr;
  bool devptr = false;
  bool done = false;
  sbie_status status = SBIE_OK;
  std::string err;
  sbie_apply_stats stats{};
};

using Clock = std::chrono::steady_clock;

int nrhs_of(int op) { return op == SBIE_OP_STOKES_S ? 3 : 1; }

constexpr int kServeBatch = 4;            // sessions one batching lane holds at most
constexpr int kServeTreeMin = 64;         // particles from which a tree session takes the tree
constexpr double kServeTheta = 0.6;       // the served tree's acceptance parameter, order and leaf size
constexpr int kServeOrder = 10, kServeLeaf = 2;
constexpr int64_t kBatchMaxNodes = 65536;  // larger sessions fill the device alone

// Whether a session may share a batched apply: a small S or D session (a
// larger one gains nothing from company and would only delay its partners)
// whose far field runs in one pair-kernel launch (T >= 32 and every partner
// offset in the reverse budget), the conditions of apply_laplace_batch.
bool batchable_shape(int M, int p, int op) {
  if (op != SBIE_OP_S && op != SBIE_OP_D) return false;
  const int T = (p + 1) * (2 * p + 2);
  if ((int64_t)M * T > kBatchMaxNodes) return false;
  const int pmax = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  return T >= 32 && pmax <= far_rev_slots(M, T);
}

}  // namespace
}  // namespace sbie

struct sbie_session {
  sbie_server* srv = nullptr;
  int64_t id = 0;
  std::vector<sbie::Particle> parts;
  int M = 0, p = 0, op = 0, prec = 0, nrhs = 1;
  double eta = 1.0;
  int64_t N = 0;
  uint64_t plan = 0, bytes = 0;  // geometry block, whole arena share
  size_t off = 0;
  bool admitted = false, closing = false, failed = false, counted_wait = false, batchable = false;
  bool tree_candidate = false, has_tree = false;  // far field through a tree in the arena
  size_t tree_off = 0, tree_bytes = 0;
  sbie_status fail = SBIE_OK;
  std::string fail_msg;
  sbie_geom* g = nullptr;
  double *d_in = nullptr, *d_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::deque<sbie::Job*> queue;
  int lane = -1;
  double open_us = 0, admit_us = 0, ready_us = 0;
};

struct sbie_server {
  int device = 0;
  bool graphs = false;
  bool batch = false;  // lanes may hold several compatible sessions
  bool tree = false;   // larger S and D sessions take their far field from a tree
  sbie::Arena arena;
  std::mutex mu;
  // Every HIP graph call of the lanes (capture, instantiation, launch,
  // destruction) is made under this lock: HIP does not promise that graph
  // calls from several threads at once are safe, so the lanes never overlap
  // them.  Launches only enqueue, so the lock is held for microseconds.
  std::mutex graph_mu;
  std::condition_variable cv_done;
  std::vector<std::unique_ptr<std::condition_variable>> lane_cv;
  std::deque<sbie_session*> pending;
  std::unordered_set<sbie_session*> sessions;
  int passes = 0;  // admissions in a row that passed the head of the queue
  std::vector<std::thread> threads;
  std::vector<sbie_ctx*> lane_ctx;
  std::vector<unsigned*> lane_status;  // pinned host words per lane, one per held session
  std::vector<sbie::BatchJobs> lane_jobs;  // batched-apply job tables per lane
  std::vector<bool> lane_idle;
  std::vector<int> lane_held;  // sessions each lane holds
  std::unordered_map<uint64_t, sbie::Job*> jobs;
  uint64_t next_ticket = 1;
  int64_t next_session = 1;
  bool stopping = false;
  sbie::Clock::time_point t0;
  int64_t n_active = 0, n_admitted = 0, n_passed = 0, n_waited = 0, n_applies = 0, n_batched = 0, n_tree = 0;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(sbie::Clock::now() - t0).count();
  }
  int lane_cap() const { return batch ? sbie::kServeBatch : 1; }
  // a lane that holds sessions admits more only when no lane is empty: the
  // sessions spread over the lanes first and share them only beyond that
  bool lane_may_admit(int lane) const {
    if (lane_held[lane] == 0) return true;
    if (lane_held[lane] >= lane_cap()) return false;
    for (int h : lane_held)
      if (h == 0) return false;
    return true;
  }
  // A session may be admitted or memory was returned: wake the lanes that
  // could take it.
  void wake_idle_lanes() {
    for (size_t k = 0; k < lane_cv.size(); ++k)
      if (lane_idle[k] || (batch && lane_may_admit((int)k))) lane_cv[k]->notify_one();
  }
};

namespace sbie {
namespace {

bool same_batch(const sbie_session* a, const sbie_session* b) {
  return a->batchable && b->batchable && a->op == b->op && a->prec == b->prec && a->p == b->p;
}

// Admission (lock held): the first pending session that fits the arena (and,
// for a lane that holds sessions, batches with them), where a session may pass
// the head of the queue only SBIE_MAX_PASS times in a row.
sbie_session* admit_locked(sbie_server* srv, int lane, const sbie_session* key) {
  for (size_t idx = 0; idx < srv->pending.size(); ++idx) {
    if (idx > 0 && srv->passes >= SBIE_MAX_PASS) break;
    sbie_session* s = srv->pending[idx];
    if (key && !same_batch(key, s)) continue;
    size_t off = 0;
    if (srv->arena.alloc(s->bytes, &off)) {
      s->off = off;
      s->admitted = true;
      s->lane = lane;
      s->admit_us = srv->now_us();
      srv->pending.erase(srv->pending.begin() + idx);
      if (idx == 0) {
        srv->passes = 0;
      } else {
        ++srv->passes;
        ++srv->n_passed;
      }
      ++srv->n_active;
      ++srv->n_admitted;
      return s;
    }
    if (!s->counted_wait) {
      s->counted_wait = true;
      ++srv->n_waited;
    }
  }
  return nullptr;
}

sbie_status launch_apply(sbie_session* s, hipStream_t st) {
  if (s->op == SBIE_OP_STOKES_S) return apply_stokes(s->g, s->prec, s->d_in, s->d_out, st, SBIE_PARTS_ALL, false, false);
  return apply_laplace(s->g, s->op, s->prec, s->d_in, s->d_out, st,
                       SBIE_PARTS_ALL | (s->has_tree ? SBIE_FAR_TREE : 0u), false);
}

// The tree of a session in the server's arena (lane thread, lock not held):
// the block is taken under the lock; if the arena has no room the session
// keeps the direct far field.
struct TreeArena {
  sbie_server* srv;
  sbie_session* s;
};

char* tree_block(void* ctx, size_t bytes) {
  TreeArena* ta = static_cast<TreeArena*>(ctx);
  std::lock_guard<std::mutex> lk(ta->srv->mu);
  const size_t b = align_up(bytes);
  size_t off = 0;
  if (!ta->srv->arena.alloc(b, &off)) return nullptr;
  ta->s->tree_off = off;
  ta->s->tree_bytes = b;
  return ta->srv->arena.base + off;
}

void build_session_tree(sbie_server* srv, sbie_session* s) {
  TreeArena ta{srv, s};
  TreeAlloc alloc;
  alloc.fn = tree_block;
  alloc.ctx = &ta;
  const sbie_status rc = build_tree(s->g, kServeTheta, kServeOrder, kServeLeaf, &alloc);
  s->has_tree = rc == SBIE_OK;
  if (!s->has_tree && s->tree_bytes) {
    // built no tree in a block it took: return the block
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->arena.release(s->tree_off, s->tree_bytes);
    s->tree_bytes = 0;
  }
  if (s->has_tree) {
    std::lock_guard<std::mutex> lk(srv->mu);
    ++srv->n_tree;
  }
}

// Geometry build in the session's arena share, then the graph capture (lane
// thread, lock not held).  A failure is kept and reported by every apply.
void build_session(sbie_server* srv, sbie_session* s, int lane) {
  sbie_ctx* lctx = srv->lane_ctx[lane];
  hipStream_t st = lctx->stream;
  char* blk = srv->arena.base + s->off;
  std::vector<Particle> parts = s->parts;
  // one stream per session: concurrency comes from the other lanes
  sbie_status rc = make_geometry(lctx, std::move(parts), s->p, s->eta, blk, s->plan, false, &s->g);
  if (rc == SBIE_OK && s->op == SBIE_OP_STOKES_S) rc = stokes_buffers(s->g);
  if (rc == SBIE_OK && s->tree_candidate) build_session_tree(srv, s);
  if (rc == SBIE_OK) {
    const size_t io = align_up(sizeof(double) * (size_t)s->nrhs * s->N);
    s->d_in = reinterpret_cast<double*>(blk + s->plan);
    s->d_out = reinterpret_cast<double*>(blk + s->plan + io);
  }
  if (rc == SBIE_OK && srv->graphs) {
    std::lock_guard<std::mutex> cap(srv->graph_mu);
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const sbie_status la = launch_apply(s, st);
      e = hipStreamEndCapture(st, &s->graph);
      if (la != SBIE_OK || e != hipSuccess) rc = la != SBIE_OK ? la : device_error(e, "hipStreamEndCapture");
    } else {
      rc = device_error(e, "hipStreamBeginCapture");
    }
    if (rc == SBIE_OK) {
      e = hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) rc = device_error(e, "hipGraphInstantiate");
    }
  }
  if (rc != SBIE_OK) {
    s->failed = true;
    s->fail = rc;
    s->fail_msg = sbie_last_error();
  }
  s->ready_us = srv->now_us();
}

// The queue of one apply on the lane's stream: stage in, graph replay (or the
// same launches), status word, stage out.
sbie_status enqueue_apply(sbie_server* srv, sbie_session* s, Job* j, hipStream_t st, unsigned* hs) {
  const size_t bytes = sizeof(double) * (size_t)s->nrhs * s->N;
  SBIE_HIP(hipMemcpyAsync(s->d_in, j->din, bytes, j->devptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (s->exec) {
    std::lock_guard<std::mutex> lk(srv->graph_mu);
    SBIE_HIP(hipGraphLaunch(s->exec, st));
  } else {
    const sbie_status rc = launch_apply(s, st);
    if (rc != SBIE_OK) return rc;
  }
  SBIE_HIP(hipMemcpyAsync(hs, s->g->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  SBIE_HIP(hipMemcpyAsync(j->dout, s->d_out, bytes, j->devptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  return SBIE_OK;
}

// The apply's outcome from its near-field status word; a set word is cleared
// for the next apply.
sbie_status status_of(sbie_session* s, unsigned status, hipStream_t st, std::string* err) {
  if (!status) return SBIE_OK;
  SBIE_HIP(hipMemsetAsync(s->g->d_status, 0, sizeof(unsigned), st));
  SBIE_HIP(hipStreamSynchronize(st));
  if (status & kStatExterior) {
    *err = "a near-field target lies inside its source spheroid";
    return SBIE_E_OVERLAP;
  }
  *err = "continued fraction for Q_N/Q_{N-1} did not converge at a near-field target";
  return SBIE_E_NUMERIC;
}

// One apply: its queue, then the wait.  The stream is synchronised on every
// path, so the caller's buffers are no longer read or written once the job is
// marked done.
sbie_status run_apply(sbie_server* srv, sbie_session* s, Job* j, int lane, std::string* err) {
  if (s->failed) {
    *err = s->fail_msg;
    return s->fail;
  }
  hipStream_t st = srv->lane_ctx[lane]->stream;
  unsigned* hs = srv->lane_status[lane];
  *hs = 0u;
  const sbie_status rc = enqueue_apply(srv, s, j, st, hs);
  const hipError_t se = hipStreamSynchronize(st);
  if (rc != SBIE_OK) {
    *err = sbie_last_error();
    return rc;
  }
  if (se != hipSuccess) {
    const sbie_status ds = device_error(se, "hipStreamSynchronize");
    *err = sbie_last_error();
    return ds;
  }
  return status_of(s, *hs, st, err);
}

// Batched applies (lock not held): every session's input, one
// apply_laplace_batch, every status word and output; then the wait.  Each
// session gets its own status, as from run_apply.
void run_batch(sbie_server* srv, const std::vector<sbie_session*>& ss, const std::vector<Job*>& js, int lane,
               std::vector<sbie_status>* rc, std::vector<std::string>* err) {
  const int n = (int)ss.size();
  hipStream_t st = srv->lane_ctx[lane]->stream;
  unsigned* hs = srv->lane_status[lane];
  auto enqueue = [&]() -> sbie_status {
    std::vector<sbie_geom*> gs(n);
    std::vector<const double*> din(n);
    std::vector<double*> dout(n);
    for (int k = 0; k < n; ++k) {
      sbie_session* s = ss[k];
      hs[k] = 0u;
      gs[k] = s->g;
      din[k] = s->d_in;
      dout[k] = s->d_out;
      SBIE_HIP(hipMemcpyAsync(s->d_in, js[k]->din, sizeof(double) * (size_t)s->N,
                              js[k]->devptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    }
    sbie_status q =
        apply_laplace_batch(gs.data(), n, ss[0]->op, ss[0]->prec, din.data(), dout.data(), &srv->lane_jobs[lane], st);
    if (q != SBIE_OK) return q;
    for (int k = 0; k < n; ++k) {
      sbie_session* s = ss[k];
      SBIE_HIP(hipMemcpyAsync(hs + k, s->g->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, st));
      SBIE_HIP(hipMemcpyAsync(js[k]->dout, s->d_out, sizeof(double) * (size_t)s->N,
                              js[k]->devptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    }
    return SBIE_OK;
  };
  const sbie_status q = enqueue();
  const hipError_t se = hipStreamSynchronize(st);
  rc->assign(n, SBIE_OK);
  err->assign(n, std::string());
  if (q != SBIE_OK || se != hipSuccess) {
    const sbie_status bad = q != SBIE_OK ? q : device_error(se, "hipStreamSynchronize");
    const std::string msg = sbie_last_error();
    for (int k = 0; k < n; ++k) {
      (*rc)[k] = bad;
      (*err)[k] = msg;
    }
    return;
  }
  for (int k = 0; k < n; ++k) (*rc)[k] = status_of(ss[k], hs[k], st, &(*err)[k]);
}

void teardown(sbie_server* srv, sbie_session* s) {
  if (s->exec || s->graph) {
    std::lock_guard<std::mutex> lk(srv->graph_mu);
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
  }
  s->exec = nullptr;
  s->graph = nullptr;
  destroy_geometry(s->g);
  s->g = nullptr;
}

// Completion of one apply (lock held).
void finish_job(sbie_server* srv, sbie_session* s, Job* j, int lane, sbie_status rc, const std::string& err) {
  j->status = rc;
  j->err = err;
  j->stats.end_us = srv->now_us();
  j->stats.session = s->id;
  j->stats.lane = lane;
  j->stats.status = rc;
  j->stats.open_us = s->open_us;
  j->stats.admit_us = s->admit_us;
  j->stats.ready_us = s->ready_us;
  j->done = true;
  ++srv->n_applies;
}

// A lane: admits sessions (one, or with batching up to kServeBatch of one
// kind), runs their applies in submission order per session (the front
// applies of all its sessions together when there are several), and tears a
// session down once it is closed and drained.
void lane_main(sbie_server* srv, int lane) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  std::vector<sbie_session*> held;
  for (;;) {
    if (!srv->stopping && srv->lane_may_admit(lane)) {
      sbie_session* s = admit_locked(srv, lane, held.empty() ? nullptr : held[0]);
      if (s) {
        held.push_back(s);
        srv->lane_held[lane] = (int)held.size();
        srv->lane_idle[lane] = false;
        lk.unlock();
        build_session(srv, s, lane);
        lk.lock();
        continue;
      }
    }
    // the sessions with queued applies; a failed one answers at once, alone
    std::vector<sbie_session*> ready;
    sbie_session* failed = nullptr;
    for (sbie_session* s : held) {
      if (s->queue.empty()) continue;
      if (s->failed && !failed) failed = s;
      if (!s->failed) ready.push_back(s);
    }
    if (failed || ready.size() == 1) {
      sbie_session* s = failed ? failed : ready[0];
      Job* j = s->queue.front();
      s->queue.pop_front();
      j->stats.start_us = srv->now_us();
      lk.unlock();
      std::string err;
      const sbie_status rc = run_apply(srv, s, j, lane, &err);
      lk.lock();
      finish_job(srv, s, j, lane, rc, err);
      srv->cv_done.notify_all();
      continue;
    }
    if (ready.size() > 1) {
      std::vector<Job*> js;
      for (sbie_session* s : ready) {
        js.push_back(s->queue.front());
        s->queue.pop_front();
        js.back()->stats.start_us = srv->now_us();
      }
      lk.unlock();
      std::vector<sbie_status> rc;
      std::vector<std::string> err;
      run_batch(srv, ready, js, lane, &rc, &err);
      lk.lock();
      for (size_t k = 0; k < ready.size(); ++k) finish_job(srv, ready[k], js[k], lane, rc[k], err[k]);
      srv->n_batched += (int64_t)ready.size();
      srv->cv_done.notify_all();
      continue;
    }
    // closed (or stopping) and drained: tear down, return the memory
    bool released = false;
    for (size_t k = 0; k < held.size(); ++k) {
      sbie_session* s = held[k];
      if (!(s->closing || srv->stopping)) continue;
      held.erase(held.begin() + k);
      srv->lane_held[lane] = (int)held.size();
      lk.unlock();
      teardown(srv, s);
      lk.lock();
      srv->arena.release(s->off, s->bytes);
      if (s->tree_bytes) srv->arena.release(s->tree_off, s->tree_bytes);
      --srv->n_active;
      srv->sessions.erase(s);
      delete s;
      released = true;
      break;
    }
    if (released) {
      srv->wake_idle_lanes();  // memory returned: waiting sessions may fit now
      continue;
    }
    if (held.empty() && srv->stopping) break;
    srv->lane_idle[lane] = held.empty();
    srv->lane_cv[lane]->wait(lk);
  }
}

void free_batch_jobs(sbie_server* srv) {
  for (BatchJobs& b : srv->lane_jobs) {
    if (b.h_far) (void)hipHostFree(b.h_far);
    if (b.h_near) (void)hipHostFree(b.h_near);
    if (b.d_far) (void)hipFree(b.d_far);
    if (b.d_near) (void)hipFree(b.d_near);
    b = BatchJobs();
  }
}

sbie_status invalid_arg(const char* msg) {
  set_error(msg);
  return SBIE_E_INVALID;
}

}  // namespace
}  // namespace sbie

using namespace sbie;

extern "C" {

uint64_t sbie_session_bytes(int32_t M, int32_t p, sbie_op op) {
  if (M < 1 || p < 1 || p > kMaxP) return 0;
  const int64_t N = (int64_t)M * (p + 1) * (2 * p + 2);
  const uint64_t plan = plan_bytes(M, p, op == SBIE_OP_STOKES_S);
  return plan + 2 * align_up(sizeof(double) * (size_t)nrhs_of(op) * N);
}

sbie_status sbie_server_create(sbie_ctx* ctx, int32_t max_sessions, uint64_t hbm_budget_bytes, uint32_t flags,
                               sbie_server** out) {
  if (!out) return invalid_arg("out is NULL");
  *out = nullptr;
  if (!ctx) return invalid_arg("ctx is NULL");
  if (max_sessions < 1 || max_sessions > 64) return invalid_arg("max_sessions must be in [1, 64]");
  if (hbm_budget_bytes < (1u << 20)) return invalid_arg("the HBM budget must be at least 1 MiB");
  SBIE_HIP(hipSetDevice(ctx->device));
  sbie_server* srv = new (std::nothrow) sbie_server;
  if (!srv) return SBIE_E_NOMEM;
  srv->device = ctx->device;
  srv->graphs = (flags & SBIE_SERVER_GRAPHS) != 0;
  srv->batch = (flags & SBIE_SERVER_BATCH) != 0;
  srv->tree = (flags & SBIE_SERVER_TREE) != 0;
  srv->t0 = Clock::now();
  const size_t bytes = align_up(hbm_budget_bytes);
  hipError_t e = hipMalloc((void**)&srv->arena.base, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete srv;
    set_error("device allocation of the " + std::to_string(bytes) + "-byte arena failed");
    return SBIE_E_NOMEM;
  }
  srv->arena.size = bytes;
  srv->arena.free_ranges.emplace(0, bytes);
  auto fail = [&](sbie_status st) {
    for (sbie_ctx* c : srv->lane_ctx) sbie_ctx_destroy(c);
    for (unsigned* h : srv->lane_status) (void)hipHostFree(h);
    free_batch_jobs(srv);
    (void)hipFree(srv->arena.base);
    delete srv;
    return st;
  };
  for (int k = 0; k < max_sessions; ++k) {
    sbie_ctx* c = nullptr;
    sbie_status st = sbie_ctx_create(ctx->device, &c);
    if (st != SBIE_OK) return fail(st);
    srv->lane_ctx.push_back(c);
    unsigned* h = nullptr;
    e = hipHostMalloc((void**)&h, sizeof(unsigned) * kServeBatch, hipHostMallocDefault);
    if (e != hipSuccess) return fail(device_error(e, "hipHostMalloc"));
    srv->lane_status.push_back(h);
    srv->lane_jobs.emplace_back();
    if (srv->batch) {
      BatchJobs& b = srv->lane_jobs.back();
      if ((e = hipHostMalloc((void**)&b.h_far, sizeof(FarJob) * kServeBatch, hipHostMallocDefault)) != hipSuccess ||
          (e = hipHostMalloc((void**)&b.h_near, sizeof(NearJob) * kServeBatch, hipHostMallocDefault)) != hipSuccess ||
          (e = hipMalloc((void**)&b.d_far, sizeof(FarJob) * kServeBatch)) != hipSuccess ||
          (e = hipMalloc((void**)&b.d_near, sizeof(NearJob) * kServeBatch)) != hipSuccess)
        return fail(device_error(e, "batch job tables"));
      b.cap = kServeBatch;
    }
    srv->lane_cv.emplace_back(new std::condition_variable);
    srv->lane_idle.push_back(false);
    srv->lane_held.push_back(0);
  }
  for (int k = 0; k < max_sessions; ++k) srv->threads.emplace_back(lane_main, srv, k);
  *out = srv;
  return SBIE_OK;
}

void sbie_server_destroy(sbie_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    for (sbie_session* s : srv->pending) {
      for (Job* j : s->queue) {
        j->status = SBIE_E_STATE;
        j->err = "the server stopped before the session was admitted";
        j->stats.status = SBIE_E_STATE;
        j->done = true;
      }
      srv->sessions.erase(s);
      delete s;
    }
    srv->pending.clear();
    for (auto& cv : srv->lane_cv) cv->notify_one();
    srv->cv_done.notify_all();
  }
  for (auto& t : srv->threads) t.join();
  (void)hipSetDevice(srv->device);
  for (auto& kv : srv->jobs) delete kv.second;
  for (sbie_ctx* c : srv->lane_ctx) sbie_ctx_destroy(c);
  for (unsigned* h : srv->lane_status) (void)hipHostFree(h);
  free_batch_jobs(srv);
  (void)hipFree(srv->arena.base);
  delete srv;
}

sbie_status sbie_session_open(sbie_server* srv, const double* centers, const double* quats, const double* A,
                              const double* C, int32_t M, int32_t p, double eta, sbie_op op, sbie_precision prec,
                              sbie_session** out) {
  if (!out) return invalid_arg("out is NULL");
  *out = nullptr;
  if (!srv) return invalid_arg("server is NULL");
  if (op != SBIE_OP_S && op != SBIE_OP_D && op != SBIE_OP_STOKES_S) return invalid_arg("unknown operator");
  if (prec != SBIE_FP64 && prec != SBIE_MIXED) return invalid_arg("unknown precision");
  std::vector<Particle> parts;
  sbie_status st = check_particles(centers, quats, A, C, M, p, eta, &parts);
  if (st != SBIE_OK) return st;
  sbie_session* s = new (std::nothrow) sbie_session;
  if (!s) return SBIE_E_NOMEM;
  s->srv = srv;
  s->parts = std::move(parts);
  s->M = M;
  s->p = p;
  s->eta = eta;
  s->op = (int)op;
  s->prec = (int)prec;
  s->nrhs = nrhs_of(op);
  s->N = (int64_t)M * (p + 1) * (2 * p + 2);
  s->plan = plan_bytes(M, p, op == SBIE_OP_STOKES_S);
  s->bytes = sbie_session_bytes(M, p, op);
  s->tree_candidate = srv->tree && (op == SBIE_OP_S || op == SBIE_OP_D) && M >= kServeTreeMin;
  s->batchable = srv->batch && !s->tree_candidate && batchable_shape(M, p, (int)op);
  if (s->bytes > srv->arena.size) {
    set_error("the session needs " + std::to_string(s->bytes) + " bytes, more than the whole arena");
    delete s;
    return SBIE_E_BUDGET;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stopping) {
    delete s;
    set_error("the server is stopping");
    return SBIE_E_STATE;
  }
  s->id = srv->next_session++;
  s->open_us = srv->now_us();
  srv->pending.push_back(s);
  srv->sessions.insert(s);
  srv->wake_idle_lanes();
  *out = s;
  return SBIE_OK;
}

sbie_status sbie_session_apply(sbie_session* s, const double* density, double* potential, uint32_t flags,
                               uint64_t* ticket) {
  if (!s || !ticket) return invalid_arg("session or ticket is NULL");
  if (!density || !potential) return invalid_arg("density or potential is NULL");
  sbie_server* srv = s->srv;
  Job* j = new (std::nothrow) Job;
  if (!j) return SBIE_E_NOMEM;
  j->din = density;
  j->dout = potential;
  j->devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (s->closing || srv->stopping) {
    delete j;
    set_error("the session is closing");
    return SBIE_E_STATE;
  }
  j->stats.submit_us = srv->now_us();
  *ticket = srv->next_ticket++;
  srv->jobs.emplace(*ticket, j);
  s->queue.push_back(j);
  if (s->admitted) srv->lane_cv[s->lane]->notify_one();
  return SBIE_OK;
}

sbie_status sbie_session_close(sbie_session* s) {
  if (!s) return invalid_arg("session is NULL");
  sbie_server* srv = s->srv;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (s->closing) {
    set_error("the session is already closing");
    return SBIE_E_STATE;
  }
  if (!s->admitted && s->queue.empty()) {
    // never admitted and nothing to run: drop it from the queue
    srv->pending.erase(std::find(srv->pending.begin(), srv->pending.end(), s));
    srv->sessions.erase(s);
    delete s;
    srv->wake_idle_lanes();
    return SBIE_OK;
  }
  s->closing = true;
  if (s->admitted) srv->lane_cv[s->lane]->notify_one();
  return SBIE_OK;
}

sbie_status sbie_wait(sbie_server* srv, uint64_t ticket, int64_t timeout_us, sbie_apply_stats* stats) {
  if (!srv) return invalid_arg("server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return invalid_arg("unknown ticket");
  // the Job stays at its address; map iterators do not survive the wait (other
  // threads insert tickets meanwhile and the table may rehash)
  Job* j = it->second;
  auto done = [j] { return j->done; };
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, done);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
    set_error("the apply has not finished");
    return SBIE_E_TIMEOUT;
  }
  if (stats) *stats = j->stats;
  const sbie_status st = j->status;
  if (st != SBIE_OK) set_error(j->err);
  srv->jobs.erase(ticket);
  delete j;
  return st;
}

sbie_status sbie_server_get_info(sbie_server* srv, sbie_server_info* out) {
  if (!srv || !out) return invalid_arg("server or out is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  out->budget_bytes = srv->arena.size;
  out->in_use_bytes = srv->arena.in_use;
  out->peak_bytes = srv->arena.peak;
  out->pending = (int64_t)srv->pending.size();
  out->active = srv->n_active;
  out->admitted = srv->n_admitted;
  out->passed = srv->n_passed;
  out->waited = srv->n_waited;
  out->applies = srv->n_applies;
  out->lanes = (int32_t)srv->threads.size();
  out->graphs = srv->graphs ? 1 : 0;
  out->batched = srv->n_batched;
  out->tree_sessions = srv->n_tree;
  return SBIE_OK;
}

}  // extern "C"
