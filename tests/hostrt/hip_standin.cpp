// A host-only stand-in for the part of the HIP runtime that the library's host
// code calls.  It lets the library's real host code (geometry set-up, the
// apply launch sequences, the served-mode lanes) run on a machine without a
// GPU, under AddressSanitizer or ThreadSanitizer, with every kernel launch a
// no-op.  It takes the freedoms the HIP runtime is allowed to take, so that
// code relying on more than the API promises fails here:
//
//  * Stream work is deferred.  hipMemcpyAsync and hipMemsetAsync only queue
//    the operation; it executes, reading its source at that moment, when the
//    stream is synchronised (or an event on it is waited for).  A host buffer
//    handed to an asynchronous copy and freed before the synchronise is then
//    read after its release, which the sanitizer reports.
//  * "Device" memory is host memory from the sanitizer's allocator, so device
//    buffers freed while work on them is still queued are reported too.
//    hipFree waits for every stream first, as the real call does.
//  * Graph calls (capture, end of capture, instantiation, launch, destruction)
//    are treated as not safe to make from several threads at once: each keeps
//    a plain counter (a data race for ThreadSanitizer when two threads make
//    such calls without ordering them) and counts calls that overlap in time.
//  * hipMemsetAsync on a capturing stream is refused (a memset node in a
//    captured graph is avoided by the library's contract).
//
// standin_report() prints the counters the driver checks.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

struct Op {
  enum Kind { kCopy, kSet, kSet32, kEvent } kind;
  void* dst = nullptr;
  const void* src = nullptr;
  size_t n = 0;
  int value = 0;
  ihipEvent_t* ev = nullptr;
};

std::recursive_mutex g_mu;  // every stream queue and the allocation table
std::atomic<long> g_graph_inside{0};
std::atomic<long> g_graph_overlaps{0};
std::atomic<long> g_capture_memsets{0};
std::atomic<long> g_sync_in_capture{0};
long g_graph_calls = 0;  // deliberately unguarded: see the header comment

void run(const Op& op);

}  // namespace

struct ihipEvent_t {
  ihipStream_t* stream = nullptr;
};

struct ihipStream_t {
  std::deque<Op> q;
  ihipGraph* capturing = nullptr;
};

struct ihipGraph {
  std::vector<Op> ops;
};

struct hipGraphExec {
  std::vector<Op> ops;
};

namespace {

ihipStream_t g_null_stream;
std::vector<ihipStream_t*> g_streams;
std::unordered_map<void*, size_t> g_allocs;

ihipStream_t* real(hipStream_t s) { return s ? s : &g_null_stream; }

void run(const Op& op) {
  switch (op.kind) {
    case Op::kCopy: std::memcpy(op.dst, op.src, op.n); break;
    case Op::kSet: std::memset(op.dst, op.value, op.n); break;
    case Op::kSet32:
      for (size_t k = 0; k < op.n; ++k) std::memcpy(static_cast<char*>(op.dst) + 4 * k, &op.value, 4);
      break;
    case Op::kEvent: break;
  }
}

void drain_locked(ihipStream_t* s) {
  while (!s->q.empty()) {
    const Op op = s->q.front();
    s->q.pop_front();
    run(op);
  }
}

void drain_all_locked() {
  drain_locked(&g_null_stream);
  for (ihipStream_t* s : g_streams) drain_locked(s);
}

hipError_t enqueue(hipStream_t st, const Op& op) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t* s = real(st);
  if (s->capturing) {
    s->capturing->ops.push_back(op);
  } else {
    s->q.push_back(op);
  }
  return hipSuccess;
}

// Scope of one graph call: counts overlapping calls and touches the plain
// counter.  The short sleep widens the window in which an unserialised second
// call would overlap.
struct GraphCall {
  GraphCall() {
    if (g_graph_inside.fetch_add(1) != 0) g_graph_overlaps.fetch_add(1);
    ++g_graph_calls;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  ~GraphCall() { g_graph_inside.fetch_sub(1); }
};

struct LaunchConfig {
  dim3 grid, block;
  size_t shmem;
  hipStream_t stream;
};
thread_local std::vector<LaunchConfig> t_launch;

}  // namespace

extern "C" void standin_report(FILE* f) {
  std::fprintf(f, "standin graph_overlaps=%ld capture_memsets=%ld sync_in_capture=%ld\n", g_graph_overlaps.load(),
               g_capture_memsets.load(), g_sync_in_capture.load());
}

extern "C" long standin_violations(void) {
  return g_graph_overlaps.load() + g_capture_memsets.load() + g_sync_in_capture.load();
}

// ---- device, errors ----
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "stand-in error"; }

// ---- memory ----
hipError_t hipMalloc(void** p, size_t n) {
  const size_t bytes = ((n ? n : 1) + 255) & ~size_t(255);
  *p = std::aligned_alloc(256, bytes);
  if (!*p) return hipErrorOutOfMemory;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_allocs[*p] = bytes;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  drain_all_locked();  // hipFree waits for the device
  g_allocs.erase(p);
  std::free(p);
  return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }

// A __device__ variable's host-side shadow has the variable's size: it stands
// in for the device copy.
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) { return hipFree(p); }

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  Op op{Op::kCopy};
  op.dst = dst;
  op.src = src;
  op.n = n;
  return enqueue(s, op);
}

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  drain_locked(&g_null_stream);
  std::memcpy(dst, src, n);
  return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int value, size_t n, hipStream_t st) {
  {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (real(st)->capturing) {
      g_capture_memsets.fetch_add(1);
      return hipErrorStreamCaptureUnsupported;
    }
  }
  Op op{Op::kSet};
  op.dst = dst;
  op.value = value;
  op.n = n;
  return enqueue(st, op);
}

hipError_t hipMemsetD32Async(hipDeviceptr_t dst, int value, size_t count, hipStream_t st) {
  {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (real(st)->capturing) {
      g_capture_memsets.fetch_add(1);
      return hipErrorStreamCaptureUnsupported;
    }
  }
  Op op{Op::kSet32};
  op.dst = dst;
  op.value = value;
  op.n = count;
  return enqueue(st, op);
}

// ---- streams and events ----
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  *s = new ihipStream_t;
  g_streams.push_back(*s);
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  drain_locked(s);
  for (size_t k = 0; k < g_streams.size(); ++k)
    if (g_streams[k] == s) {
      g_streams.erase(g_streams.begin() + k);
      break;
    }
  delete s;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t st) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t* s = real(st);
  if (s->capturing) {
    g_sync_in_capture.fetch_add(1);
    return hipErrorStreamCaptureUnsupported;
  }
  drain_locked(s);
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t st) {
  {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    e->stream = real(st);
  }
  Op op{Op::kEvent};
  op.ev = e;
  return enqueue(st, op);
}

hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (e->stream && !e->stream->capturing) drain_locked(e->stream);
  return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  hipEventSynchronize(a);
  hipEventSynchronize(b);
  *ms = 0.0f;
  return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned int) {
  // the dependency is met by running the event's stream now
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (e->stream && !e->stream->capturing) drain_locked(e->stream);
  return hipSuccess;
}

// ---- graphs ----
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) {
  GraphCall gc;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t* s = real(st);
  if (s->capturing) return hipErrorIllegalState;
  s->capturing = new ihipGraph;
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* g) {
  GraphCall gc;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t* s = real(st);
  if (!s->capturing) return hipErrorIllegalState;
  *g = s->capturing;
  s->capturing = nullptr;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  GraphCall gc;
  *ex = new hipGraphExec;
  (*ex)->ops = g->ops;
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t st) {
  GraphCall gc;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  for (const Op& op : ex->ops) real(st)->q.push_back(op);
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
  GraphCall gc;
  delete ex;
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
  GraphCall gc;
  delete g;
  return hipSuccess;
}

// ---- kernel launches: recorded nowhere, executed never ----
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
  t_launch.push_back({grid, block, shmem, stream});
  return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shmem, hipStream_t* stream) {
  if (t_launch.empty()) return hipErrorInvalidConfiguration;
  const LaunchConfig c = t_launch.back();
  t_launch.pop_back();
  *grid = c.grid;
  *block = c.block;
  *shmem = c.shmem;
  *stream = c.stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void*, dim3, dim3, void**, size_t, hipStream_t) { return hipSuccess; }

extern "C" {
void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*, void*, void*,
                           int*) {}
void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}
void __hipUnregisterFatBinary(void**) {}
}
