// Host emulation of the HIP runtime calls and of the kernel launchers that the library's host
// sources use (test infrastructure; see hip/hip_runtime.h).  It exists to run the host code --
// the serving worker thread, its locks and buffer lifetimes, the batch schedule and the graph
// capture bookkeeping -- under ThreadSanitizer and AddressSanitizer on a machine without a GPU.
//
// Streams are asynchronous, as on the device: each stream has a thread of its own that runs the
// stream's work in order, after a short random delay per operation, while the caller goes on.  A
// copy between device memory and pinned host memory (hipHostMalloc) reads its source and writes
// its destination when it runs; as with the runtime's staged copies, a copy from pageable host
// memory takes its source when it is queued, and a copy into pageable host memory returns once
// it has run.  A launch runs its emulated
// kernel then, an event completes when the work recorded before it on its stream has run, and a
// stream that waits for an event holds its later work until then.  So a host write into a
// buffer that queued work still reads, a read of results before their stream was synchronised,
// or a missing wait between streams shows up as a data race (ThreadSanitizer), a use after free
// (AddressSanitizer) or a wrong result.  The null stream runs work at once in the caller.  A
// stream in capture mode, or one that joined a capture through an event recorded in it, records
// the work into the capture instead, and a launched graph runs the recorded work as one
// operation of the stream it is launched on.  "Device" memory is host memory.  The GA launchers
// emulate the job-table state machine of the real kernels (initial population, generations,
// local-search picks, the epilogue that counts evaluations, swaps populations, advances the
// generation and finishes the job) with values that depend only on a job's own seed, run,
// individual and generation, so a request's result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "internal.h"

struct Capture {
  std::vector<std::function<void()>> ops;
  std::vector<MockStream*> streams;
};

struct MockStream {
  Capture* cap = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  long long queued = 0, done = 0;   // operations queued and run so far
  bool quit = false;
  std::thread th;
};

struct MockEvent {
  Capture* cap = nullptr;
  MockStream* s = nullptr;          // recorded on s after `target` operations (null: complete)
  long long target = 0;
};

struct MockGraph {
  std::vector<std::function<void()>> ops;
};
struct MockGraphExec {
  std::vector<std::function<void()>> ops;
};

namespace {

std::mutex g_streams_mu;
std::set<MockStream*> g_streams;

// pinned host allocations: start -> size
std::mutex g_pinned_mu;
std::map<const char*, size_t> g_pinned;

bool is_pinned(const void* p) {
  const char* c = static_cast<const char*>(p);
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  auto it = g_pinned.upper_bound(c);
  if (it == g_pinned.begin()) return false;
  --it;
  return c < it->first + it->second;
}

void stream_main(MockStream* s) {
  std::mt19937 rng((unsigned)reinterpret_cast<uintptr_t>(s));
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv.wait(lk, [&] { return s->quit || !s->q.empty(); });
    if (s->q.empty()) return;
    std::function<void()> f = std::move(s->q.front());
    s->q.pop_front();
    lk.unlock();
    // the device's share of the operation: lets the host and the other streams run meanwhile
    std::this_thread::sleep_for(std::chrono::microseconds(rng() % 40));
    f();
    lk.lock();
    ++s->done;
    s->cv.notify_all();
  }
}

// Waits until stream s has run its first `target` operations.
void wait_for(MockStream* s, long long target) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&] { return s->done >= target; });
}

long long enqueue(MockStream* s, std::function<void()> f) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->q.push_back(std::move(f));
  s->cv.notify_all();
  return ++s->queued;
}

void sync_stream(MockStream* s) {
  long long target;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    target = s->queued;
  }
  wait_for(s, target);
}

// (holds the registry's lock, so no stream is destroyed meanwhile; stream threads never take it)
void sync_all() {
  std::lock_guard<std::mutex> lk(g_streams_mu);
  for (MockStream* s : g_streams) sync_stream(s);
}

// Work for stream s: recorded into its capture, run at once (null stream) or queued.
void run_or_record(hipStream_t s, std::function<void()> f) {
  if (s && s->cap)
    s->cap->ops.push_back(std::move(f));
  else if (!s)
    f();
  else
    enqueue(s, std::move(f));
}

bool capturing(hipStream_t s) { return s && s->cap; }

}  // namespace

hipError_t hipGetDevice(int* dev) {
  if (!dev) return hipErrorInvalidValue;
  *dev = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipDeviceSynchronize() {
  sync_all();
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated runtime error"; }

hipError_t hipMalloc(void** p, size_t bytes) {
  if (!p) return hipErrorInvalidValue;
  *p = std::aligned_alloc(256, (std::max<size_t>(bytes, 1) + 255) & ~size_t(255));
  if (!*p) return hipErrorOutOfMemory;
  std::memset(*p, 0xA5, bytes);   // device memory starts with no defined contents
  return hipSuccess;
}
// like the runtime's, waits for the device's queued work first
hipError_t hipFree(void* p) {
  sync_all();
  std::free(p);
  return hipSuccess;
}
hipError_t hipMallocAsync(void** p, size_t bytes, hipStream_t s) {
  if (capturing(s)) return hipErrorStreamCaptureUnsupported;
  return hipMalloc(p, bytes);
}
hipError_t hipFreeAsync(void* p, hipStream_t s) {
  if (capturing(s)) return hipErrorStreamCaptureUnsupported;
  run_or_record(s, [p] { std::free(p); });
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned[static_cast<const char*>(*p)] = std::max<size_t>(bytes, 1);
  }
  return e;
}
hipError_t hipHostFree(void* p) {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned.erase(static_cast<const char*>(p));
  }
  return hipFree(p);
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  if (bytes && (!dst || !src)) return hipErrorInvalidValue;
  sync_all();
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  if (bytes && (!dst || !src)) return hipErrorInvalidValue;
  if (capturing(s)) return hipErrorStreamCaptureUnsupported;   // the library records no copies
  if (!bytes) return hipSuccess;
  if (kind == hipMemcpyHostToDevice && !is_pinned(src)) {
    // staged: the pageable source is taken now
    auto staged = std::make_shared<std::vector<char>>(static_cast<const char*>(src),
                                                      static_cast<const char*>(src) + bytes);
    run_or_record(s, [dst, staged] { std::memmove(dst, staged->data(), staged->size()); });
    return hipSuccess;
  }
  run_or_record(s, [dst, src, bytes] { std::memmove(dst, src, bytes); });
  if (kind == hipMemcpyDeviceToHost && !is_pinned(dst) && s) sync_stream(s);   // pageable destination
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  if (!s) return hipErrorInvalidValue;
  MockStream* x = new MockStream();
  x->th = std::thread(stream_main, x);
  {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    g_streams.insert(x);
  }
  *s = x;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s || s->cap) return hipErrorInvalidValue;
  {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    g_streams.erase(s);
  }
  sync_stream(s);   // the runtime lets queued work finish
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->quit = true;
    s->cv.notify_all();
  }
  s->th.join();
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (capturing(s)) return hipErrorStreamCaptureUnsupported;
  if (s) sync_stream(s);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  if (!s || !e) return hipErrorInvalidValue;
  if (e->cap && s->cap != e->cap) {
    if (s->cap) return hipErrorInvalidValue;
    s->cap = e->cap;
    e->cap->streams.push_back(s);
    return hipSuccess;
  }
  if (s->cap) return hipSuccess;   // inside one capture the recorded order is kept
  if (e->s && e->s != s) {
    MockStream* src = e->s;
    const long long target = e->target;
    enqueue(s, [src, target] { wait_for(src, target); });
  }
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->cap) return hipErrorInvalidValue;
  s->cap = new Capture();
  s->cap->streams.push_back(s);
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* graph) {
  if (!s || !s->cap || !graph || s->cap->streams.front() != s) return hipErrorInvalidValue;
  Capture* c = s->cap;
  for (MockStream* x : c->streams) x->cap = nullptr;
  *graph = new MockGraph{std::move(c->ops)};
  delete c;
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  if (!e) return hipErrorInvalidValue;
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!e) return hipErrorInvalidValue;
  e->cap = s ? s->cap : nullptr;
  e->s = nullptr;
  e->target = 0;
  if (s && !s->cap) {
    std::lock_guard<std::mutex> lk(s->mu);
    e->s = s;
    e->target = s->queued;
  }
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (!e) return hipErrorInvalidValue;
  if (e->s) wait_for(e->s, e->target);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!ms || !a || !b) return hipErrorInvalidValue;
  if (a->s) wait_for(a->s, a->target);
  if (b->s) wait_for(b->s, b->target);
  *ms = 0.25f;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, void*, char*, size_t) {
  if (!exec || !graph) return hipErrorInvalidValue;
  *exec = new MockGraphExec{graph->ops};
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph) {
  delete graph;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  sync_all();   // a launched graph may still be running
  delete exec;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
  if (!exec) return hipErrorInvalidValue;
  const MockGraphExec* x = exec;
  run_or_record(s, [x] {
    for (const auto& f : x->ops) f();
  });
  return hipSuccess;
}

// ------------------------------------------------------------------ emulated kernels
namespace mdock {

namespace {

// a value in [-1, 1) from a job's own coordinates
float val(unsigned long long seed, long long a, long long b, long long c) {
  unsigned long long z = seed * 0x9E3779B97F4A7C15ull + (unsigned long long)a * 0xBF58476D1CE4E5B9ull +
                         (unsigned long long)b * 0x94D049BB133111EBull + (unsigned long long)c;
  z ^= z >> 31;
  z *= 0xD6E9F6B2A5E37A35ull;
  z ^= z >> 29;
  return (float)((double)(z >> 11) / (double)(1ull << 52)) * 2.f - 1.f;
}

long long job_rows(const JobDev& J) { return (long long)J.P.n_runs * J.P.pop_size; }

bool bad_blocks(const int2* blocks, int n) { return n < 0 || (n > 0 && !blocks); }

}  // namespace

hipError_t launch_eval(const LigDev& L, const RecDev&, int n, const float* genes, float* energy, float* grad,
                       hipStream_t s) {
  if (n < 0) return hipErrorInvalidValue;
  const int G = L.n_genes;
  run_or_record(s, [=] {
    for (int k = 0; k < n; ++k) {
      float e = 0.f;
      for (int g = 0; g < G; ++g) e += genes[(size_t)k * G + g] * genes[(size_t)k * G + g];
      energy[k] = e;
      if (grad)
        for (int g = 0; g < G; ++g) grad[(size_t)k * G + g] = 2.f * genes[(size_t)k * G + g];
    }
  });
  return hipSuccess;
}

hipError_t launch_pose(const LigDev& L, int n, const float* genes, float* xyz, hipStream_t s) {
  if (n < 0) return hipErrorInvalidValue;
  const int G = L.n_genes, N = L.n_atoms;
  run_or_record(s, [=] {
    for (int k = 0; k < n; ++k)
      for (int a = 0; a < N; ++a)
        for (int c = 0; c < 3; ++c) xyz[((size_t)k * N + a) * 3 + c] = genes[(size_t)k * G + (a + c) % G] + (float)a;
  });
  return hipSuccess;
}

hipError_t launch_local_search(const LigDev& L, const RecDev&, int n, const float* genes_in, float* genes_out,
                               float* energy_out, int iters, float, float, float* trace, float*, float*,
                               hipStream_t s) {
  if (n < 0 || iters < 1) return hipErrorInvalidValue;
  const int G = L.n_genes;
  run_or_record(s, [=] {
    for (int k = 0; k < n; ++k) {
      for (int g = 0; g < G; ++g) genes_out[(size_t)k * G + g] = 0.5f * genes_in[(size_t)k * G + g];
      energy_out[k] = -(float)k;
      if (trace)
        for (int t = 0; t < iters; ++t) trace[(size_t)k * iters + t] = -(float)k;
    }
  });
  return hipSuccess;
}

hipError_t launch_solis_wets(const LigDev& L, const RecDev& R, int n, const float* genes_in, float* genes_out,
                             float* energy_out, int n_evals, unsigned long long, float* trace, hipStream_t s) {
  return launch_local_search(L, R, n, genes_in, genes_out, energy_out, n_evals, 0.f, 0.f, trace, nullptr, nullptr, s);
}

hipError_t launch_ga_init(JobDev* jobs, const int2* blocks, int n_blocks, int, int wpb, int, const RecDev&,
                          hipStream_t s) {
  if (!jobs || bad_blocks(blocks, n_blocks) || wpb < 1) return hipErrorInvalidValue;
  run_or_record(s, [=] {
    for (int b = 0; b < n_blocks; ++b) {
      JobDev& J = jobs[blocks[b].x];
      if (J.state != kJobInit) continue;
      const int G = J.P.n_genes;
      for (long long w = blocks[b].y; w < blocks[b].y + wpb && w < job_rows(J); ++w) {
        for (int g = 0; g < G; ++g) J.genes[J.cur][w * G + g] = val(J.P.seed, w, g, 0);
        J.energy[J.cur][w] = val(J.P.seed, w, -1, 0);
        J.evals[w] = 1;
      }
    }
  });
  return hipSuccess;
}

hipError_t launch_ga_generation(JobDev* jobs, const int2* blocks, int n_blocks, int, int wpb, int, const RecDev&,
                                hipStream_t s) {
  if (!jobs || bad_blocks(blocks, n_blocks) || wpb < 1) return hipErrorInvalidValue;
  run_or_record(s, [=] {
    for (int b = 0; b < n_blocks; ++b) {
      JobDev& J = jobs[blocks[b].x];
      if (J.state != kJobRunning) continue;
      const int G = J.P.n_genes, nxt = J.cur ^ 1;
      for (long long w = blocks[b].y; w < blocks[b].y + wpb && w < job_rows(J); ++w) {
        for (int g = 0; g < G; ++g)
          J.genes[nxt][w * G + g] = 0.5f * J.genes[J.cur][w * G + g] + val(J.P.seed, w, g, J.gen);
        J.energy[nxt][w] = std::fmin(J.energy[J.cur][w], val(J.P.seed, w, -1, J.gen));
        J.evals[w] = 1;
      }
    }
  });
  return hipSuccess;
}

hipError_t launch_ga_ls_pick(JobDev* jobs, const int2* blocks, int n_blocks, hipStream_t s) {
  if (!jobs || bad_blocks(blocks, n_blocks)) return hipErrorInvalidValue;
  run_or_record(s, [=] {
    for (int b = 0; b < n_blocks; ++b) {
      JobDev& J = jobs[blocks[b].x];
      if (J.state != kJobRunning) continue;
      for (int run = blocks[b].y; run < blocks[b].y + kWavesPerBlock && run < J.P.n_runs; ++run)
        for (int k = 0; k < J.P.n_ls; ++k) J.ls_rows[run * J.P.n_ls + k] = run * J.P.pop_size + k % J.P.pop_size;
    }
  });
  return hipSuccess;
}

hipError_t launch_ga_local_search(JobDev* jobs, const int2* blocks, int n_blocks, int, int wpb, int wpp, int,
                                  int ls_method, const RecDev&, hipStream_t s) {
  if (!jobs || bad_blocks(blocks, n_blocks) || wpb < 1 || wpp < 1 || wpb % wpp) return hipErrorInvalidValue;
  if (ls_method != kLsAdadelta && ls_method != kLsSolisWets) return hipErrorInvalidValue;
  const int per_block = wpb / wpp;
  run_or_record(s, [=] {
    for (int b = 0; b < n_blocks; ++b) {
      JobDev& J = jobs[blocks[b].x];
      if (J.state != kJobRunning) continue;
      const long long searches = (long long)J.P.n_runs * J.P.n_ls;
      for (long long k = blocks[b].y; k < blocks[b].y + per_block && k < searches; ++k) {
        const int row = J.ls_rows[k];
        J.energy[J.cur ^ 1][row] -= 0.125f;
        J.evals[row] += J.P.ls_iters;
      }
    }
  });
  return hipSuccess;
}

hipError_t enable_large_lds() { return hipSuccess; }

namespace {

void advance_one(JobDev& J) {
  const int state = J.state;
  if (state != kJobInit && state != kJobRunning) return;
  for (int run = 0; run < J.P.n_runs; ++run) {
    long long sum = 0;
    for (int i = 0; i < J.P.pop_size; ++i) sum += J.evals[run * J.P.pop_size + i];
    J.evals_of_runs[run] = (state == kJobInit ? 0ll : J.evals_of_runs[run]) + sum;
  }
  int cur = J.cur, gen = J.gen;
  if (state == kJobInit) {
    gen = 1;
  } else {
    cur ^= 1;
    gen += 1;
  }
  const bool done = gen > J.planned;
  if (done) {
    const int G = J.P.n_genes;
    for (int run = 0; run < J.P.n_runs; ++run) {
      const long long base = (long long)run * J.P.pop_size;
      long long bi = base;
      for (long long i = base; i < base + J.P.pop_size; ++i)
        if (J.energy[cur][i] < J.energy[cur][bi]) bi = i;
      for (int g = 0; g < G; ++g) J.best_genes[run * G + g] = J.genes[cur][bi * G + g];
      if (J.best_xyz) {
        const int N = J.L.n_atoms;
        for (int a = 0; a < N; ++a)
          for (int c = 0; c < 3; ++c)
            J.best_xyz[((size_t)run * N + a) * 3 + c] = J.best_genes[run * G + (a + c) % G] + (float)a;
      }
      J.best_row[run] = (int)bi;
      J.best_energy[run] = J.energy[cur][bi];
    }
  }
  J.cur = cur;
  J.gen = gen;
  J.state = done ? kJobDone : kJobRunning;
}

}  // namespace

hipError_t launch_join(hipStream_t s) {
  run_or_record(s, [] {});
  return hipSuccess;
}

hipError_t launch_ga_advance(JobDev* jobs, int n_jobs, hipStream_t s) {
  if (!jobs || n_jobs < 0) return hipErrorInvalidValue;
  run_or_record(s, [=] {
    for (int k = 0; k < n_jobs; ++k) advance_one(jobs[k]);
  });
  return hipSuccess;
}

hipError_t launch_ga_advance_list(JobDev* jobs, const int2* list, int n, hipStream_t s) {
  if (!jobs || bad_blocks(list, n)) return hipErrorInvalidValue;
  run_or_record(s, [=] {
    for (int k = 0; k < n; ++k) advance_one(jobs[list[k].x]);
  });
  return hipSuccess;
}

}  // namespace mdock
