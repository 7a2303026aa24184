// Continuous-batching docking server of libmdock (md_server_* in include/mdock.h).
//
// The paper's screening workflow docks a large, heterogeneous stream of ligands against one
// receptor, which makes scheduling and load balance part of the problem (introduction, the
// high-throughput workflow figure and the paragraph on heterogeneously sized ligands).  Here
// requests arrive while others run: a worker thread admits queued requests into free slots as
// long as their device buffers fit in a fixed HBM pool, advances every resident request per tick
// through the same job-table kernels as md_dock_batch, and retires finished requests as soon as
// their tick is done, so their slots and memory are reused.  Ticks are pipelined two deep: the
// next tick is queued on the device before the host reads the previous tick's job table and
// copies out its finished results (on a stream of its own), so the device does not wait for the
// host between ticks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "mdock.h"

namespace mdock {
// shared with api.cpp
md_status server_fail(md_status st, const std::string& msg);
int n_local_search_of(const md_dock_params* p);
std::string check_dock_params(const md_dock_params* p);
}  // namespace mdock

using namespace mdock;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// With graphs, a tick advances each size class by up to this many generations: cheap classes
// run several while the most expensive runs one, so the device stays busy through its tail.
constexpr int kTickMaxGenerations = 8;

// First-fit allocator over one device pool (offsets only).
class Pool {
 public:
  explicit Pool(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

enum ReqState { kQueued, kResident, kFinished, kCanceled, kFailed };

struct Request {
  unsigned long long ticket = 0;
  // the ligand, read only while the request holds it (queued or resident: see drop_hold); the
  // result shape is kept apart so finished requests never touch the ligand again
  const md_ligand* lig = nullptr;
  bool held = false;
  int n_genes = 0, n_atoms = 0;
  md_dock_params params{};
  ReqState state = kQueued;
  bool cancel_requested = false;   // resident: leaves its slot once its entry is cleared
  long long cancel_tick = -1;      // the tick queued after its entry was cleared
  int slot = -1;
  size_t off = 0, bytes = 0;
  // offsets inside the request's pool block
  size_t o_ga, o_gb, o_ea, o_eb, o_ev, o_er, o_lsr, o_br, o_be, o_bg, o_bx;
  int planned = 0;
  double t_submit = 0, t_start = 0, t_end = 0;
  // results (runs sorted by energy)
  std::vector<float> best_energy, best_genes, best_xyz;
  std::vector<int> run_index;
  std::vector<long long> evals;
  std::string error;
};

}  // namespace

struct md_server {
  const md_receptor* rec = nullptr;
  md_server_params params{};
  int device = 0;
  hipStream_t stream = nullptr;
  char* pool_base = nullptr;
  std::unique_ptr<Pool> pool;
  JobDev* d_table = nullptr;     // [max_slots]
  JobDev* h_table = nullptr;     // pinned: the host's copy of every entry
  JobDev* h_up[2] = {nullptr, nullptr};     // pinned: entries uploaded before tick t, for t even / odd
                                            //     (reused only after that tick is done)
  JobDev* h_tick[2] = {nullptr, nullptr};   // pinned: the table after tick t, for t even / odd
  hipEvent_t tick_done[2] = {nullptr, nullptr};
  hipStream_t copy_stream = nullptr;        // result copies, beside the next tick
  int2* d_blocks = nullptr;
  size_t blocks_cap = 0;
  std::vector<std::shared_ptr<Request>> slots;   // resident request per slot (or null)
  // launch schedule of the resident set, rebuilt when the set changes; `graph` provides the
  // branch streams and fork/join events of the direct launch
  bool resident_changed = true;
  GenSchedule sched;
  GenGraph graph;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<unsigned long long, std::shared_ptr<Request>> requests;
  unsigned long long next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  long long ticks = 0, completed = 0;
  double busy_s = 0;
  std::string fatal;
};

namespace {

// The request no longer reads its ligand (it left the queue or its slot): release the hold
// taken at submit.  Caller holds the server lock.
void drop_hold(Request& r) {
  if (r.held) {
    r.lig->holds.fetch_sub(1);
    r.held = false;
  }
}

void layout(Request& r) {
  const LigDev& L = r.lig->dev;
  const md_dock_params& p = r.params;
  const size_t rows = (size_t)p.n_runs * p.pop_size;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = (off + b + 15) & ~size_t(15);
    return o;
  };
  r.o_ga = take(rows * L.n_genes * 4);
  r.o_gb = take(rows * L.n_genes * 4);
  r.o_ea = take(rows * 4);
  r.o_eb = take(rows * 4);
  r.o_ev = take(rows * 4);
  r.o_er = take((size_t)p.n_runs * 8);
  r.o_lsr = take((size_t)p.n_runs * std::max(n_local_search_of(&p), 1) * 4);
  r.o_br = take((size_t)p.n_runs * 4);
  r.o_be = take((size_t)p.n_runs * 4);
  r.o_bg = take((size_t)p.n_runs * L.n_genes * 4);
  r.o_bx = take((size_t)p.n_runs * L.n_atoms * 12);
  r.bytes = off;
}

JobDev make_job(md_server* s, const Request& r) {
  JobDev J{};
  const md_dock_params& p = r.params;
  char* w = s->pool_base + r.off;
  J.L = r.lig->dev;
  GaDev& P = J.P;
  P.n_runs = p.n_runs;
  P.pop_size = p.pop_size;
  P.n_genes = J.L.n_genes;
  P.n_ls = n_local_search_of(&p);
  P.ls_iters = p.ls_iters;
  P.ls_method = p.ls_method;
  P.elitism = p.elitism;
  P.rho = p.rho;
  P.eps = p.eps;
  P.crossover_rate = p.crossover_rate;
  P.mutation_rate = p.mutation_rate;
  P.tournament_rate = p.tournament_rate;
  P.mut_trans = p.mut_trans;
  P.mut_rot = p.mut_rot;
  P.mut_tors = p.mut_tors;
  P.seed = p.seed;
  J.genes[0] = reinterpret_cast<float*>(w + r.o_ga);
  J.genes[1] = reinterpret_cast<float*>(w + r.o_gb);
  J.energy[0] = reinterpret_cast<float*>(w + r.o_ea);
  J.energy[1] = reinterpret_cast<float*>(w + r.o_eb);
  J.evals = reinterpret_cast<int*>(w + r.o_ev);
  J.evals_of_runs = reinterpret_cast<long long*>(w + r.o_er);
  J.ls_rows = reinterpret_cast<int*>(w + r.o_lsr);
  J.best_row = reinterpret_cast<int*>(w + r.o_br);
  J.best_energy = reinterpret_cast<float*>(w + r.o_be);
  J.best_genes = reinterpret_cast<float*>(w + r.o_bg);
  J.best_xyz = reinterpret_cast<float*>(w + r.o_bx);
  J.gen = 0;
  J.cur = 0;
  J.planned = r.planned;
  J.state = kJobInit;
  return J;
}

// Queues one tick: every resident request advances by one phase sequence.  With use_graphs the
// size classes' chains are launched directly as parallel branches (fork/join events over the
// branch streams), several generations for the cheap classes; the worker captures no graph (graph
// capture in this thread coincided with two host crashes whose cause is not known; md_dock_batch
// captures on the caller's thread).  The tick ends with a copy of the job table into
// h_tick[t & 1] and the event tick_done[t & 1].  Returns the HIP status.
// jobs: the resident set when it changed since the last tick (taken under the server's lock), or
// null to keep the schedule.
hipError_t queue_tick(md_server* s, long long t, const std::vector<SchedJob>* jobs, bool any_init, bool any_running) {
  const int n_slots = (int)s->slots.size();
  hipError_t e = hipSuccess;
  if (jobs) {
    build_schedule(*jobs, s->sched, (s->params.use_graphs && use_graphs()) ? kTickMaxGenerations : 0, 1);
    const size_t nb = s->sched.blocks.size();
    if (nb > s->blocks_cap) {
      // the tick in flight reads the block table: let it finish before the buffer goes
      e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return e;
      if (s->d_blocks) (void)hipFree(s->d_blocks);
      s->blocks_cap = std::max<size_t>(nb, 2 * s->blocks_cap);
      e = hipMalloc(&s->d_blocks, s->blocks_cap * sizeof(int2));
      if (e != hipSuccess) {
        s->d_blocks = nullptr;
        s->blocks_cap = 0;
        return e;
      }
    }
    // stream-ordered after the tick in flight, which still reads the old table
    if (nb) e = hipMemcpyAsync(s->d_blocks, s->sched.blocks.data(), nb * sizeof(int2), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return e;
  }
  const RecDev& R = s->rec->dev;
  if (any_init) e = launch_init_phase(s->sched, s->d_table, s->d_blocks, R, s->stream, nullptr);
  if (e == hipSuccess) {
    if (!any_running) {
      e = launch_ga_advance(s->d_table, n_slots, s->stream);
    } else if (s->params.use_graphs && use_graphs()) {
      e = s->graph.launch_direct(s->sched, s->d_table, s->d_blocks, R, s->stream);
    } else {
      e = launch_generation_phase(s->sched, s->d_table, s->d_blocks, R, s->stream, nullptr);
    }
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->h_tick[t & 1], s->d_table, sizeof(JobDev) * n_slots, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipEventRecord(s->tick_done[t & 1], s->stream);
  return e;
}

// Copy a finished request's results to the host on the copy stream, after the tick that finished
// it (the tick queued behind it skips the request).  Called by the worker without the lock.
hipError_t collect(md_server* s, Request& r, hipEvent_t finished_tick) {
  const LigDev& L = r.lig->dev;
  const int runs = r.params.n_runs, G = L.n_genes, N = L.n_atoms;
  char* w = s->pool_base + r.off;
  // the generation epilogue that finished the request wrote its best genes, energies and poses
  std::vector<float> be(runs), bg((size_t)runs * G), bx((size_t)runs * N * 3);
  std::vector<long long> er(runs);
  hipStream_t cs = s->copy_stream;
  hipError_t e = hipStreamWaitEvent(cs, finished_tick, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(be.data(), w + r.o_be, runs * 4, hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess) e = hipMemcpyAsync(bg.data(), w + r.o_bg, bg.size() * 4, hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess) e = hipMemcpyAsync(bx.data(), w + r.o_bx, bx.size() * 4, hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess) e = hipMemcpyAsync(er.data(), w + r.o_er, runs * 8, hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess) e = hipStreamSynchronize(cs);
  if (e != hipSuccess) return e;
  std::vector<int> order(runs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return be[a] < be[b]; });
  r.best_energy.resize(runs);
  r.best_genes.resize((size_t)runs * G);
  r.best_xyz.resize((size_t)runs * N * 3);
  r.run_index.resize(runs);
  r.evals.resize(runs);
  for (int k = 0; k < runs; ++k) {
    const int q = order[k];
    r.best_energy[k] = be[q];
    std::memcpy(&r.best_genes[(size_t)k * G], &bg[(size_t)q * G], (size_t)G * 4);
    std::memcpy(&r.best_xyz[(size_t)k * N * 3], &bx[(size_t)q * N * 3], (size_t)N * 12);
    r.run_index[k] = q;
    r.evals[k] = er[q];
  }
  return hipSuccess;
}

// The worker: each pass (1) admits queued requests and clears the entries of canceled ones,
// (2) queues tick t for the resident requests, (3) waits for tick t - 1, retires the requests it
// finished (results copied out beside tick t) and frees the slots of requests canceled before it.
// Tick t - 1's table is read only for the requests that occupied their slots when it was queued.
void worker_loop(md_server* s) {
  (void)hipSetDevice(s->device);
  const int n_slots = (int)s->slots.size();
  // occupants of every slot when tick t & 1 was queued
  std::vector<std::shared_ptr<Request>> occ[2] = {std::vector<std::shared_ptr<Request>>(n_slots),
                                                  std::vector<std::shared_ptr<Request>>(n_slots)};
  long long t = 0;                 // next tick
  bool prev_inflight = false;      // tick t - 1 queued and not yet processed
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // admit queued requests into free slots while their buffers fit in the pool
    std::vector<int> uploads;
    bool any_init = false;
    for (int j = 0; j < n_slots && !s->queue.empty(); ++j) {
      if (s->slots[j]) continue;
      auto r = s->queue.front();
      size_t off;
      if (!s->pool->alloc(r->bytes, &off)) break;    // head of line waits for memory
      s->queue.pop_front();
      r->off = off;
      r->slot = j;
      r->state = kResident;
      r->t_start = now_s();
      s->slots[j] = r;
      s->resident_changed = true;
      s->h_table[j] = make_job(s, *r);
      uploads.push_back(j);
      any_init = true;
    }
    // requests canceled while resident: their entries are cleared before the next tick, their
    // slots and memory are freed once the tick in flight (the last one that may run them) is done
    for (int j = 0; j < n_slots; ++j) {
      auto& r = s->slots[j];
      if (r && r->cancel_requested && r->cancel_tick < 0) {
        JobDev empty{};
        empty.state = kJobEmpty;
        s->h_table[j] = empty;
        uploads.push_back(j);
        r->cancel_tick = t;
        s->resident_changed = true;
      }
    }
    bool any = false, any_running = false;
    for (int j = 0; j < n_slots; ++j) {
      const auto& r = s->slots[j];
      if (r && !r->cancel_requested) {
        any = true;
        if (std::find(uploads.begin(), uploads.end(), j) == uploads.end()) any_running = true;
      }
    }
    const bool cancels = std::any_of(s->slots.begin(), s->slots.end(),
                                     [](const std::shared_ptr<Request>& r) { return r && r->cancel_requested; });
    if (!any && !prev_inflight && !cancels) {
      if (s->stop) break;
      s->cv_work.wait(lk);
      continue;
    }
    const bool queue_now = any || cancels;
    std::vector<SchedJob> jobs;
    bool rebuild = false;
    if (queue_now) {
      for (int j = 0; j < n_slots; ++j) occ[t & 1][j] = (s->slots[j] && !s->slots[j]->cancel_requested) ? s->slots[j] : nullptr;
      if (s->resident_changed) {
        for (int j = 0; j < n_slots; ++j) {
          const auto& r = occ[t & 1][j];
          if (!r) continue;
          const md_dock_params& p = r->params;
          jobs.push_back(SchedJob{j, &r->lig->dev, p.n_runs, p.pop_size, n_local_search_of(&p), p.ls_iters,
                                  p.ls_method});
        }
        rebuild = true;
        s->resident_changed = false;
      }
    }
    lk.unlock();
    const double t0 = now_s();
    hipError_t e = hipSuccess;
    // (2) upload new and cleared entries, queue tick t.  The copies read their pinned source when
    // they run, so each tick parity has its own staging entries, rewritten only after that
    // parity's previous tick (and the uploads queued before it) is done.
    for (int j : uploads) {
      s->h_up[t & 1][j] = s->h_table[j];
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_table + j, s->h_up[t & 1] + j, sizeof(JobDev), hipMemcpyHostToDevice, s->stream);
    }
    const bool queued = queue_now && e == hipSuccess;
    if (queued) e = queue_tick(s, t, rebuild ? &jobs : nullptr, any_init, any_running);
    // (3) tick t - 1: wait, find the requests it finished, copy their results beside tick t
    std::vector<std::shared_ptr<Request>> finished;
    if (e == hipSuccess && prev_inflight) {
      const int pb = (int)((t - 1) & 1);
      e = hipEventSynchronize(s->tick_done[pb]);
      // (a request finished by tick t - 2 is still in tick t - 1's occupants, already retired;
      // only this thread changes the state of a request that reached a slot)
      if (e == hipSuccess)
        for (int j = 0; j < n_slots; ++j)
          if (occ[pb][j] && occ[pb][j]->state == kResident && s->h_tick[pb][j].state == kJobDone)
            finished.push_back(occ[pb][j]);
      for (auto& r : finished)
        if (e == hipSuccess) e = collect(s, *r, s->tick_done[pb]);
    }
    const double t1 = now_s();
    lk.lock();
    s->busy_s += t1 - t0;
    if (queued) ++s->ticks;
    if (e != hipSuccess) {
      s->fatal = std::string("device error in the serving loop: ") + hipGetErrorString(e);
      for (auto& r : s->slots)
        if (r) {
          r->state = kFailed;
          r->error = s->fatal;
          drop_hold(*r);
        }
      for (auto& r : s->queue) {
        r->state = kFailed;
        r->error = s->fatal;
        drop_hold(*r);
      }
      s->queue.clear();
      std::fill(s->slots.begin(), s->slots.end(), nullptr);
      s->cv_done.notify_all();
      break;
    }
    for (auto& r : finished) {
      r->t_end = t1;
      r->state = kFinished;   // a cancel that came after its last tick was queued is too late
      ++s->completed;
      drop_hold(*r);
      s->pool->release(r->off, r->bytes);
      s->slots[r->slot] = nullptr;
      s->resident_changed = true;
      s->h_table[r->slot].state = kJobEmpty;
    }
    // canceled requests whose entry was cleared before tick t - 1: no tick runs them any more
    bool dropped = false;
    if (prev_inflight)
      for (int j = 0; j < n_slots; ++j) {
        auto& r = s->slots[j];
        if (r && r->cancel_requested && r->cancel_tick >= 0 && r->cancel_tick <= t - 1) {
          s->pool->release(r->off, r->bytes);
          r->state = kCanceled;
          r->t_end = t1;
          drop_hold(*r);
          r = nullptr;
          s->resident_changed = true;
          dropped = true;
        }
      }
    if (prev_inflight) occ[(t - 1) & 1].assign(n_slots, nullptr);
    prev_inflight = queued;
    if (queued) ++t;
    if (!finished.empty() || dropped) s->cv_done.notify_all();
  }
  // a fatal error leaves the stream to md_server_destroy, which synchronises it
}

md_status fill_result(const Request& r, md_dock_result* out) {
  const int runs = r.params.n_runs, G = r.n_genes, N = r.n_atoms;
  if (out->n_runs < runs || out->n_genes < G || !out->best_energy || !out->best_genes)
    return server_fail(MD_EINVAL, "md_server: result buffers too small or null");
  if (out->best_xyz && out->n_atoms < N) return server_fail(MD_EINVAL, "md_server: best_xyz capacity too small");
  for (int k = 0; k < runs; ++k) {
    out->best_energy[k] = r.best_energy[k];
    std::memcpy(out->best_genes + (size_t)k * out->n_genes, &r.best_genes[(size_t)k * G], (size_t)G * 4);
    if (out->best_xyz)
      std::memcpy(out->best_xyz + (size_t)k * out->n_atoms * 3, &r.best_xyz[(size_t)k * N * 3], (size_t)N * 12);
    if (out->run_index) out->run_index[k] = r.run_index[k];
    if (out->evals) out->evals[k] = r.evals[k];
    if (out->generations) out->generations[k] = r.planned;
  }
  return MD_OK;
}

}  // namespace

extern "C" {

md_status md_server_create(const md_receptor* rec, const md_server_params* p, md_server** out) {
  if (!rec || !p || !out) return server_fail(MD_EINVAL, "md_server_create: null argument");
  if (p->max_slots < 1 || p->max_slots > 4096) return server_fail(MD_ERANGE, "md_server_create: max_slots must be in [1, 4096]");
  if (p->hbm_budget_bytes < (1u << 20)) return server_fail(MD_EINVAL, "md_server_create: hbm_budget_bytes must be >= 1 MiB");
  if (p->use_graphs != 0 && p->use_graphs != 1) return server_fail(MD_EINVAL, "md_server_create: use_graphs must be 0 or 1");
  auto* s = new (std::nothrow) md_server();
  if (!s) return server_fail(MD_ENOMEM, "md_server_create: out of host memory");
  s->rec = rec;
  s->params = *p;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->pool_base), p->hbm_budget_bytes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_table), sizeof(JobDev) * p->max_slots);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->h_table), sizeof(JobDev) * p->max_slots);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipHostMalloc(reinterpret_cast<void**>(&s->h_tick[k]), sizeof(JobDev) * p->max_slots);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipHostMalloc(reinterpret_cast<void**>(&s->h_up[k]), sizeof(JobDev) * p->max_slots);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->tick_done[k], hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    if (s->pool_base) (void)hipFree(s->pool_base);
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->h_table) (void)hipHostFree(s->h_table);
    for (int k = 0; k < 2; ++k) {
      if (s->h_tick[k]) (void)hipHostFree(s->h_tick[k]);
      if (s->h_up[k]) (void)hipHostFree(s->h_up[k]);
      if (s->tick_done[k]) (void)hipEventDestroy(s->tick_done[k]);
    }
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return e == hipErrorOutOfMemory ? server_fail(MD_ENOMEM, "md_server_create: out of device memory")
                                    : server_fail(MD_EDEVICE, std::string("md_server_create: ") + hipGetErrorString(e));
  }
  for (int j = 0; j < p->max_slots; ++j) {
    JobDev empty{};
    empty.state = kJobEmpty;
    s->h_table[j] = empty;
  }
  e = hipMemcpy(s->d_table, s->h_table, sizeof(JobDev) * p->max_slots, hipMemcpyHostToDevice);
  s->pool.reset(new Pool(p->hbm_budget_bytes));
  s->slots.assign(p->max_slots, nullptr);
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return e == hipSuccess ? MD_OK : server_fail(MD_EDEVICE, "md_server_create: table upload failed");
}

md_status md_server_submit(md_server* s, const md_ligand* lig, const md_dock_params* p, unsigned long long* ticket) {
  if (!s || !lig || !p || !ticket) return server_fail(MD_EINVAL, "md_server_submit: null argument");
  const std::string err = check_dock_params(p);
  if (!err.empty()) return server_fail(MD_EINVAL, "md_server_submit: " + err);
  auto r = std::make_shared<Request>();
  r->lig = lig;
  r->n_genes = lig->dev.n_genes;
  r->n_atoms = lig->dev.n_atoms;
  r->params = *p;
  r->planned = md_dock_planned_generations(p);
  layout(*r);
  if (r->bytes > s->params.hbm_budget_bytes)
    return server_fail(MD_ENOMEM, "md_server_submit: request needs more device memory than the server's budget");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) return server_fail(MD_EDEVICE, s->fatal);
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  lig->holds.fetch_add(1);
  r->held = true;
  s->requests[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return MD_OK;
}

md_status md_server_poll(md_server* s, unsigned long long ticket, md_dock_result* out, int* done) {
  if (!s || !done) return server_fail(MD_EINVAL, "md_server_poll: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return server_fail(MD_ENOTFOUND, "md_server_poll: unknown ticket");
  const Request& r = *it->second;
  *done = (r.state == kFinished || r.state == kCanceled || r.state == kFailed) ? 1 : 0;
  if (r.state == kCanceled) return server_fail(MD_ECANCELED, "md_server_poll: request was canceled");
  if (r.state == kFailed) return server_fail(MD_EDEVICE, r.error);
  if (r.state == kFinished && out) return fill_result(r, out);
  return MD_OK;
}

md_status md_server_wait(md_server* s, unsigned long long ticket, md_dock_result* out, double timeout_s) {
  if (!s) return server_fail(MD_EINVAL, "md_server_wait: null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return server_fail(MD_ENOTFOUND, "md_server_wait: unknown ticket");
  std::shared_ptr<Request> r = it->second;
  auto finished = [&] { return r->state == kFinished || r->state == kCanceled || r->state == kFailed; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, finished);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
    return server_fail(MD_EBUSY, "md_server_wait: timed out");
  }
  if (r->state == kCanceled) return server_fail(MD_ECANCELED, "md_server_wait: request was canceled");
  if (r->state == kFailed) return server_fail(MD_EDEVICE, r->error);
  return out ? fill_result(*r, out) : MD_OK;
}

md_status md_server_cancel(md_server* s, unsigned long long ticket) {
  if (!s) return server_fail(MD_EINVAL, "md_server_cancel: null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return server_fail(MD_ENOTFOUND, "md_server_cancel: unknown ticket");
  auto& r = it->second;
  if (r->state == kQueued) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
    r->state = kCanceled;
    drop_hold(*r);
  } else if (r->state == kResident) {
    r->cancel_requested = true;   // the worker clears its entry, then frees the slot
    s->cv_work.notify_one();
  }
  s->cv_done.notify_all();
  return MD_OK;
}

md_status md_server_request_times(md_server* s, unsigned long long ticket, double* submit_s, double* start_s,
                                  double* end_s) {
  if (!s) return server_fail(MD_EINVAL, "md_server_request_times: null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return server_fail(MD_ENOTFOUND, "md_server_request_times: unknown ticket");
  if (submit_s) *submit_s = it->second->t_submit;
  if (start_s) *start_s = it->second->t_start;
  if (end_s) *end_s = it->second->t_end;
  return MD_OK;
}

md_status md_server_release(md_server* s, unsigned long long ticket) {
  if (!s) return server_fail(MD_EINVAL, "md_server_release: null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return server_fail(MD_ENOTFOUND, "md_server_release: unknown ticket");
  const ReqState st = it->second->state;
  if (st == kQueued || st == kResident || it->second->held)
    return server_fail(MD_EBUSY, "md_server_release: request still queued or on the device");
  s->requests.erase(it);
  return MD_OK;
}

md_status md_server_get_stats(md_server* s, md_server_stats* out) {
  if (!s || !out) return server_fail(MD_EINVAL, "md_server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->ticks = s->ticks;
  out->completed = s->completed;
  out->queued = (int)s->queue.size();
  int resident = 0;
  for (auto& r : s->slots) resident += r ? 1 : 0;
  out->resident = resident;
  out->pool_used_bytes = s->pool->used();
  out->busy_seconds = s->busy_s;
  return MD_OK;
}

md_status md_server_destroy(md_server* s) {
  if (!s) return MD_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& r : s->queue) {   // queued work is dropped, resident work drains
      r->state = kCanceled;
      drop_hold(*r);
    }
    s->queue.clear();
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
  }
  // the device work is drained; drop the executable graph before the buffers and the stream it
  // was launched on
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->copy_stream);
  s->graph.reset();
  if (s->d_blocks) (void)hipFree(s->d_blocks);
  (void)hipFree(s->d_table);
  (void)hipHostFree(s->h_table);
  for (int k = 0; k < 2; ++k) {
    (void)hipHostFree(s->h_tick[k]);
    (void)hipHostFree(s->h_up[k]);
    (void)hipEventDestroy(s->tick_done[k]);
  }
  (void)hipFree(s->pool_base);
  (void)hipStreamDestroy(s->copy_stream);
  (void)hipStreamDestroy(s->stream);
  delete s;
  return MD_OK;
}

}  // extern "C"
