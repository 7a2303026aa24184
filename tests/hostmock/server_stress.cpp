// Concurrency stress of the docking server's host code through the public C API, built against
// the emulated runtime (mock_runtime.cpp) and run under ThreadSanitizer or AddressSanitizer by
// tests/test_server_host.py.  Several client threads submit, wait on, poll, cancel and release
// requests of ligands of several sizes while the worker thread admits, ticks and retires them
// (with the branch launch and with kernel-by-kernel ticks), another thread docks the same
// requests through md_dock and md_dock_batch, and servers are destroyed with work queued and
// resident.  Every finished request must match every other result of the same (ligand,
// parameters): the emulated kernels make a result depend on the request alone.
// Exit status 0 on success; the first failure is printed.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "mdock.h"

md_receptor* g_rec = nullptr;

namespace {

std::atomic<int> g_failures{0};
std::atomic<int> g_done{0}, g_canceled{0}, g_timeouts{0};
std::mutex g_print;

void fail(const std::string& msg) {
  std::lock_guard<std::mutex> lk(g_print);
  if (g_failures.fetch_add(1) < 5) std::fprintf(stderr, "FAIL: %s (last error: %s)\n", msg.c_str(), md_last_error());
}

#define CHECK(cond, msg)  \
  do {                    \
    if (!(cond)) fail(msg); \
  } while (0)

struct Lig {
  md_ligand* h = nullptr;
  int n_atoms = 0, n_genes = 0;
};

// A zig-zag chain of n atoms; every third inner bond is rotatable.
Lig make_ligand(int n) {
  std::vector<float> xyz(n * 3), q(n), tp(7 * 7);
  std::vector<int> type(n), bonds(2 * (n - 1)), tors;
  for (int i = 0; i < n; ++i) {
    xyz[3 * i] = 1.25f * i;
    xyz[3 * i + 1] = (i % 2) ? 0.8f : 0.f;
    xyz[3 * i + 2] = 0.3f * (float)(i % 3);
    type[i] = i % 7;
    q[i] = 0.05f * (float)((i % 5) - 2);
  }
  for (int i = 0; i + 1 < n; ++i) {
    bonds[2 * i] = i;
    bonds[2 * i + 1] = i + 1;
    if (i >= 1 && i + 1 <= n - 2 && i % 3 == 1 && (int)tors.size() < 32) tors.push_back(i);
  }
  for (int t = 0; t < 7; ++t) {
    const float row[7] = {3.6f + 0.1f * t, 0.15f, 20.f, -0.001f, 0.f, 0.f, 0.f};
    std::memcpy(&tp[7 * t], row, sizeof row);
  }
  md_ligand_desc d{};
  d.n_atoms = n;
  d.xyz = xyz.data();
  d.type = type.data();
  d.charge = q.data();
  d.n_bonds = n - 1;
  d.bonds = bonds.data();
  d.n_torsions = (int)tors.size();
  d.torsions = tors.data();
  d.root_atom = 0;
  d.n_types = 7;
  d.type_params = tp.data();
  Lig l;
  if (md_ligand_create(&d, &l.h) != MD_OK) {
    fail("md_ligand_create n=" + std::to_string(n));
    return l;
  }
  l.n_atoms = md_ligand_num_atoms(l.h);
  l.n_genes = md_ligand_num_genes(l.h);
  return l;
}

md_dock_params params_for(std::mt19937& rng, bool big) {
  md_dock_params p{};
  p.n_runs = big ? 8 : 1 + (int)(rng() % 4);
  p.pop_size = big ? 200 : 8 + (int)(rng() % 33);
  p.max_evals_per_run = 1ll << 40;
  p.max_generations = 1 + (int)(rng() % 6);
  p.ls_rate = (rng() % 3) ? 0.25f : 0.f;
  p.ls_iters = 1 + (int)(rng() % 12);
  p.rho = 0.8f;
  p.eps = 1e-6f;
  p.crossover_rate = 0.8f;
  p.mutation_rate = 0.02f;
  p.tournament_rate = 0.6f;
  p.elitism = 1;
  p.mut_trans = 2.f;
  p.mut_rot = 0.1f;
  p.mut_tors = 0.5f;
  p.seed = rng();
  p.ls_method = (rng() % 2) ? MD_LS_ADADELTA : MD_LS_SOLIS_WETS;
  return p;
}

struct Result {
  std::vector<float> e, g, x;
  std::vector<int> run, gens;
  std::vector<long long> evals;
  md_dock_result view(const Lig& l, int runs) {
    e.assign(runs, 0.f);
    g.assign((size_t)runs * l.n_genes, 0.f);
    x.assign((size_t)runs * l.n_atoms * 3, 0.f);
    run.assign(runs, -1);
    gens.assign(runs, -1);
    evals.assign(runs, -1);
    return md_dock_result{runs, l.n_genes, l.n_atoms, e.data(), g.data(), x.data(), run.data(), evals.data(), gens.data()};
  }
  bool operator==(const Result& o) const {
    return e == o.e && g == o.g && x == o.x && run == o.run && gens == o.gens && evals == o.evals;
  }
};

// first result seen per request; later results of the same request must be equal
std::mutex g_golden_mu;
std::map<int, Result> g_golden;

void check_result(int id, const md_dock_params& p, const Result& r, const char* who) {
  const int planned = md_dock_planned_generations(&p);
  for (int k = 0; k < p.n_runs; ++k) {
    CHECK(r.gens[k] == planned, std::string(who) + ": generations");
    CHECK(r.evals[k] > 0, std::string(who) + ": evaluations");
    if (k) CHECK(r.e[k - 1] <= r.e[k], std::string(who) + ": energies not sorted");
  }
  std::lock_guard<std::mutex> lk(g_golden_mu);
  auto it = g_golden.find(id);
  if (it == g_golden.end())
    g_golden.emplace(id, r);
  else
    CHECK(it->second == r, std::string(who) + ": result differs from another run of the same request");
}

// The requests the threads draw from: a small set, so that the same request runs many times,
// through the server with and without the branch launch, md_dock and md_dock_batch.
constexpr int kRequests = 24;
md_dock_params request(int id) {
  std::mt19937 rng(1234u + (unsigned)id);
  return params_for(rng, id % 8 == 0);
}
int lig_of(int id, const std::vector<Lig>& ligs) { return id % (int)ligs.size(); }

void client(md_server* srv, const std::vector<Lig>& ligs, unsigned seed, int n_req) {
  std::mt19937 rng(seed);
  for (int it = 0; it < n_req; ++it) {
    const int id = (int)(rng() % kRequests);
    const int li = lig_of(id, ligs);
    md_dock_params p = request(id);
    unsigned long long t = 0;
    if (md_server_submit(srv, ligs[li].h, &p, &t) != MD_OK) {
      fail("submit");
      continue;
    }
    const int action = (int)(rng() % 6);
    Result r;
    md_dock_result out = r.view(ligs[li], p.n_runs);
    md_status st = MD_OK;
    if (action == 0) {   // cancel at once: canceled, or already finished
      md_server_cancel(srv, t);
      st = md_server_wait(srv, t, &out, 30.0);
      CHECK(st == MD_OK || st == MD_ECANCELED, "wait after cancel");
    } else if (action == 1) {   // poll until done
      int done = 0;
      for (int k = 0; k < 200000 && !done; ++k) {
        st = md_server_poll(srv, t, &out, &done);
        if (st != MD_OK) break;
        if (!done) std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
      CHECK(st == MD_OK && done, "poll");
    } else if (action == 2) {   // cancel after a while
      std::this_thread::sleep_for(std::chrono::microseconds(200 + rng() % 2000));
      md_server_cancel(srv, t);
      st = md_server_wait(srv, t, &out, 30.0);
      CHECK(st == MD_OK || st == MD_ECANCELED, "wait after late cancel");
    } else if (action == 3) {   // a short wait that may time out, then a full one
      st = md_server_wait(srv, t, &out, 1e-4);
      if (st == MD_EBUSY) {
        ++g_timeouts;
        st = md_server_wait(srv, t, &out, 30.0);
      }
      CHECK(st == MD_OK, "wait after timeout");
    } else {
      st = md_server_wait(srv, t, &out, 30.0);
      CHECK(st == MD_OK, "wait");
    }
    if (st == MD_OK) check_result(id, p, r, "server");
    ++(st == MD_OK ? g_done : g_canceled);
    md_server_stats stats{};
    CHECK(md_server_get_stats(srv, &stats) == MD_OK, "stats");
    double a, b, c;
    CHECK(md_server_request_times(srv, t, &a, &b, &c) == MD_OK, "times");
    CHECK(md_server_release(srv, t) == MD_OK, "release");
  }
}

// docks requests through md_dock / md_dock_batch on this thread while the server runs
void direct(const std::vector<Lig>& ligs, unsigned seed, int n) {
  std::mt19937 rng(seed);
  for (int it = 0; it < n; ++it) {
    const int id = (int)(rng() % kRequests);
    const int li = lig_of(id, ligs);
    md_dock_params p = request(id);
    Result r;
    md_dock_result out = r.view(ligs[li], p.n_runs);
    if (it % 2) {
      md_dock_job job{ligs[li].h, p, &out};
      CHECK(md_dock_batch(g_rec, 1, &job, nullptr) == MD_OK, "md_dock_batch");
    } else {
      CHECK(md_dock(g_rec, ligs[li].h, &p, &out, nullptr) == MD_OK, "md_dock");
    }
    check_result(id, p, r, "md_dock");
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? std::atoi(argv[1]) : 1;
  const int n = 16;
  std::vector<float> maps((size_t)9 * n * n * n);
  for (size_t i = 0; i < maps.size(); ++i) maps[i] = 0.01f * (float)(i % 97) - 0.3f;
  md_grid_desc gd{n, n, n, 0.375f, {-3.f, -3.f, -3.f}, 7};
  if (md_receptor_create(&gd, maps.data(), MD_MAP_FP32, nullptr, &g_rec) != MD_OK) {
    std::fprintf(stderr, "FAIL: md_receptor_create: %s\n", md_last_error());
    return 1;
  }
  std::vector<Lig> ligs;
  for (int na : {6, 20, 40, 70, 100, 128}) ligs.push_back(make_ligand(na));
  if (g_failures) return 1;

  for (int round = 0; round < rounds; ++round) {
    for (int graphs : {1, 0}) {
      md_server_params sp{};
      sp.hbm_budget_bytes = 1u << 20;
      sp.max_slots = 3;
      sp.use_graphs = graphs;
      md_server* srv = nullptr;
      if (md_server_create(g_rec, &sp, &srv) != MD_OK) {
        fail("md_server_create");
        break;
      }
      std::vector<std::thread> th;
      for (int c = 0; c < 4; ++c) th.emplace_back(client, srv, std::cref(ligs), 1000u * round + 10u * graphs + c, 24);
      th.emplace_back(direct, std::cref(ligs), 77u + round + graphs, 8);
      for (auto& t : th) t.join();
      // requests still queued and resident when the server goes away
      for (int k = 0; k < 10; ++k) {
        md_dock_params p = request(k);
        unsigned long long t = 0;
        CHECK(md_server_submit(srv, ligs[lig_of(k, ligs)].h, &p, &t) == MD_OK, "late submit");
      }
      CHECK(md_server_destroy(srv) == MD_OK, "destroy with work pending");
    }
  }
  // a queued or resident request holds its ligand: the ligand can be neither destroyed nor
  // re-planned and the request not released until it has left the device; a canceled resident
  // request is reported canceled only once its slot is free, and then everything goes
  {
    md_server_params sp{};
    sp.hbm_budget_bytes = 1u << 20;
    sp.max_slots = 1;
    sp.use_graphs = 1;
    md_server* srv = nullptr;
    CHECK(md_server_create(g_rec, &sp, &srv) == MD_OK, "create");
    Lig own = make_ligand(30);
    std::mt19937 rng(11);
    md_dock_params p = params_for(rng, false);
    p.max_generations = 1 << 20;
    unsigned long long t1 = 0, t2 = 0;
    CHECK(md_server_submit(srv, own.h, &p, &t1) == MD_OK, "submit long");
    CHECK(md_server_submit(srv, own.h, &p, &t2) == MD_OK, "submit queued");
    CHECK(md_ligand_destroy(own.h) == MD_EBUSY, "destroy of a held ligand refused");
    md_plan plan{65536, 3, 4, 0, 0, 0, 1};
    CHECK(md_ligand_set_plan(own.h, &plan) == MD_EBUSY, "re-plan of a held ligand refused");
    CHECK(md_server_release(srv, t1) == MD_EBUSY, "release of a running request refused");
    md_server_stats st{};
    for (int k = 0; k < 100000 && st.resident == 0; ++k) {   // wait until t1 is on the device
      CHECK(md_server_get_stats(srv, &st) == MD_OK, "stats");
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    CHECK(md_server_cancel(srv, t2) == MD_OK && md_server_release(srv, t2) == MD_OK, "queued cancel frees at once");
    CHECK(md_server_cancel(srv, t1) == MD_OK, "cancel resident");
    CHECK(md_server_wait(srv, t1, nullptr, 30.0) == MD_ECANCELED, "wait sees the cancel");
    CHECK(md_server_get_stats(srv, &st) == MD_OK && st.resident == 0 && st.pool_used_bytes == 0, "slot freed");
    CHECK(md_server_release(srv, t1) == MD_OK, "release after the slot is free");
    CHECK(md_ligand_destroy(own.h) == MD_OK, "destroy once no request holds the ligand");
    md_server_destroy(srv);
  }
  // a request larger than the pool is refused at submit
  {
    md_server_params sp{};
    sp.hbm_budget_bytes = 1u << 20;
    sp.max_slots = 2;
    sp.use_graphs = 1;
    md_server* srv = nullptr;
    CHECK(md_server_create(g_rec, &sp, &srv) == MD_OK, "create");
    std::mt19937 rng(9);
    md_dock_params p = params_for(rng, true);
    p.n_runs = 64;
    p.pop_size = 1000;
    unsigned long long t = 0;
    CHECK(md_server_submit(srv, ligs[5].h, &p, &t) == MD_ENOMEM, "oversized request refused");
    md_server_destroy(srv);
  }
  for (auto& l : ligs) md_ligand_destroy(l.h);
  md_receptor_destroy(g_rec);
  std::printf("server stress: %d rounds, %zu distinct requests; server requests: %d finished, %d canceled, %d waits timed out; %d failures\n",
              rounds, g_golden.size(), g_done.load(), g_canceled.load(), g_timeouts.load(), g_failures.load());
  return g_failures ? 1 : 0;
}
