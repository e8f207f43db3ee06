// Drives the library's real host code against the stand-in runtime
// (hip_standin.cpp): plain geometries built and applied from the main thread,
// then a served-mode run with graph replay, in which sixteen client threads
// open forty small sessions on eight lanes and wait for their applies, as the
// concurrent-clients GPU test does, and the same with batching lanes (two
// lanes, so that sessions of one kind share a lane and run together).  Kernels do not run, so the values are
// not checked; the run checks statuses, and the sanitizer and the stand-in
// check memory lifetimes and the serialisation of graph calls.
//
// Exit status 0 iff every call succeeded and the stand-in saw no violation.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "sbie.h"

extern "C" void standin_report(FILE* f);
extern "C" long standin_violations(void);

namespace {

std::atomic<int> g_failures{0};

void check(sbie_status st, const char* what) {
  if (st != SBIE_OK) {
    std::fprintf(stderr, "%s failed: %s (%s)\n", what, sbie_status_str(st), sbie_last_error());
    g_failures.fetch_add(1);
  }
}

// m spheroids on a line, 4 apart (far from each other), alternately prolate
// and oblate, with seeded unit quaternions.
struct Particles {
  std::vector<double> c, q, A, C;
};

Particles line_of(int m, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd;
  Particles P;
  for (int i = 0; i < m; ++i) {
    P.c.insert(P.c.end(), {4.0 * i, 0.3 * (i % 2), 0.0});
    double q[4], n = 0;
    for (double& x : q) {
      x = nd(rng);
      n += x * x;
    }
    n = std::sqrt(n);
    for (double x : q) P.q.push_back(x / n);
    P.A.push_back(i % 2 ? 1.0 : 0.5);
    P.C.push_back(i % 2 ? 0.6 : 1.0);
  }
  return P;
}

void plain_path() {
  sbie_ctx* ctx = nullptr;
  check(sbie_ctx_create(0, &ctx), "sbie_ctx_create");
  if (!ctx) return;
  const int p = 6;  // T = 98 >= 32: the pair-symmetric far path and its records
  for (int m : {1, 2, 3, 5}) {
    Particles P = line_of(m, 11 + m);
    sbie_geom* g = nullptr;
    check(sbie_geom_create(ctx, P.c.data(), P.q.data(), P.A.data(), P.C.data(), m, p, 1.0, &g), "sbie_geom_create");
    if (!g) continue;
    const int64_t N = sbie_geom_num_nodes(g);
    std::vector<double> dens(3 * N, 1.0), out(4 * N, 0.0);
    for (sbie_op op : {SBIE_OP_S, SBIE_OP_D}) {
      for (sbie_precision pr : {SBIE_FP64, SBIE_MIXED})
        check(sbie_apply(g, op, pr, 1, dens.data(), out.data(), nullptr, SBIE_TIMING), "sbie_apply");
    }
    check(sbie_apply(g, SBIE_OP_STOKES_S, SBIE_FP64, 3, dens.data(), out.data(), nullptr, 0), "sbie_apply stokes");
    check(sbie_apply(g, SBIE_OP_STOKES_D, SBIE_MIXED, 3, dens.data(), out.data(), nullptr, 0), "sbie_apply stresslet");
    // three densities in one S and one D apply (the shared far-field path)
    check(sbie_apply(g, SBIE_OP_S, SBIE_MIXED, 3, dens.data(), out.data(), nullptr, 0), "sbie_apply nrhs 3");
    check(sbie_apply(g, SBIE_OP_D, SBIE_FP64, 2, dens.data(), out.data(), nullptr, 0), "sbie_apply nrhs 2");
    std::vector<double> xyz(3 * N), nrm(3 * N), w(N);
    check(sbie_geom_nodes(g, xyz.data(), nrm.data(), w.data()), "sbie_geom_nodes");
    // targets: the allocating call with host pointers, the allocation-free one
    // with "device" pointers (host memory under the stand-in), twice
    std::vector<double> pts = {0.0, 0.0, 9.0, 2.0, -8.0, 1.0, 30.0, 0.5, 0.5}, val(3), grad(9);
    check(sbie_eval_targets(g, SBIE_OP_S, SBIE_FP64, dens.data(), 3, pts.data(), val.data(), grad.data(), nullptr, 0),
          "sbie_eval_targets");
    for (int64_t n : {3, 2})
      check(sbie_eval_targets_noalloc(g, SBIE_OP_D, SBIE_MIXED, dens.data(), n, pts.data(), val.data(), grad.data(),
                                      nullptr, SBIE_DEVICE_PTRS),
            "sbie_eval_targets_noalloc");
    sbie_geom_destroy(g);
  }
  sbie_ctx_destroy(ctx);
}

void served_path(int lanes, uint32_t flags) {
  sbie_ctx* ctx = nullptr;
  check(sbie_ctx_create(0, &ctx), "sbie_ctx_create");
  if (!ctx) return;
  sbie_server* srv = nullptr;
  check(sbie_server_create(ctx, lanes, 256ull << 20, flags, &srv), "sbie_server_create");
  if (!srv) return;
  const int nsess = 40, nclients = 16, napply = 5;
  auto client = [&](int t) {
    for (int k = t; k < nsess; k += nclients) {
      const int m = 2 + k % 3;
      const int p = k % 4 == 3 ? 6 : 4;
      const sbie_op op = k % 7 == 5 ? SBIE_OP_STOKES_S : (k % 2 ? SBIE_OP_D : SBIE_OP_S);
      const sbie_precision pr = k % 3 == 2 ? SBIE_MIXED : SBIE_FP64;
      Particles P = line_of(m, 200 + k);
      sbie_session* s = nullptr;
      check(sbie_session_open(srv, P.c.data(), P.q.data(), P.A.data(), P.C.data(), m, p, 1.0, op, pr, &s),
            "sbie_session_open");
      if (!s) continue;
      const int64_t n = (int64_t)(op == SBIE_OP_STOKES_S ? 3 : 1) * m * (p + 1) * (2 * p + 2);
      for (int r = 0; r < napply; ++r) {
        // fresh host buffers per apply, released as soon as the wait returns
        std::vector<double> dens(n, 1.0 + r), out(n, 0.0);
        uint64_t ticket = 0;
        check(sbie_session_apply(s, dens.data(), out.data(), 0, &ticket), "sbie_session_apply");
        sbie_apply_stats st;
        check(sbie_wait(srv, ticket, -1, &st), "sbie_wait");
      }
      check(sbie_session_close(s), "sbie_session_close");
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nclients; ++t) th.emplace_back(client, t);
  for (auto& x : th) x.join();
  sbie_server_info info;
  check(sbie_server_get_info(srv, &info), "sbie_server_get_info");
  std::printf("served: admitted %lld, applies %lld, lanes %d, graphs %d%s\n", (long long)info.admitted,
              (long long)info.applies, info.lanes, info.graphs, info.batched > 0 ? ", batched" : "");
  if (info.applies != (int64_t)nsess * napply) g_failures.fetch_add(1);
  sbie_server_destroy(srv);
  sbie_ctx_destroy(ctx);
}

// Served sessions with the tree far field (two of 64 particles, S and D, and
// one of 3 that keeps the direct field) on three lanes (one per session: the
// sessions stay open across all their applies) with graph replay.
void served_tree_path() {
  sbie_ctx* ctx = nullptr;
  check(sbie_ctx_create(0, &ctx), "sbie_ctx_create");
  if (!ctx) return;
  sbie_server* srv = nullptr;
  check(sbie_server_create(ctx, 3, 512ull << 20, SBIE_SERVER_GRAPHS | SBIE_SERVER_TREE, &srv), "sbie_server_create");
  if (!srv) return;
  const int p = 4;
  std::vector<sbie_session*> ss;
  std::vector<int64_t> ns;
  for (int k = 0; k < 3; ++k) {
    const int m = k < 2 ? 64 : 3;
    Particles P = line_of(m, 900 + k);
    sbie_session* s = nullptr;
    check(sbie_session_open(srv, P.c.data(), P.q.data(), P.A.data(), P.C.data(), m, p, 1.0,
                            k == 1 ? SBIE_OP_D : SBIE_OP_S, k == 0 ? SBIE_MIXED : SBIE_FP64, &s),
          "sbie_session_open tree");
    ss.push_back(s);
    ns.push_back((int64_t)m * (p + 1) * (2 * p + 2));
  }
  for (int r = 0; r < 2; ++r)
    for (size_t k = 0; k < ss.size(); ++k) {
      if (!ss[k]) continue;
      std::vector<double> dens(ns[k], 1.0 + r), out(ns[k], 0.0);
      uint64_t ticket = 0;
      check(sbie_session_apply(ss[k], dens.data(), out.data(), 0, &ticket), "sbie_session_apply tree");
      check(sbie_wait(srv, ticket, -1, nullptr), "sbie_wait tree");
    }
  for (sbie_session* s : ss)
    if (s) check(sbie_session_close(s), "sbie_session_close tree");
  sbie_server_info info;
  check(sbie_server_get_info(srv, &info), "sbie_server_get_info");
  std::printf("served tree: applies %lld, tree sessions %lld\n", (long long)info.applies,
              (long long)info.tree_sessions);
  if (info.applies != 6 || info.tree_sessions != 2) g_failures.fetch_add(1);
  sbie_server_destroy(srv);
  sbie_ctx_destroy(ctx);
}

}  // namespace

int main() {
  plain_path();
  served_path(8, SBIE_SERVER_GRAPHS);
  served_path(2, SBIE_SERVER_GRAPHS | SBIE_SERVER_BATCH);
  served_tree_path();
  standin_report(stdout);
  const long v = standin_violations();
  std::printf("failures %d violations %ld\n", g_failures.load(), v);
  return (g_failures.load() == 0 && v == 0) ? 0 : 1;
}
