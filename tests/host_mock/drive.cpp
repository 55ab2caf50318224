// Scenarios for the host runtime under AddressSanitizer (see mock_runtime.cpp).
// Usage: drive <scenario>; prints "ok <scenario>" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/sr.h"

extern "C" size_t sr_mock_live_allocations();
extern "C" size_t sr_mock_malloc_calls();

#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c, \
                   sr_last_error(nullptr));                                   \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

static sr_params params(int L, double window, double horizon, uint64_t seed) {
  sr_params p;
  std::memset(&p, 0, sizeof(p));
  p.Lx = p.Ly = L;
  p.J = 1.0; p.h = 0.1; p.T = 2.0;
  p.window = window; p.horizon = horizon; p.seed = seed;
  p.log_mode = SR_LOG_DIGEST;
  return p;
}

// A tuned window shrinks when windows need many iterations: more windows are
// committed than the first window length predicts, and iters_out is bounded
// by n_windows only.
static void tuned() {
  sr_params p = params(128, 0.0, 3.0, 1);
  sr_sim* s = nullptr;
  CHECK(sr_create(&p, nullptr, &s) == SR_OK);
  sr_obs o;
  CHECK(sr_observables(s, &o) == SR_OK);
  const long long predicted = (o.horizon_ticks + o.window_ticks - 1) / o.window_ticks;
  int32_t g[4], done = 0;
  CHECK(sr_run_window(s, -1, g, &done) == SR_EINVAL);    // unbounded count
  long long total = 0;
  for (;;) {
    int rc = sr_run_window(s, 4, g, &done);
    if (rc == SR_EDONE) break;
    CHECK(rc == SR_OK && done >= 1 && done <= 4);
    for (int i = 0; i < done; ++i) CHECK(g[i] == std::atoi(std::getenv("SR_MOCK_G")));
    total += done;
  }
  CHECK(sr_observables(s, &o) == SR_OK);
  CHECK(o.tick == o.horizon_ticks && o.windows == total);
  CHECK(o.subdomain_runs == o.iterations * o.n_sub);   // every subdomain, every iteration
  CHECK(total > predicted);
  CHECK(sr_run_window(s, -1, nullptr, &done) == SR_OK && done == 0);
  sr_destroy(s);
  std::printf("windows %lld, first-window estimate %lld\n", total, predicted);
}

// Requests arrive between rounds, are admitted by footprint and retired;
// afterwards plain simulations are created, run and destroyed again.
static void server() {
  sr_server* v = nullptr;
  CHECK(sr_server_create((size_t)64 << 20, 3, nullptr, &v) == SR_OK);
  std::vector<uint64_t> ids;
  int32_t open = 0;
  for (int i = 0; i < 10; ++i) {
    sr_params p = params(64 + 16 * (i % 9), 0.0, 0.5 + 0.3 * i, 7000 + i);
    uint64_t id = 0;
    CHECK(sr_server_submit(v, &p, &id) == SR_OK);
    ids.push_back(id);
    CHECK(sr_server_pump(v, &open) == SR_OK);
  }
  sr_params big = params(4096, 0.0, 5.0, 1);
  uint64_t id = 0;
  CHECK(sr_server_submit(v, &big, &id) == SR_ENOMEM);
  for (int r = 0; open && r < 10000; ++r) CHECK(sr_server_pump(v, &open) == SR_OK);
  CHECK(open == 0);
  sr_result res[16];
  int32_t n = 0;
  CHECK(sr_server_poll(v, res, 16, &n) == SR_OK && n == 10);
  for (int i = 0; i < n; ++i) CHECK(res[i].status == SR_OK && res[i].t_done >= res[i].t_start);
  sr_server_info info;
  CHECK(sr_server_stats(v, &info) == SR_OK);
  CHECK(info.completed == 10 && info.failed == 0 && info.bytes_in_use == 0);
  CHECK(info.peak_bytes <= (int64_t)(64 << 20));
  sr_server_destroy(v);
  for (int i = 0; i < 10; ++i) {
    sr_params p = params(64 + 16 * (i % 9), 0.0, 0.5 + 0.3 * i, 7000 + i);
    sr_sim* s = nullptr;
    CHECK(sr_create(&p, nullptr, &s) == SR_OK);
    int32_t done = 0;
    CHECK(sr_run_window(s, -1, nullptr, &done) == SR_OK && done > 0);
    sr_destroy(s);
  }
}

// Launches that give up (SR_MOCK_GIVE_UP = how many, on lattice 0): up to
// three in a row, the lattice continues from its last committed window in
// the next launch and every request completes; a fourth makes the pump
// return SR_EDEVICE with the reason as the calling thread's last error, and
// the server stays usable.
static void server_give_up() {
  const int gu = std::atoi(std::getenv("SR_MOCK_GIVE_UP"));
  sr_server* v = nullptr;
  CHECK(sr_server_create((size_t)64 << 20, 3, nullptr, &v) == SR_OK);
  for (int i = 0; i < 3; ++i) {
    sr_params p = params(64, 0.0, 2.0, 7100 + i);
    uint64_t id = 0;
    CHECK(sr_server_submit(v, &p, &id) == SR_OK);
  }
  int32_t open = 1;
  int rc = SR_OK;
  for (int r = 0; r < 10000 && open && rc == SR_OK; ++r) rc = sr_server_pump(v, &open);
  sr_result res[4];
  int32_t n = 0;
  sr_server_info info;
  CHECK(sr_server_stats(v, &info) == SR_OK);
  if (gu <= 3) {
    CHECK(rc == SR_OK && open == 0);
    CHECK(sr_server_poll(v, res, 4, &n) == SR_OK && n == 3);
    for (int i = 0; i < n; ++i) CHECK(res[i].status == SR_OK);
    CHECK(info.restarts == gu && info.failed == 0 && info.completed == 3);
  } else {
    CHECK(rc == SR_EDEVICE);
    const char* why = sr_last_error(nullptr);
    std::printf("reason: %s\n", why);
    CHECK(std::strstr(why, "server launch") && std::strstr(why, "gave up waiting"));
    CHECK(sr_server_poll(v, res, 4, &n) == SR_OK && n >= 1);
    int bad = 0;
    for (int i = 0; i < n; ++i) bad += res[i].status == SR_EDEVICE;
    CHECK(bad >= 1 && info.restarts == 3 && info.failed >= 1);
  }
  CHECK(info.bytes_in_use == 0 || open > 0);
  sr_server_destroy(v);
}

// The same for sr_batch_run: lattices a launch gave up on run again until
// their horizon; after three launches in a row it reports SR_EDEVICE.
static void batch_give_up() {
  const int gu = std::atoi(std::getenv("SR_MOCK_GIVE_UP"));
  std::vector<sr_sim*> sims;
  for (int i = 0; i < 3; ++i) {
    sr_params p = params(32 + 16 * i, 0.5, 2.0 + i, 400 + i);
    sr_sim* s = nullptr;
    CHECK(sr_create(&p, nullptr, &s) == SR_OK);
    sims.push_back(s);
  }
  sr_obs o;
  if (gu <= 3) {
    CHECK(sr_batch_step(sims.data(), 3, 2, nullptr) == SR_OK);
    for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.windows >= 1 && o.windows <= 2);
    CHECK(sr_batch_run(sims.data(), 3, nullptr) == SR_OK);
    for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
  } else {
    CHECK(sr_batch_run(sims.data(), 3, nullptr) == SR_EDEVICE);
    std::printf("reason: %s\n", sr_last_error(sims[0]));
    CHECK(std::strstr(sr_last_error(sims[0]), "gave up waiting"));
  }
  for (sr_sim* s : sims) sr_destroy(s);
}

// Batched runs from four threads at once, each on its own simulations and
// stream, with some launches giving up (SR_MOCK_GIVE_UP): every simulation
// reaches its horizon.
static void batch_threads() {
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) {
    th.emplace_back([t]() {
      std::vector<sr_sim*> sims;
      for (int i = 0; i < 2; ++i) {
        sr_params p = params(32 + 16 * i, 0.5, 2.0 + t, 500 + 10 * t + i);
        sr_sim* s = nullptr;
        CHECK(sr_create(&p, nullptr, &s) == SR_OK);
        sims.push_back(s);
      }
      CHECK(sr_batch_step(sims.data(), 2, 2, nullptr) == SR_OK);
      CHECK(sr_batch_run(sims.data(), 2, nullptr) == SR_OK);
      sr_obs o;
      for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
      for (sr_sim* s : sims) sr_destroy(s);
    });
  }
  for (auto& x : th) x.join();
}

// Budgeted batch steps, resumption, and the overflow fallback to the plain
// path (buffers grown, the window re-run from its committed state).
static void batch() {
  std::vector<sr_sim*> sims;
  const char* ovf = std::getenv("SR_MOCK_OVERFLOW");
  for (int i = 0; i < 5; ++i) {
    sr_params p = params(32 + 16 * i, i % 2 ? 0.0 : 0.5, 2.0 + i, 100 + i);
    // lattice 0 already at the largest list capacity: an overflow of its
    // window log alone must grow the log, not fail on the lists
    if (i == 0 && ovf && std::atoi(ovf) == 2) p.hist_cap = 1024;
    sr_sim* s = nullptr;
    CHECK(sr_create(&p, nullptr, &s) == SR_OK);
    sims.push_back(s);
  }
  CHECK(sr_batch_step(sims.data(), 5, 2, nullptr) == SR_OK);
  sr_obs o;
  for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.windows <= 2 && o.windows >= 1);
  CHECK(sr_batch_run(sims.data(), 5, nullptr) == SR_OK);
  for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
  for (sr_sim* s : sims) CHECK(sr_reset(s) == SR_OK);
  CHECK(sr_batch_run(sims.data(), 5, nullptr) == SR_OK);
  for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
  for (sr_sim* s : sims) sr_destroy(s);
}

// The no-allocation batch step: no device allocation or free inside the call,
// two calls in a row (the second on fewer lattices) reuse the one array, an
// overflow is reported instead of regrown, too many lattices are refused.
static void static_step() {
  std::vector<sr_sim*> sims;
  for (int i = 0; i < 5; ++i) {
    sr_params p = params(32 + 16 * i, i % 2 ? 0.0 : 0.5, 2.0 + i, 300 + i);
    sr_sim* s = nullptr;
    CHECK(sr_create(&p, nullptr, &s) == SR_OK);
    sims.push_back(s);
  }
  const char* ovf = std::getenv("SR_MOCK_OVERFLOW");
  const size_t calls = sr_mock_malloc_calls();
  const size_t live = sr_mock_live_allocations();
  if (ovf && std::atoi(ovf)) {
    CHECK(sr_batch_step_static(sims.data(), 5, 2, nullptr) == SR_EOVERFLOW);
    CHECK(sr_mock_malloc_calls() == calls && sr_mock_live_allocations() == live);
    for (sr_sim* s : sims) sr_destroy(s);
    return;
  }
  CHECK(sr_batch_step_static(sims.data(), 5, 2, nullptr) == SR_OK);
  CHECK(sr_batch_step_static(sims.data() + 3, 2, -1, nullptr) == SR_OK);
  CHECK(sr_mock_malloc_calls() == calls && sr_mock_live_allocations() == live);
  sr_obs o;
  for (int i = 0; i < 5; ++i) {
    CHECK(sr_observables(sims[i], &o) == SR_OK);
    if (i < 3) CHECK(o.windows >= 1 && o.windows <= 2);
    else CHECK(o.tick == o.horizon_ticks);
  }
  CHECK(sr_batch_step_static(sims.data(), 5, -1, nullptr) == SR_OK);
  for (sr_sim* s : sims) CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
  for (sr_sim* s : sims) sr_destroy(s);
  // more lattices than the array's record space: refused before device work
  std::vector<sr_sim*> many;
  for (int i = 0; i < 1025; ++i) {
    sr_params p = params(8, 0.5, 1.0, 900 + i);
    p.bx = p.by = 4;
    sr_sim* s = nullptr;
    CHECK(sr_create(&p, nullptr, &s) == SR_OK);
    many.push_back(s);
  }
  CHECK(sr_batch_step_static(many.data(), 1025, -1, nullptr) == SR_EINVAL);
  CHECK(sr_batch_step_static(many.data(), 1024, -1, nullptr) == SR_OK);
  for (sr_sim* s : many) sr_destroy(s);
}

// Save / load round trip and argument errors.
static void errors() {
  sr_params p = params(64, 0.5, 2.0, 5);
  sr_sim* s = nullptr;
  CHECK(sr_create(&p, nullptr, &s) == SR_OK);
  CHECK(sr_run_window(s, 2, nullptr, nullptr) == SR_OK);
  size_t n = 0;
  CHECK(sr_save(s, nullptr, 0, &n) == SR_OK && n > 0);
  std::vector<char> blob(n);
  CHECK(sr_save(s, blob.data(), n, &n) == SR_OK);
  CHECK(sr_save(s, blob.data(), n - 1, &n) == SR_EINVAL);
  sr_sim* t = nullptr;
  CHECK(sr_load(blob.data(), blob.size(), nullptr, &t) == SR_OK);
  CHECK(sr_load(blob.data(), 16, nullptr, &t) == SR_EINVAL);
  sr_obs a, b;
  CHECK(sr_observables(s, &a) == SR_OK && sr_observables(t, &b) == SR_OK);
  CHECK(a.tick == b.tick && a.windows == b.windows && a.M == b.M);
  sr_destroy(t);
  // a user start survives a checkpoint: the loaded copy can be reset
  {
    sr_params u = params(32, 0.5, 2.0, 9);
    std::vector<int8_t> sp(32 * 32);
    for (size_t i = 0; i < sp.size(); ++i) sp[i] = (i * 7 % 3) ? 1 : -1;
    u.init = SR_INIT_USER;
    u.init_spins = sp.data();
    sr_sim* a = nullptr;
    CHECK(sr_create(&u, nullptr, &a) == SR_OK);
    CHECK(sr_run_window(a, 2, nullptr, nullptr) == SR_OK);
    size_t m = 0;
    CHECK(sr_save(a, nullptr, 0, &m) == SR_OK);
    std::vector<char> ub(m);
    CHECK(sr_save(a, ub.data(), m, &m) == SR_OK);
    sr_sim* c = nullptr;
    CHECK(sr_load(ub.data(), ub.size(), nullptr, &c) == SR_OK);
    CHECK(sr_reset(c) == SR_OK && sr_reset(a) == SR_OK);
    sr_obs oa, oc;
    CHECK(sr_observables(a, &oa) == SR_OK && sr_observables(c, &oc) == SR_OK);
    CHECK(oa.tick == 0 && oc.tick == 0 && oa.M == oc.M);
    sr_destroy(a);
    sr_destroy(c);
  }
  // a tuned step size survives a checkpoint
  {
    sr_params q = params(64, 0.0, 3.0, 11);
    sr_sim* a = nullptr;
    CHECK(sr_create(&q, nullptr, &a) == SR_OK);
    sr_obs o0, oa, oc;
    CHECK(sr_observables(a, &o0) == SR_OK);
    CHECK(sr_run_window(a, 3, nullptr, nullptr) == SR_OK);
    CHECK(sr_observables(a, &oa) == SR_OK && oa.window_ticks != o0.window_ticks);
    size_t m = 0;
    CHECK(sr_save(a, nullptr, 0, &m) == SR_OK);
    std::vector<char> qb(m);
    CHECK(sr_save(a, qb.data(), m, &m) == SR_OK);
    sr_sim* c = nullptr;
    CHECK(sr_load(qb.data(), qb.size(), nullptr, &c) == SR_OK);
    CHECK(sr_observables(c, &oc) == SR_OK);
    CHECK(oc.window_ticks == oa.window_ticks && oc.tick == oa.tick && oc.windows == oa.windows);
    int32_t da = 0, dc = 0;
    CHECK(sr_run_window(a, -1, nullptr, &da) == SR_OK && sr_run_window(c, -1, nullptr, &dc) == SR_OK);
    CHECK(da == dc);
    sr_destroy(a);
    sr_destroy(c);
  }
  sr_params bad = p;
  bad.bx = 3; bad.by = 3;
  CHECK(sr_create(&bad, nullptr, &t) == SR_EINVAL);
  bad = p;
  bad.T = 0.0;
  CHECK(sr_create(&bad, nullptr, &t) == SR_EINVAL);
  sr_batch_run(&s, 1, nullptr);
  sr_destroy(s);
}

// Several threads each drive their own simulations (create, run, observe,
// fail a creation on purpose, destroy) at the same time.
static void threads() {
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) {
    th.emplace_back([t]() {
      for (int i = 0; i < 3; ++i) {
        sr_params p = params(32 + 16 * ((t + i) % 4), i % 2 ? 0.0 : 0.5, 1.0 + 0.5 * i, 100 * t + i);
        sr_sim* s = nullptr;
        CHECK(sr_create(&p, nullptr, &s) == SR_OK);
        int32_t done = 0;
        CHECK(sr_run_window(s, -1, nullptr, &done) == SR_OK && done > 0);
        sr_obs o;
        CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
        sr_params bad = p;
        bad.T = -1.0;
        sr_sim* b = nullptr;
        CHECK(sr_create(&bad, nullptr, &b) == SR_EINVAL && std::strstr(sr_last_error(nullptr), "T > 0"));
        sr_destroy(s);
      }
    });
  }
  for (auto& x : th) x.join();
}

// The plain comparison of the batch workload: 8 host threads, each driving
// its share of 64 simulations on its own stream, window graphs built,
// replayed, dropped and rebuilt as lists grow (SR_MOCK_REGROW), then all
// destroyed; graph nodes carry arguments that lived on the builder's stack.
static void graph_threads() {
  const int nth = 8, per = 8;
  std::vector<std::vector<sr_sim*>> sims(nth);
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t) {
    th.emplace_back([t, &sims]() {
      for (int i = 0; i < per; ++i) {
        sr_params p = params(32 + 16 * ((t * per + i) % 6), (t + i) % 3 ? 0.0 : 0.5, 2.0 + 0.5 * (i % 4),
                             1000 * t + i);
        sr_sim* s = nullptr;
        CHECK(sr_create(&p, nullptr, &s) == SR_OK);
        sims[t].push_back(s);
      }
      for (int rep = 0; rep < 2; ++rep)
        for (sr_sim* s : sims[t]) {
          CHECK(sr_reset(s) == SR_OK);
          int32_t done = 0;
          CHECK(sr_run_window(s, -1, nullptr, &done) == SR_OK && done > 0);
          sr_obs o;
          CHECK(sr_observables(s, &o) == SR_OK && o.tick == o.horizon_ticks);
        }
    });
  }
  for (auto& x : th) x.join();
  for (auto& v : sims)
    for (sr_sim* s : v) sr_destroy(s);
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const char* w = argv[1];
  if (!std::strcmp(w, "tuned")) tuned();
  else if (!std::strcmp(w, "server")) server();
  else if (!std::strcmp(w, "server_give_up")) server_give_up();
  else if (!std::strcmp(w, "batch_give_up")) batch_give_up();
  else if (!std::strcmp(w, "batch_threads")) batch_threads();
  else if (!std::strcmp(w, "batch")) batch();
  else if (!std::strcmp(w, "errors")) errors();
  else if (!std::strcmp(w, "threads")) threads();
  else if (!std::strcmp(w, "static")) static_step();
  else if (!std::strcmp(w, "graph_threads")) graph_threads();
  else return 2;
  CHECK(sr_mock_live_allocations() == 0);
  std::printf("ok %s\n", w);
  return 0;
}
