// Host-only stand-ins for the HIP runtime and for the library's kernel
// launchers, so that the host runtime (sr_api.hip) can be exercised under
// AddressSanitizer without a GPU.  Device memory is host memory; every
// allocation is tracked and a bad free aborts.  The "kernels" do no physics:
//   relaxation  -- a window converges after SR_MOCK_G iterations (default 1);
//   batch       -- every lattice commits windows of its current length, with
//                  the same step-size rule and window budget as the device
//                  decider; SR_MOCK_OVERFLOW=1 makes lattice 0 report an
//                  overflow of both buffers (2: of its window log only) so
//                  that the plain fallback runs; SR_MOCK_GIVE_UP=n makes the
//                  first n launches leave lattice 0 running and give up, as
//                  the device kernel does when it waits far too long for
//                  work.
#include "hip/hip_runtime.h"

#include <atomic>
#include <cstdio>
#include <mutex>
#include <set>
#include <vector>

#include "../../paper_cs_0405053_amd/csrc/sr_internal.h"

static std::set<void*> g_dev, g_host, g_ev;
static std::mutex g_mu;   // the stand-in runtime may be called from several threads
static size_t g_malloc_calls = 0;

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

hipError_t hipMalloc(void** p, size_t n) {
  *p = std::calloc(1, n ? n : 1);
  std::lock_guard<std::mutex> g(g_mu);
  g_malloc_calls++;
  g_dev.insert(*p);
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_dev.erase(p)) { std::fprintf(stderr, "hipFree of unknown pointer %p\n", p); std::abort(); }
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = std::calloc(1, n ? n : 1);
  std::lock_guard<std::mutex> g(g_mu);
  g_host.insert(*p);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_host.erase(p)) { std::fprintf(stderr, "hipHostFree of unknown pointer %p\n", p); std::abort(); }
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t)std::malloc(8);
  std::lock_guard<std::mutex> g(g_mu);
  g_ev.insert(*e);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ev.erase(e)) { std::fprintf(stderr, "hipEventDestroy of unknown event\n"); std::abort(); }
  std::free(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.01f; return hipSuccess; }
// every stand-in launch completes before it returns
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "host stand-in error"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// a __device__ array is a host array here: its "device address" is itself
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }

// Graphs.  A kernel node copies its arguments when it is added (as HIP
// does), interpreted by the stand-in kernel it names; an instantiated graph
// replays its nodes in order.  Graph objects are tracked like allocations.
static char g_clear_kernel, g_relax_kernel;          // stand-in kernel addresses
struct MockNode {
  int kind;                 // 0 = clear flags, 1 = relaxation iteration
  sr::IterFlags* flags;     // clear: first flag entry
  int n;                    // clear: entries; relax: node index i
  sr::Lattice L;            // relax: lattice descriptor (by value)
  const sr::Step* step;     // relax: window descriptor, read at replay
};
struct ihipGraphNode_t { int index; };
struct ihipGraph_t { std::vector<MockNode> nodes; std::vector<ihipGraphNode_t*> handles; };
struct ihipGraphExec_t { std::vector<MockNode> nodes; };
static std::set<void*> g_graphs, g_execs;

static void relax_flags(sr::IterFlags* f, int it, const sr::Lattice& L) {
  std::memset(f, 0, sizeof(*f));
  f->changed = it < env_int("SR_MOCK_G", 1) - 1;
  // SR_MOCK_REGROW=1: the boundary lists of a lattice overflow until they
  // hold 128 entries (the host grows them, dropping and rebuilding graphs)
  if (env_int("SR_MOCK_REGROW", 0) && L.hcap < 128) f->ovf_hist = 1;
}
static void count_runs(const sr::Lattice& L) {
  for (int d = 0; d < L.nsub; ++d) L.stat[d].runs += 1;
}
// Iterations queued behind one that converged (or overflowed) do nothing, as
// on the device.
static bool queued_after_convergence(const sr::IterFlags* f, int fi) {
  return fi > 0 && (!f[fi - 1].changed || f[fi - 1].ovf_hist || f[fi - 1].ovf_log);
}

hipError_t hipGraphCreate(hipGraph_t* g, unsigned) {
  *g = new ihipGraph_t();
  std::lock_guard<std::mutex> lk(g_mu);
  g_graphs.insert(*g);
  return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* p) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_graphs.count(g)) { std::fprintf(stderr, "node added to unknown graph\n"); std::abort(); }
  }
  // the library builds chains: each node depends on the one before
  if (g->nodes.empty() ? ndeps != 0 : (ndeps != 1 || deps[0] != g->handles.back())) {
    std::fprintf(stderr, "graph node dependencies are not a chain\n");
    std::abort();
  }
  MockNode n{};
  if (p->func == &g_clear_kernel) {
    n.kind = 0;
    n.flags = *(sr::IterFlags**)p->kernelParams[0];
    n.n = *(int*)p->kernelParams[1];
  } else if (p->func == &g_relax_kernel) {
    n.kind = 1;
    n.L = *(sr::Lattice*)p->kernelParams[0];
    n.step = *(const sr::Step**)p->kernelParams[1];
    n.n = *(int*)p->kernelParams[2];
  } else {
    std::fprintf(stderr, "unknown kernel in graph node\n");
    std::abort();
  }
  g->nodes.push_back(n);
  g->handles.push_back(new ihipGraphNode_t{(int)g->nodes.size() - 1});
  *node = g->handles.back();
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new ihipGraphExec_t{g->nodes};
  std::lock_guard<std::mutex> lk(g_mu);
  g_execs.insert(*e);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_graphs.erase(g)) { std::fprintf(stderr, "hipGraphDestroy of unknown graph\n"); std::abort(); }
  }
  for (auto* h : g->handles) delete h;
  delete g;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_execs.count(e)) { std::fprintf(stderr, "hipGraphLaunch of unknown graph\n"); std::abort(); }
  }
  for (const MockNode& n : e->nodes) {
    if (n.kind == 0) {
      std::memset(n.flags, 0, (size_t)n.n * sizeof(sr::IterFlags));
    } else {
      const int i = n.n;
      if (queued_after_convergence(n.L.flags, i)) continue;
      relax_flags(&n.L.flags[i], n.step->it + i, n.L);
      count_runs(n.L);
    }
  }
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_execs.erase(e)) { std::fprintf(stderr, "hipGraphExecDestroy of unknown graph\n"); std::abort(); }
  }
  delete e;
  return hipSuccess;
}

extern "C" size_t sr_mock_malloc_calls() {
  std::lock_guard<std::mutex> g(g_mu);
  return g_malloc_calls;
}

extern "C" size_t sr_mock_live_allocations() {
  std::lock_guard<std::mutex> g(g_mu);
  return g_dev.size() + g_host.size() + g_ev.size() + g_graphs.size() + g_execs.size();
}

namespace sr {
hipError_t launch_relax(const Lattice& L, const Step& st, hipStream_t) {
  if (queued_after_convergence(L.flags, st.fi)) return hipSuccess;
  relax_flags(&L.flags[st.fi], st.it, L);
  count_runs(L);
  return hipSuccess;
}
hipError_t launch_init_random(int8_t* s, int64_t n, uint64_t seed, hipStream_t) {
  for (int64_t i = 0; i < n; ++i) s[i] = ((seed + (uint64_t)i) & 1) ? 1 : -1;
  return hipSuccess;
}
hipError_t launch_fill(int8_t* s, int64_t n, int8_t v, hipStream_t) {
  std::memset(s, (unsigned char)v, (size_t)n);
  return hipSuccess;
}
hipError_t launch_observables(const int8_t* s, int Lx, int Ly, unsigned long long* out, hipStream_t) {
  long long m = 0;
  for (int64_t i = 0; i < (int64_t)Lx * Ly; ++i) m += s[i];
  out[0] = (unsigned long long)m;
  out[1] = 0;
  return hipSuccess;
}
hipError_t launch_observables3d(const int8_t* s, int Lx, int Ly, int Lz, unsigned long long* out, hipStream_t) {
  long long m = 0;
  for (int64_t i = 0; i < (int64_t)Lx * Ly * Lz; ++i) m += s[i];
  out[0] = (unsigned long long)m;
  out[1] = 0;
  return hipSuccess;
}
static std::atomic<int> g_batch_launches{0};
hipError_t launch_batch(const BatchArgs& B, int, int, size_t, hipStream_t) {
  const int G = env_int("SR_MOCK_G", 1);
  const bool give_up = g_batch_launches++ < env_int("SR_MOCK_GIVE_UP", 0);
  for (uint32_t k = 0; k < B.nlat; ++k) {
    LatRun& r = B.run[k];
    const int ovf = env_int("SR_MOCK_OVERFLOW", 0);
    if (k == 0 && give_up) {
      r.status = kRunning;
      B.ctr->abort = 1;
      continue;
    }
    if (k == 0 && ovf) {
      // 1: both buffers overflowed; 2: only the window log did
      r.status = kOverflow;
      r.fl.ovf_hist = ovf == 1;
      r.fl.ovf_log = 1;
      B.ctr->done++;
      continue;
    }
    int budget = r.win_budget;
    r.status = kRunning;
    while (r.status == kRunning) {
      r.st.t_c = r.st.t_end;
      r.st.wp ^= 1;
      r.windows++;
      r.iterations += G;
      r.last_g = G;
      if (r.tune) r.W = tune_window(r.W, G, r.Wmin, r.Wmax, kTargetGBatch);
      if (r.st.t_c >= r.H) { r.status = kDone; break; }
      r.st.t_end = r.st.t_c + r.W < r.H ? r.st.t_c + r.W : r.H;
      if (budget > 0 && --budget == 0) r.status = kPaused;
    }
    B.ctr->done++;
  }
  return hipSuccess;
}
// workgroups land on XCDs 0..7 in turn, as on the device
hipError_t launch_zero(void* p, size_t bytes, hipStream_t) {
  std::memset(p, 0, bytes);
  return hipSuccess;
}
int batch_waves_per_cu(int, size_t) { return 4; }
size_t relax_lds(const Lattice& L) { return 1024 + 64 * (size_t)L.hcap; }
const void* clear_flags_kernel_ptr() { return &g_clear_kernel; }
const void* relax_graph_kernel_ptr(const Lattice&) { return &g_relax_kernel; }
}  // namespace sr
