// sr_api.hip -- host runtime and C ABI of the synchronous-relaxation library
// (declarations and contracts in include/sr.h).
//
// A simulation owns: the committed lattice and per-subdomain carry, each
// double-buffered by window parity (the converged iteration writes the other
// parity, so committing a window is a parity flip: nothing is copied); the
// four boundary lists of every subdomain, double-buffered by iteration
// parity (iteration r reads r-1's lists and writes its own); a per-subdomain
// window event log; and one block of per-iteration flags.  The window loop of
// Sec. 4 runs on the host: launch one relaxation iteration, read the 24-byte
// flags, repeat until no boundary list changed, flip the window parity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <ctime>
#include <deque>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sr.h"
#include "sr_internal.h"

namespace sr {
hipError_t launch_relax(const Lattice& L, const Step& st, hipStream_t stream);
hipError_t launch_init_random(int8_t* s, int64_t n, uint64_t seed, hipStream_t stream);
hipError_t launch_fill(int8_t* s, int64_t n, int8_t v, hipStream_t stream);
hipError_t launch_observables(const int8_t* s, int Lx, int Ly, unsigned long long* out,
                              hipStream_t stream);
hipError_t launch_observables3d(const int8_t* s, int Lx, int Ly, int Lz, unsigned long long* out,
                                hipStream_t stream);
hipError_t launch_batch(const BatchArgs& B, int shape, int waves, size_t lds, hipStream_t stream);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);
const void* clear_flags_kernel_ptr();
const void* relax_graph_kernel_ptr(const Lattice& L);
int batch_waves_per_cu(int shape, size_t lds);
size_t relax_lds(const Lattice& L);
}  // namespace sr

using namespace sr;

struct sr_sim {
  sr_params p;
  Lattice L;
  Step st;
  hipStream_t stream = nullptr;
  int64_t W = 0, H = 0;             // window and horizon in ticks
  int64_t W0 = 0;                   // window at creation (or load): reset returns to it
  bool tune = false;                // window chosen by the tuner: adapt it
  int64_t Wmin = 1, Wmax = 1;       // bounds of the adapted window
  int64_t windows = 0, iterations = 0;
  int64_t events_base = 0, runs_base = 0;  // work done before a checkpoint load
  int32_t last_g = 0;
  unsigned long long* obs = nullptr;   // device scratch for observables
  int8_t* init_copy = nullptr;         // initial spins for sr_reset (SR_INIT_USER)
  hipEvent_t ev[2] = {};               // brackets the timed device work
  int32_t batch_hint = 8;              // iterations to queue per round trip
  int64_t relax_launches = 0;
  double relax_ms = 0.0;
  int64_t batch_tasks = 0;
  int failed = SR_OK;                   // last batched run ended in this error
  // A persistent launch that gave up waiting for work before this lattice
  // finished its window: it continues from its last committed window in a
  // later launch (gave_up), unless that happened kMaxGiveUps times in a row.
  bool gave_up = false;
  int give_ups_in_row = 0;
  int64_t restarts = 0;
  int64_t call_windows0 = 0;            // windows before the current batch call
  uint8_t* need = nullptr;              // batched form's "runs now" bytes
  double last_batch_ms = 0.0;
  // captured windows: graph of k iterations, keyed by k (rebuilt when the
  // buffers move); the window descriptor is read from dstep
  bool use_graphs = true;
  Step* dstep = nullptr;
  Step* hstep = nullptr;
  std::vector<std::pair<int, hipGraphExec_t>> graphs;
  IterFlags* hflags = nullptr;         // pinned host mirror of the flags
  std::vector<std::vector<int64_t>> log_tick, log_site;   // SR_LOG_FULL
  std::string err;
};

static thread_local std::string g_create_err;   // per calling thread

#define SR_FAIL(sim, code, ...)                                           \
  do {                                                                    \
    char _b[512];                                                         \
    std::snprintf(_b, sizeof(_b), __VA_ARGS__);                           \
    if (sim) (sim)->err = _b; else g_create_err = _b;                     \
    return (code);                                                        \
  } while (0)

#define HIP_OR_FAIL(sim, call)                                            \
  do {                                                                    \
    hipError_t _e = (call);                                               \
    if (_e != hipSuccess)                                                 \
      SR_FAIL(sim, SR_EDEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
  } while (0)

// ------------------------------------------------------------ parameters
// llround of x * 2^tick_bits for x >= 0 (scaling by a power of two is exact).
static int64_t to_ticks(double x, int tick_bits) {
  return (int64_t)std::llround(std::ldexp(x, tick_bits));
}

// Class rates round(2^28 p_k), k = (z+1)*[s=-1] + n_up for z neighbours (z = 4
// on the square lattice, 10 classes; z = 6 on the simple-cubic one, 14); p
// from eq. pMin or eq. pglauber with dE = 2 s (J (2 n_up - z) + h) (eq.
// hamil, each bond once).
static int rate_table(double J, double h, double T, int rule, int z, uint32_t out[kMaxClasses]) {
  if (!(T > 0.0) || (rule != SR_METROPOLIS && rule != SR_GLAUBER)) return -1;
  const int ncls = 2 * (z + 1);
  for (int k = 0; k < ncls; ++k) {
    int s = (k <= z) ? 1 : -1;
    int nup = k % (z + 1);
    double x = -(2.0 * s * (J * (2 * nup - z) + h)) / T;
    double p;
    if (rule == SR_METROPOLIS) {
      double theta = std::exp(x);
      p = theta < 1.0 ? theta : 1.0;
    } else {
      p = 1.0 / (1.0 + std::exp(-x));
    }
    double q = std::nearbyint(std::ldexp(p, kRateBits));
    if (q > (double)kRateOne) q = (double)kRateOne;
    out[k] = (uint32_t)q;
  }
  return 0;
}

extern "C" int sr_rate_table(const sr_params* p, uint32_t out[10]) {
  if (!p || !out) return SR_EINVAL;
  if (!(p->T > 0.0) || !std::isfinite(p->T) || !std::isfinite(p->J) || !std::isfinite(p->h))
    return SR_EINVAL;
  return rate_table(p->J, p->h, p->T, p->rule, p->Lz > 1 ? 6 : 4, out) == 0 ? SR_OK : SR_EINVAL;
}

static int sites_per_lane_shift(int nblk) {
  int S = (nblk + 63) / 64, sh = 0;
  while ((1 << sh) < S) sh++;
  return sh;
}

static const char* check_block(int Lx, int Ly, int bx, int by) {
  if (bx < 2 || by < 2 || bx > 64 || by > 64) return "bx and by must be in [2, 64]";
  if (bx * by > 1024) return "bx*by must be <= 1024";
  if (Lx % bx || Ly % by) return "Lx % bx and Ly % by must be 0";
  return nullptr;
}

// 3D blocks: every face holds at most 64 sites (a halo face is one 64-bit
// mask per wave) and the block at most 1024.
static const char* check_block3(int Lx, int Ly, int Lz, int bx, int by, int bz) {
  if (bx < 2 || by < 2 || bz < 2) return "bx, by and bz must be >= 2";
  if (bx * by > 64 || by * bz > 64 || bx * bz > 64) return "every face of a 3D block must hold <= 64 sites";
  if (Lx % bx || Ly % by || Lz % bz) return "Lx % bx, Ly % by and Lz % bz must be 0";
  return nullptr;
}

static bool is3d(const sr_params& p) { return p.Lz > 1; }
static int faces_of(const Lattice& L) { return L.Lz > 1 ? kFaces3 : kEdges; }
static size_t sites_of(const Lattice& L) { return (size_t)L.Lx * L.Ly * L.Lz; }
static int classes_of(const Lattice& L) { return L.Lz > 1 ? kClasses3 : kClasses; }

// The wipe rule makes the trajectory depend on the window, so it needs a
// window fixed by the caller (a tuned one adapts to measured iterations).
static const char* check_step_rule(int rule, bool tuned_window) {
  if (rule != SR_STEP_CONTINUE && rule != SR_STEP_WIPE) return "unknown step rule";
  if (rule == SR_STEP_WIPE && tuned_window) return "the wipe step rule needs a fixed window (window > 0)";
  return nullptr;
}

// ------------------------------------------------------------ tuner
// Block: a fixed table (never load-dependent, since the block changes the
// random streams and hence the trajectory).  Window: the step-size rule of
// Sec. 5, T_max = log N / (lambda |dG_i|), times a factor that keeps the
// expected boundary events per subdomain-window near a target; the window
// does not change results, only iteration counts.
extern "C" int sr_tune(const sr_params* p, int32_t* bx, int32_t* by, double* window) {
  if (!p || p->Lx < 4 || p->Ly < 4) return SR_EINVAL;
  if (p->Lz > 1) {
    // 3D: a cubic block, 8^3 (64-site faces) halved until it divides the
    // lattice; |dG| = b^3 - (b-2)^3 surface sites
    if (p->Lz < 4) return SR_EINVAL;
    int b = 8;
    while (b > 2 && (p->Lx % b || p->Ly % b || p->Lz % b)) b >>= 1;
    if (check_block3(p->Lx, p->Ly, p->Lz, b, b, b)) return SR_EINVAL;
    if (bx) *bx = b;
    if (by) *by = b;
    if (window) {
      double nsub = (double)(p->Lx / b) * (double)(p->Ly / b) * (double)(p->Lz / b);
      double dG = (double)(b * b * b - (b - 2) * (b - 2) * (b - 2));
      double tmax = std::log(std::max(nsub, 2.0)) / dG;
      *window = std::min(std::max(4.0 * tmax, 0.125), 2.0);
    }
    return SR_OK;
  }
  int b = 16;
  int minL = std::min(p->Lx, p->Ly);
  if (minL >= 2048 && p->T <= 1.25) b = 32;   // sparse flips: amortise per-window cost
  while (b > 2 && (p->Lx % b || p->Ly % b)) b >>= 1;
  int tbx = b, tby = b;
  if (check_block(p->Lx, p->Ly, tbx, tby)) return SR_EINVAL;
  if (bx) *bx = tbx;
  if (by) *by = tby;
  if (window) {
    double nsub = (double)(p->Lx / tbx) * (double)(p->Ly / tby);
    double dG = 2.0 * (tbx + tby) - 4.0;
    double tmax = std::log(std::max(nsub, 2.0)) / dG;
    *window = std::min(std::max(4.0 * tmax, 0.125), 2.0);
  }
  return SR_OK;
}

// ------------------------------------------------------------ buffers
static void drop_graphs(sr_sim* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.second);
  s->graphs.clear();
}

static void free_hist(sr_sim* s) {
  drop_graphs(s);
  if (s->L.hist) (void)hipFree(s->L.hist);
  s->L.hist = nullptr;
  if (s->L.wlog) (void)hipFree(s->L.wlog);
  s->L.wlog = nullptr;
}

static int alloc_hist(sr_sim* s) {
  Lattice& L = s->L;
  size_t nh = 2 * (size_t)L.nsub * faces_of(L) * (size_t)L.hcap;
  if (hipMalloc(&L.hist, nh * sizeof(uint64_t)) != hipSuccess)
    SR_FAIL(s, SR_ENOMEM, "cannot allocate %zu boundary-list entries", nh);
  if (hipMalloc(&L.wlog, (size_t)L.nsub * L.wcap * sizeof(uint64_t)) != hipSuccess)
    SR_FAIL(s, SR_ENOMEM, "cannot allocate window logs");
  return SR_OK;
}

static void free_all(sr_sim* s) {
  Lattice& L = s->L;
  free_hist(s);
  if (L.spins) (void)hipFree(L.spins);
  if (L.carry) (void)hipFree(L.carry);
  if (L.hcnt) (void)hipFree(L.hcnt);
  if (L.slot) (void)hipFree(L.slot);
  if (L.chg) (void)hipFree(L.chg);
  if (L.fct) (void)hipFree(L.fct);
  if (L.stat) (void)hipFree(L.stat);
  L.stat = nullptr;
  if (L.ck) (void)hipFree(L.ck);
  if (L.ckn) (void)hipFree(L.ckn);
  L.spins = nullptr; L.carry = nullptr; L.hcnt = nullptr; L.slot = nullptr; L.chg = nullptr;
  L.fct = nullptr; L.ck = nullptr; L.ckn = nullptr;
  if (L.wcnt) (void)hipFree(L.wcnt);
  if (L.flags) (void)hipFree(L.flags);
  if (s->obs) (void)hipFree(s->obs);
  if (s->hflags) (void)hipHostFree(s->hflags);
  if (s->init_copy) (void)hipFree(s->init_copy);
  if (s->need) (void)hipFree(s->need);
  s->need = nullptr;
  if (s->dstep) (void)hipFree(s->dstep);
  if (s->hstep) (void)hipHostFree(s->hstep);
  s->dstep = nullptr; s->hstep = nullptr;
  for (auto& e : s->ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  s->init_copy = nullptr;
  L.wcnt = nullptr; L.flags = nullptr; s->obs = nullptr; s->hflags = nullptr;
}

// Buffer capacities of a lattice whose windows are at most Wmax ticks, and
// the device bytes it will own.  Capacities: every rate is at most lambda =
// 1, so a window holds at most about (sites x window) events: that plus six
// standard deviations, boundary lists in steps of 32 entries (a relaxation
// wave holds 12 of them in LDS: 3 KB at 32, which lets more waves of the
// persistent kernel share a CU; an overflow re-runs the window with double
// capacity and the same result).  Checkpoints every kCkInt events or break
// points, up to 32 per run, enough for 1.5 x the largest expected count.
struct Plan {
  int hcap, wcap, ckint, nck;
  size_t bytes;
};
// Items between checkpoints (measured: 4 is fastest for the 1024x1024
// workload on the plain path and for the 512-lattice batch in the persistent
// kernel: 2.00 s per launch against 2.02 / 2.06 / 2.12 s at 8 / 12 / 16).
constexpr int kCkInt = 4;
static Plan plan(const sr_params& p, int64_t Wmax) {
  Plan pl;
  const bool d3 = is3d(p);
  const int bz = d3 ? p.bz : 1, Lz = d3 ? p.Lz : 1, nf = d3 ? kFaces3 : kEdges;
  double wt = std::ldexp((double)Wmax, -p.tick_bits);
  double face = d3 ? (double)std::max(p.bx * p.by, std::max(p.by * bz, p.bx * bz)) : (double)std::max(p.bx, p.by);
  double edge = face * wt, blk = (double)p.bx * p.by * bz * wt;
  pl.hcap = (int)std::min((double)(d3 ? kMaxHistCap3 : kMaxHistCap),
                          std::max(32.0, std::ceil((edge + 6.0 * std::sqrt(edge)) / 32.0) * 32.0));
  pl.wcap = (int)std::max(64.0, std::ceil((blk + 6.0 * std::sqrt(blk) + 32.0) / 64.0) * 64.0);
  if (p.hist_cap > 0) pl.hcap = p.hist_cap;
  if (p.wlog_cap > 0) pl.wcap = p.wlog_cap;
  pl.ckint = kCkInt;
  // (3D runs always start at the window start: one unused checkpoint slot)
  pl.nck = d3 ? 1 : (int)std::min(32.0, std::max(4.0, std::ceil(1.5 * blk / pl.ckint) + 1.0));
  size_t nsub = (size_t)(p.Lx / p.bx) * (p.Ly / p.by) * (Lz / bz), nsite = (size_t)p.Lx * p.Ly * Lz;
  pl.bytes = 2 * nsite + 2 * nsub * sizeof(Carry) + 2 * nsub * nf * (sizeof(uint32_t) + sizeof(int64_t)) +
             4 * (size_t)need_stride((int)nsub) + nsub * pl.nck * sizeof(Ckpt) + 2 * nsub * sizeof(uint32_t) +
             2 * nsub * nf * (size_t)pl.hcap * sizeof(uint64_t) + nsub * (size_t)pl.wcap * sizeof(uint64_t) +
             2 * (size_t)need_stride((int)nsub) + nsub * sizeof(SubStat) + (p.init == SR_INIT_USER ? nsite : 0) +
             64 * 1024;
  return pl;
}

// Parameters after validation and tuning (block, first window); 0 or SR_EINVAL.
static int resolve(sr_params& p, bool& tuned_window, std::string& why) {
  if (p.Lx < 4 || p.Ly < 4) { why = "Lx and Ly must be >= 4"; return SR_EINVAL; }
  if (p.tick_bits == 0) p.tick_bits = 28;
  if (p.tick_bits < 4 || p.tick_bits > 28) { why = "tick_bits must be in [4, 28]"; return SR_EINVAL; }
  tuned_window = (p.window == 0.0);
  if (p.Lz < 0 || p.Lz == 2 || p.Lz == 3) { why = "Lz must be 0 or 1 (2D) or >= 4 (3D)"; return SR_EINVAL; }
  if (p.bx == 0 || p.by == 0 || (is3d(p) && p.bz == 0) || p.window == 0.0) {
    int32_t tbx, tby; double tw;
    if (sr_tune(&p, &tbx, &tby, &tw) != SR_OK) { why = "tuner found no block"; return SR_EINVAL; }
    if (p.bx == 0 || p.by == 0 || (is3d(p) && p.bz == 0)) { p.bx = tbx; p.by = tby; if (is3d(p)) p.bz = tbx; }
    if (p.window == 0.0) p.window = tw;
  }
  if (const char* w = is3d(p) ? check_block3(p.Lx, p.Ly, p.Lz, p.bx, p.by, p.bz) : check_block(p.Lx, p.Ly, p.bx, p.by)) {
    why = w;
    return SR_EINVAL;
  }
  if (!(p.window > 0.0) || !std::isfinite(p.window)) { why = "window must be > 0"; return SR_EINVAL; }
  if (const char* w = check_step_rule(p.step_rule, tuned_window)) { why = w; return SR_EINVAL; }
  return SR_OK;
}

static int create_impl(const sr_params* pin, void* stream, sr_sim** out, bool init_state) {
  if (!pin || !out) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "null argument");
  *out = nullptr;
  sr_params p = *pin;
  if (p.Lx < 4 || p.Ly < 4) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "Lx and Ly must be >= 4");
  if (p.tick_bits == 0) p.tick_bits = 28;
  if (p.tick_bits < 4 || p.tick_bits > 28) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "tick_bits must be in [4, 28]");
  if (!(p.T > 0.0) || !std::isfinite(p.J) || !std::isfinite(p.h))
    SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "need T > 0 and finite J, h");
  if (p.rule != SR_METROPOLIS && p.rule != SR_GLAUBER) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "unknown rule");
  if (!(p.horizon >= 0.0) || !std::isfinite(p.horizon)) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "horizon must be >= 0");
  if (p.log_mode != SR_LOG_DIGEST && p.log_mode != SR_LOG_FULL) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "unknown log mode");
  if (p.init == SR_INIT_USER && !p.init_spins && init_state)
    SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "SR_INIT_USER needs init_spins");
  if (p.init != SR_INIT_RANDOM && p.init != SR_INIT_ALL_UP && p.init != SR_INIT_USER)
    SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "unknown init mode");
  const bool tuned_window = (p.window == 0.0);
  if (const char* why = check_step_rule(p.step_rule, tuned_window)) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "%s", why);
  if (p.Lz < 0 || p.Lz == 2 || p.Lz == 3) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "Lz must be 0 or 1 (2D) or >= 4 (3D)");
  if (p.bx == 0 || p.by == 0 || (is3d(p) && p.bz == 0) || p.window == 0.0) {
    int32_t tbx, tby; double tw;
    if (sr_tune(&p, &tbx, &tby, &tw) != SR_OK) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "tuner found no block");
    if (p.bx == 0 || p.by == 0 || (is3d(p) && p.bz == 0)) { p.bx = tbx; p.by = tby; if (is3d(p)) p.bz = tbx; }
    if (p.window == 0.0) p.window = tw;
  }
  if (const char* why = is3d(p) ? check_block3(p.Lx, p.Ly, p.Lz, p.bx, p.by, p.bz) : check_block(p.Lx, p.Ly, p.bx, p.by))
    SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "%s", why);
  if (!is3d(p)) { p.Lz = 0; p.bz = 0; }
  if (!(p.window > 0.0) || !std::isfinite(p.window)) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "window must be > 0");
  int64_t W = to_ticks(p.window, p.tick_bits), H = to_ticks(p.horizon, p.tick_bits);
  if (W < 1) W = 1;
  if (H >= ((int64_t)1 << 46)) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "horizon too long for the tick grid");
  if (p.max_iters <= 0) p.max_iters = 10000;
  if (p.hist_cap < 0 || p.wlog_cap < 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "capacities must be >= 0");
  if (p.hist_cap > (is3d(p) ? kMaxHistCap3 : kMaxHistCap))   // a wave keeps 12 (3D: 18) lists of this length in LDS
    SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "hist_cap must be <= %d", is3d(p) ? kMaxHistCap3 : kMaxHistCap);

  sr_sim* s = new sr_sim();
  s->p = p;
  s->p.init_spins = nullptr;
  s->stream = (hipStream_t)stream;
  s->W = W; s->W0 = W; s->H = H;
  s->tune = tuned_window;
  s->Wmin = std::max<int64_t>(1, to_ticks(1.0 / 64.0, p.tick_bits));
  s->Wmax = std::max<int64_t>(s->Wmin, to_ticks(4.0, p.tick_bits));
  Lattice& L = s->L;
  std::memset(&L, 0, sizeof(L));
  L.Lx = p.Lx; L.Ly = p.Ly; L.bx = p.bx; L.by = p.by;
  L.Lz = is3d(p) ? p.Lz : 1; L.bz = is3d(p) ? p.bz : 1;
  L.nbx = p.Lx / p.bx; L.nby = p.Ly / p.by; L.nbz = L.Lz / L.bz; L.nsub = L.nbx * L.nby * L.nbz;
  L.sshift = sites_per_lane_shift(p.bx * p.by * L.bz);
  L.S = 1 << L.sshift;
  L.tick_bits = p.tick_bits;
  L.wipe = p.step_rule == SR_STEP_WIPE ? 1 : 0;
  if (rate_table(p.J, p.h, p.T, p.rule, is3d(p) ? 6 : 4, L.rate) != 0) { delete s; SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "bad rate parameters"); }
  L.seed_lo = (uint32_t)p.seed; L.seed_hi = (uint32_t)(p.seed >> 32);
  if (s->tune) s->Wmax = std::max(s->Wmin, std::min(s->Wmax, 4 * W));
  const Plan pl = plan(p, s->tune ? s->Wmax : W);
  L.hcap = pl.hcap;
  L.wcap = pl.wcap;
  L.ckint = pl.ckint;
  L.nck = pl.nck;

  size_t nsite = sites_of(L);
  auto fail = [&](int code, const char* what) {
    g_create_err = what;
    free_all(s);
    delete s;
    return code;
  };
  if (hipMalloc(&L.spins, 2 * nsite) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate lattice");
  if (hipMalloc(&L.carry, 2 * (size_t)L.nsub * sizeof(Carry)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate carry");
  if (hipMalloc(&L.hcnt, 2 * (size_t)L.nsub * faces_of(L) * sizeof(uint32_t)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate list counts");
  if (hipMalloc(&L.slot, 2 * (size_t)need_stride(L.nsub)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate slots");
  if (hipMalloc(&L.chg, 2 * (size_t)need_stride(L.nsub)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate change flags");
  if (hipMalloc(&L.fct, 2 * (size_t)L.nsub * faces_of(L) * sizeof(int64_t)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate change ticks");
  if (hipMalloc(&L.ck, (size_t)L.nsub * L.nck * sizeof(Ckpt)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate checkpoints");
  if (hipMalloc(&L.ckn, (size_t)L.nsub * sizeof(uint32_t)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate checkpoint counts");
  if (hipMalloc(&L.stat, (size_t)L.nsub * sizeof(SubStat)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate work counters");
  if (hipMemsetAsync(L.stat, 0, (size_t)L.nsub * sizeof(SubStat), s->stream) != hipSuccess)
    return fail(SR_EDEVICE, "work counter init failed");
  if (hipMalloc(&L.wcnt, (size_t)L.nsub * sizeof(uint32_t)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate log counts");
  if (hipMalloc(&L.flags, kMaxBatch * sizeof(IterFlags)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate flags");
  if (hipMalloc(&s->obs, 4 * sizeof(unsigned long long)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate scratch");
  if (hipHostMalloc(&s->hflags, kMaxBatch * sizeof(IterFlags), hipHostMallocDefault) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate pinned flags");
  if (alloc_hist(s) != SR_OK) return fail(SR_ENOMEM, "cannot allocate boundary lists");
  for (auto& e : s->ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(SR_EDEVICE, "cannot create events");
  if (hipMalloc(&s->dstep, sizeof(Step)) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate step");
  if (hipMalloc(&s->need, 2 * (size_t)need_stride(L.nsub)) != hipSuccess)
    return fail(SR_ENOMEM, "cannot allocate run marks");
  if (hipHostMalloc(&s->hstep, sizeof(Step), hipHostMallocDefault) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate pinned step");
  {
    const char* ng = std::getenv("SR_NO_GRAPHS");
    s->use_graphs = !(ng && ng[0] == '1');
  }
  if (p.init == SR_INIT_USER && init_state) {
    if (hipMalloc(&s->init_copy, nsite) != hipSuccess) return fail(SR_ENOMEM, "cannot allocate initial spins");
  }

  if (init_state) {
    hipError_t e = hipSuccess;
    if (p.init == SR_INIT_RANDOM) e = launch_init_random(spins_at(L, 0), (int64_t)nsite, p.seed, s->stream);
    else if (p.init == SR_INIT_ALL_UP) e = launch_fill(spins_at(L, 0), (int64_t)nsite, 1, s->stream);
    else {
      for (size_t i = 0; i < nsite; ++i)
        if (pin->init_spins[i] != 1 && pin->init_spins[i] != -1) return fail(SR_EINVAL, "init_spins must be +1/-1");
      e = hipMemcpyAsync(spins_at(L, 0), pin->init_spins, nsite, hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->init_copy, spins_at(L, 0), nsite, hipMemcpyDeviceToDevice, s->stream);
    }
    if (e != hipSuccess) return fail(SR_EDEVICE, "initial spins failed");
    if (hipMemsetAsync(carry_at(L, 0), 0, (size_t)L.nsub * sizeof(Carry), s->stream) != hipSuccess)
      return fail(SR_EDEVICE, "carry init failed");
  }
  if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(SR_EDEVICE, "stream sync failed");
  if (p.log_mode == SR_LOG_FULL) {
    s->log_tick.resize(L.nsub);
    s->log_site.resize(L.nsub);
  }
  s->st.t_c = 0; s->st.t_end = 0; s->st.wp = 0; s->st.it = 0;
  *out = s;
  return SR_OK;
}

extern "C" int sr_create(const sr_params* p, void* hip_stream, sr_sim** out) {
  return create_impl(p, hip_stream, out, true);
}

extern "C" void sr_destroy(sr_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream); else (void)hipDeviceSynchronize();
  free_all(s);
  delete s;
}

extern "C" const char* sr_last_error(const sr_sim* s) {
  return s ? s->err.c_str() : g_create_err.c_str();
}

// ------------------------------------------------------------ window loop
constexpr int32_t kMaxWcap = 1 << 22;   // window log entries per subdomain

static int grow(sr_sim* s, uint32_t ovf) {
  Lattice& L = s->L;
  if (ovf & 1u) {
    const int cap = L.Lz > 1 ? kMaxHistCap3 : kMaxHistCap;
    if (L.hcap >= cap) SR_FAIL(s, SR_EOVERFLOW, "boundary list capacity limit reached");
    L.hcap = std::min(2 * L.hcap, cap);
  }
  if (ovf & 2u) {
    if (L.wcap >= kMaxWcap) SR_FAIL(s, SR_EOVERFLOW, "window log capacity limit reached");
    L.wcap *= 2;
  }
  free_hist(s);
  return alloc_hist(s);
}

// A window of `span` ticks overflowed its boundary lists (bit 0 of ovf) or
// its window log (bit 1).  Below the capacity limits the buffers grow and
// the window is redone.  At a limit, under the continue rule, the step size
// is halved instead (the trajectory does not depend on it: Sec. 4 box, and
// subsequent steps continue the pending pair, Sec. 5), so the same committed
// events come out in shorter windows; the tuner's bounds follow, so it does
// not climb back.  Under the wipe rule the trajectory depends on the step
// size: there the limit is an error.
static int on_overflow(sr_sim* s, uint32_t ovf, int64_t span) {
  Lattice& L = s->L;
  const bool hist_full = (ovf & 1u) && L.hcap >= (L.Lz > 1 ? kMaxHistCap3 : kMaxHistCap);
  const bool log_full = (ovf & 2u) && L.wcap >= kMaxWcap;
  if (!hist_full && !log_full) return grow(s, ovf);
  if (L.wipe)
    SR_FAIL(s, SR_EOVERFLOW, "%s capacity limit reached (the wipe-the-slate rule cannot shorten its step)",
            hist_full ? "boundary list" : "window log");
  if (span <= 1) SR_FAIL(s, SR_EOVERFLOW, "capacity limit reached by a one-tick window");
  s->W = std::max<int64_t>(1, span / 2);
  s->Wmax = std::min(s->Wmax, s->W);
  s->Wmin = std::min(s->Wmin, s->W);
  const uint32_t rest = ((ovf & 1u) && !hist_full ? 1u : 0u) | ((ovf & 2u) && !log_full ? 2u : 0u);
  return rest ? grow(s, rest) : SR_OK;
}

static int commit(sr_sim* s) {
  Lattice& L = s->L;
  if (s->p.log_mode == SR_LOG_FULL) {
    std::vector<uint32_t> cnt(L.nsub);
    std::vector<uint64_t> wl((size_t)L.nsub * L.wcap);
    HIP_OR_FAIL(s, hipMemcpyAsync(cnt.data(), L.wcnt, cnt.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HIP_OR_FAIL(s, hipMemcpyAsync(wl.data(), L.wlog, wl.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
    for (int d = 0; d < L.nsub; ++d) {
      const int x0 = (d % L.nbx) * L.bx, y0 = ((d / L.nbx) % L.nby) * L.by, z0 = (d / (L.nbx * L.nby)) * L.bz;
      for (uint32_t i = 0; i < cnt[d]; ++i) {
        uint64_t e = wl[(size_t)d * L.wcap + i];
        int v = (int)(e & 0xFFFF);
        int lx = v % L.bx, t = v / L.bx, ly = t % L.by, lz = t / L.by;
        s->log_tick[d].push_back((int64_t)(e >> kPosBits));
        s->log_site[d].push_back(((int64_t)(z0 + lz) * L.Ly + y0 + ly) * L.Lx + x0 + lx);
      }
    }
  }
  s->st.wp ^= 1;
  s->st.t_c = s->st.t_end;
  s->windows++;
  return SR_OK;
}

// A graph of k iterations of one window: clear the flags, then k relaxation
// kernels in sequence.  Node i reads the window descriptor from dstep
// (written before every replay) and is iteration dstep->it + i.  Kernel-node
// arguments are copied when a node is added, so they may live on the stack.
static hipError_t build_window_graph(const Lattice& L, const Step* dstep, int k, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr, node = nullptr;
  IterFlags* fl = L.flags;
  int nclear = k;
  void* cargs[] = {&fl, &nclear};
  hipKernelNodeParams kp = {};
  kp.func = const_cast<void*>(clear_flags_kernel_ptr());
  kp.gridDim = dim3(1);
  kp.blockDim = dim3(kMaxBatch);
  kp.sharedMemBytes = 0;
  kp.kernelParams = cargs;
  kp.extra = nullptr;
  e = hipGraphAddKernelNode(&node, g, nullptr, 0, &kp);
  prev = node;
  Lattice Lc = L;
  const Step* sp = dstep;
  std::vector<int> idx(k);
  const size_t lds = relax_lds(L);
  for (int i = 0; i < k && e == hipSuccess; ++i) {
    idx[i] = i;
    void* rargs[] = {&Lc, &sp, &idx[i]};
    hipKernelNodeParams rp = {};
    rp.func = const_cast<void*>(relax_graph_kernel_ptr(L));
    rp.gridDim = dim3(L.nsub);
    rp.blockDim = dim3(64);
    rp.sharedMemBytes = (unsigned)lds;
    rp.kernelParams = rargs;
    rp.extra = nullptr;
    e = hipGraphAddKernelNode(&node, g, &prev, 1, &rp);
    prev = node;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

// One window of the Sec. 4 box.  Iterations are queued K at a time on the
// stream; an iteration queued after the one that converged (no boundary list
// changed) or overflowed exits at once, so the host reads the flags of a
// whole batch in one round trip.
static int run_one_window(sr_sim* s, int32_t* g_out) {
  Lattice& L = s->L;
  s->st.t_end = std::min(s->st.t_c + s->W, s->H);
  int it = 0;
  // power-of-two batch sizes, so that few graphs cover every window
  int K = 2;
  while (K < s->batch_hint && K < kMaxBatch) K <<= 1;
  while (it < s->p.max_iters) {
    int k = std::min(K, s->p.max_iters - it);
    if (s->use_graphs) {
      hipGraphExec_t ge = nullptr;
      for (auto& g : s->graphs)
        if (g.first == k) ge = g.second;
      if (!ge) {
        if (s->graphs.size() >= 8) drop_graphs(s);
        HIP_OR_FAIL(s, build_window_graph(L, s->dstep, k, &ge));
        s->graphs.push_back({k, ge});
      }
      Step hs = s->st;
      hs.it = it;
      hs.fi = 0;
      *s->hstep = hs;
      HIP_OR_FAIL(s, hipMemcpyAsync(s->dstep, s->hstep, sizeof(Step), hipMemcpyHostToDevice, s->stream));
      HIP_OR_FAIL(s, hipEventRecord(s->ev[0], s->stream));
      HIP_OR_FAIL(s, hipGraphLaunch(ge, s->stream));
      HIP_OR_FAIL(s, hipEventRecord(s->ev[1], s->stream));
    } else {
      HIP_OR_FAIL(s, hipMemsetAsync(L.flags, 0, (size_t)k * sizeof(IterFlags), s->stream));
      HIP_OR_FAIL(s, hipEventRecord(s->ev[0], s->stream));
      for (int i = 0; i < k; ++i) {
        Step st = s->st;
        st.it = it + i;
        st.fi = i;
        HIP_OR_FAIL(s, launch_relax(L, st, s->stream));
      }
      HIP_OR_FAIL(s, hipEventRecord(s->ev[1], s->stream));
    }
    HIP_OR_FAIL(s, hipMemcpyAsync(s->hflags, L.flags, (size_t)k * sizeof(IterFlags), hipMemcpyDeviceToHost, s->stream));
    HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
    {
      float ms = 0.f;
      HIP_OR_FAIL(s, hipEventElapsedTime(&ms, s->ev[0], s->ev[1]));
      s->relax_ms += ms;
    }
    s->relax_launches += k;
    for (int i = 0; i < k; ++i) {
      const IterFlags& f = s->hflags[i];
      s->iterations++;
      if (f.ovf_hist || f.ovf_log) {
        int rc = on_overflow(s, (f.ovf_hist ? 1u : 0u) | (f.ovf_log ? 2u : 0u), s->st.t_end - s->st.t_c);
        if (rc != SR_OK) return rc;
        // re-run the window from its committed state (its step may be shorter)
        s->st.t_end = std::min(s->st.t_c + s->W, s->H);
        it = -k;
        break;
      }
      if (!f.changed) {
        int g = it + i + 1;
        s->last_g = g;
        if (g_out) *g_out = g;
        // queue about as many iterations as the last window needed
        s->batch_hint = std::max(2, std::min(kMaxBatch, g + 1));
        int rc = commit(s);
        if (s->tune) s->W = tune_window(s->W, g, s->Wmin, s->Wmax, kTargetGPlain);
        return rc;
      }
    }
    it += k;
    K = std::max(2, K / 2);
  }
  SR_FAIL(s, SR_ENOCONV, "window [%lld, %lld) did not converge in %d iterations",
          (long long)s->st.t_c, (long long)s->st.t_end, s->p.max_iters);
}

extern "C" int sr_run_window(sr_sim* s, int32_t n_windows, int32_t* iters_out, int32_t* n_done) {
  if (!s) return SR_EINVAL;
  if (n_done) *n_done = 0;
  if (n_windows < 0 && iters_out)
    SR_FAIL(s, SR_EINVAL, "iters_out needs n_windows >= 0 (its size bounds the windows run)");
  int32_t done = 0;
  while (n_windows < 0 || done < n_windows) {
    if (s->st.t_c >= s->H) {
      if (n_windows < 0 || done > 0) break;
      SR_FAIL(s, SR_EDONE, "committed time already at the horizon");
    }
    int32_t g = 0;
    int rc = run_one_window(s, &g);
    if (rc != SR_OK) return rc;
    if (iters_out) iters_out[done] = g;
    done++;
    if (n_done) *n_done = done;
  }
  return SR_OK;
}

// ------------------------------------------------------------ queries
extern "C" int sr_observables(sr_sim* s, sr_obs* o) {
  if (!s || !o) return SR_EINVAL;
  Lattice& L = s->L;
  unsigned long long h[2];
  HIP_OR_FAIL(s, hipMemsetAsync(s->obs, 0, 2 * sizeof(unsigned long long), s->stream));
  if (L.Lz > 1) HIP_OR_FAIL(s, launch_observables3d(spins_at(L, s->st.wp), L.Lx, L.Ly, L.Lz, s->obs, s->stream));
  else HIP_OR_FAIL(s, launch_observables(spins_at(L, s->st.wp), L.Lx, L.Ly, s->obs, s->stream));
  HIP_OR_FAIL(s, hipMemcpyAsync(h, s->obs, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  std::vector<Carry> c(L.nsub);
  std::vector<SubStat> w(L.nsub);
  HIP_OR_FAIL(s, hipMemcpyAsync(c.data(), carry_at(L, s->st.wp), c.size() * sizeof(Carry), hipMemcpyDeviceToHost, s->stream));
  HIP_OR_FAIL(s, hipMemcpyAsync(w.data(), L.stat, w.size() * sizeof(SubStat), hipMemcpyDeviceToHost, s->stream));
  HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
  std::memset(o, 0, sizeof(*o));
  o->tick = s->st.t_c;
  o->M = (int64_t)h[0];
  o->bond_sum = (int64_t)h[1];
  int64_t fmax = 0;
  for (const Carry& x : c) {
    o->flips += x.flips;
    fmax = std::max(fmax, x.nbmax);
  }
  o->events_processed = s->events_base;
  o->subdomain_runs = s->runs_base;
  for (const SubStat& x : w) {
    o->events_processed += (int64_t)x.events;
    o->subdomain_runs += (int64_t)x.runs;
  }
  o->windows = s->windows;
  o->iterations = s->iterations;
  o->last_g = s->last_g;
  o->last_f = s->windows > 0 ? (int32_t)fmax : 0;
  o->tick_bits = s->p.tick_bits;
  o->n_sub = L.nsub;
  o->bx = L.bx; o->by = L.by;
  o->Lx = L.Lx; o->Ly = L.Ly;
  o->Lz = L.Lz > 1 ? L.Lz : 0; o->bz = L.Lz > 1 ? L.bz : 0;
  o->window_ticks = s->W;
  o->horizon_ticks = s->H;
  o->relax_launches = s->relax_launches;
  o->relax_ms = s->relax_ms;
  return SR_OK;
}

extern "C" int sr_reset(sr_sim* s) {
  if (!s) return SR_EINVAL;
  Lattice& L = s->L;
  int64_t nsite = (int64_t)sites_of(L);
  if (s->p.init == SR_INIT_RANDOM) HIP_OR_FAIL(s, launch_init_random(spins_at(L, 0), nsite, s->p.seed, s->stream));
  else if (s->p.init == SR_INIT_ALL_UP) HIP_OR_FAIL(s, launch_fill(spins_at(L, 0), nsite, 1, s->stream));
  else if (s->init_copy) HIP_OR_FAIL(s, hipMemcpyAsync(spins_at(L, 0), s->init_copy, (size_t)nsite, hipMemcpyDeviceToDevice, s->stream));
  else SR_FAIL(s, SR_EINVAL, "no initial spins kept (simulation was loaded from a checkpoint)");
  HIP_OR_FAIL(s, hipMemsetAsync(carry_at(L, 0), 0, (size_t)L.nsub * sizeof(Carry), s->stream));
  HIP_OR_FAIL(s, hipMemsetAsync(L.stat, 0, (size_t)L.nsub * sizeof(SubStat), s->stream));
  HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
  s->st.t_c = 0; s->st.t_end = 0; s->st.wp = 0; s->st.it = 0;
  s->W = s->W0;                      // an adapted step size starts over
  s->windows = s->iterations = 0;
  s->events_base = s->runs_base = 0;
  s->last_g = 0;
  s->relax_launches = 0;
  s->relax_ms = 0.0;
  for (auto& v : s->log_tick) v.clear();
  for (auto& v : s->log_site) v.clear();
  return SR_OK;
}

extern "C" int sr_get_spins(sr_sim* s, int8_t* out) {
  if (!s || !out) return SR_EINVAL;
  HIP_OR_FAIL(s, hipMemcpyAsync(out, spins_at(s->L, s->st.wp), sites_of(s->L), hipMemcpyDeviceToHost, s->stream));
  HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
  return SR_OK;
}

extern "C" int sr_get_log(sr_sim* s, int32_t d, int64_t* ticks, int64_t* sites, int64_t cap, int64_t* n) {
  if (!s || d < 0 || d >= s->L.nsub || !n) return SR_EINVAL;
  if (s->p.log_mode != SR_LOG_FULL) SR_FAIL(s, SR_EINVAL, "event logs need SR_LOG_FULL");
  const auto& t = s->log_tick[d];
  const auto& v = s->log_site[d];
  *n = (int64_t)t.size();
  int64_t m = std::min<int64_t>(cap, (int64_t)t.size());
  for (int64_t i = 0; i < m; ++i) {
    if (ticks) ticks[i] = t[i];
    if (sites) sites[i] = v[i];
  }
  return SR_OK;
}

static int fetch_carry(sr_sim* s, std::vector<Carry>& c) {
  c.resize(s->L.nsub);
  HIP_OR_FAIL(s, hipMemcpyAsync(c.data(), carry_at(s->L, s->st.wp), c.size() * sizeof(Carry), hipMemcpyDeviceToHost, s->stream));
  HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
  return SR_OK;
}

extern "C" int sr_get_digests(sr_sim* s, uint64_t* digests, int64_t* flips) {
  if (!s) return SR_EINVAL;
  std::vector<Carry> c;
  int rc = fetch_carry(s, c);
  if (rc) return rc;
  for (int d = 0; d < s->L.nsub; ++d) {
    if (digests) digests[d] = c[d].digest;
    if (flips) flips[d] = c[d].flips;
  }
  return SR_OK;
}

extern "C" int sr_get_carry(sr_sim* s, int64_t* out) {
  if (!s || !out) return SR_EINVAL;
  std::vector<Carry> c;
  int rc = fetch_carry(s, c);
  if (rc) return rc;
  for (int d = 0; d < s->L.nsub; ++d) {
    out[3 * d + 0] = (int64_t)c[d].j;
    out[3 * d + 1] = c[d].anchor;
    out[3 * d + 2] = (int64_t)c[d].acc;
  }
  return SR_OK;
}

extern "C" int sr_get_rate_table(sr_sim* s, uint32_t out[10]) {
  if (!s || !out) return SR_EINVAL;
  std::memcpy(out, s->L.rate, (size_t)classes_of(s->L) * sizeof(uint32_t));
  return SR_OK;
}

// ------------------------------------------------------------ checkpoint
// Blob: header, committed spins, committed carry, then (SR_INIT_USER only)
// the initial spins, so that sr_reset works on a loaded simulation too.  A
// tuned simulation keeps its tuner state: the step size it had reached and
// the bounds it adapts within.
struct SaveHeader {
  char magic[8];
  sr_params p;
  int64_t t_c, windows, iterations, events;
  int32_t last_g, last_f;
  int32_t nsub, tune;
  int64_t W, Wmin, Wmax;
  int32_t has_init, pad;
};

extern "C" int sr_save(sr_sim* s, void* blob, size_t cap, size_t* n) {
  if (!s || !n) return SR_EINVAL;
  size_t nsite = sites_of(s->L);
  const bool has_init = s->init_copy != nullptr;
  size_t need = sizeof(SaveHeader) + nsite + (size_t)s->L.nsub * sizeof(Carry) + (has_init ? nsite : 0);
  *n = need;
  if (!blob) return SR_OK;
  if (cap < need) SR_FAIL(s, SR_EINVAL, "checkpoint buffer too small (%zu < %zu)", cap, need);
  SaveHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "SRCKPT3", 8);
  h.p = s->p;
  h.p.init_spins = nullptr;
  sr_obs o;
  int rc = sr_observables(s, &o);
  if (rc != SR_OK) return rc;
  h.t_c = s->st.t_c; h.windows = s->windows; h.iterations = s->iterations; h.events = o.events_processed;
  h.last_g = s->last_g; h.last_f = o.last_f; h.nsub = s->L.nsub;
  h.tune = s->tune ? 1 : 0;
  h.W = s->W; h.Wmin = s->Wmin; h.Wmax = s->Wmax;
  h.has_init = has_init ? 1 : 0;
  char* b = (char*)blob;
  std::memcpy(b, &h, sizeof(h));
  size_t at = sizeof(h);
  HIP_OR_FAIL(s, hipMemcpyAsync(b + at, spins_at(s->L, s->st.wp), nsite, hipMemcpyDeviceToHost, s->stream));
  at += nsite;
  HIP_OR_FAIL(s, hipMemcpyAsync(b + at, carry_at(s->L, s->st.wp), (size_t)s->L.nsub * sizeof(Carry), hipMemcpyDeviceToHost, s->stream));
  at += (size_t)s->L.nsub * sizeof(Carry);
  if (has_init) HIP_OR_FAIL(s, hipMemcpyAsync(b + at, s->init_copy, nsite, hipMemcpyDeviceToHost, s->stream));
  HIP_OR_FAIL(s, hipStreamSynchronize(s->stream));
  return SR_OK;
}

extern "C" int sr_load(const void* blob, size_t n, void* stream, sr_sim** out) {
  if (!blob || !out || n < sizeof(SaveHeader)) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "bad checkpoint");
  *out = nullptr;
  SaveHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (std::memcmp(h.magic, "SRCKPT3", 8) != 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "not a checkpoint");
  if (h.p.Lx < 4 || h.p.Ly < 4 || h.nsub <= 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "bad checkpoint header");
  size_t nsite = (size_t)h.p.Lx * h.p.Ly * (h.p.Lz > 1 ? h.p.Lz : 1);
  size_t need = sizeof(h) + nsite + (size_t)h.nsub * sizeof(Carry) + (h.has_init ? nsite : 0);
  if (n < need) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "truncated checkpoint");
  // a tuned simulation is re-created as tuned (the tuner is deterministic,
  // so the first window, its bounds and the buffer plan come out the same),
  // then given the step size it had reached
  sr_params p = h.p;
  if (h.tune) p.window = 0.0;
  int rc = create_impl(&p, stream, out, false);
  if (rc != SR_OK) return rc;
  sr_sim* s = *out;
  if (s->L.nsub != h.nsub) { sr_destroy(s); *out = nullptr; SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "checkpoint does not match its parameters"); }
  const char* b = (const char*)blob;
  size_t at = sizeof(h);
  auto fail = [&](const char* what) {
    sr_destroy(s);
    *out = nullptr;
    SR_FAIL((sr_sim*)nullptr, SR_EDEVICE, "%s", what);
  };
  if (hipMemcpyAsync(spins_at(s->L, 0), b + at, nsite, hipMemcpyHostToDevice, s->stream) != hipSuccess)
    return fail("checkpoint spins upload failed");
  at += nsite;
  if (hipMemcpyAsync(carry_at(s->L, 0), b + at, (size_t)h.nsub * sizeof(Carry), hipMemcpyHostToDevice, s->stream) != hipSuccess)
    return fail("checkpoint carry upload failed");
  at += (size_t)h.nsub * sizeof(Carry);
  if (h.has_init) {
    if (hipMalloc(&s->init_copy, nsite) != hipSuccess) {
      sr_destroy(s);
      *out = nullptr;
      SR_FAIL((sr_sim*)nullptr, SR_ENOMEM, "cannot allocate initial spins");
    }
    if (hipMemcpyAsync(s->init_copy, b + at, nsite, hipMemcpyHostToDevice, s->stream) != hipSuccess)
      return fail("checkpoint initial spins upload failed");
  }
  if (hipStreamSynchronize(s->stream) != hipSuccess) return fail("stream sync failed");
  s->st.t_c = h.t_c; s->st.wp = 0;
  s->windows = h.windows; s->iterations = h.iterations; s->events_base = h.events;
  s->last_g = h.last_g;
  if (h.tune) {
    s->tune = true;
    s->W = h.W; s->W0 = h.W; s->Wmin = h.Wmin; s->Wmax = h.Wmax;
  }
  return SR_OK;
}

// ------------------------------------------------------------ batched form
// One persistent launch runs every listed simulation to its horizon: resident
// waves take (lattice, subdomain) tasks from a device queue; the last task of
// a lattice's iteration decides convergence and enqueues the next iteration
// (only subdomains whose inputs changed) or the next window.  Lattices whose
// buffers overflowed are finished afterwards by the plain path with larger
// buffers, from their last committed window.
extern "C" int sr_batch_step(sr_sim* const* sims, int32_t n, int32_t max_windows, void* stream_);

extern "C" int sr_batch_run(sr_sim* const* sims, int32_t n, void* stream_) {
  return sr_batch_step(sims, n, -1, stream_);
}

// Device memory of one persistent launch, carved from one block: lattice
// descriptors, per-lattice run records, per-(lattice, shard) task counts, the
// queue counters and the kShards task rings.  Regions start on 256-byte
// boundaries, so the ones that must start zeroed (counts, counters, rings)
// are cleared by one kernel over a contiguous range.
struct BatchLayout {
  size_t lat, run, rem, ctr, q, total;
};
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static BatchLayout batch_layout(int m, uint64_t qn) {
  BatchLayout b;
  b.lat = 0;
  b.run = align256(b.lat + (size_t)m * sizeof(Lattice));
  b.rem = align256(b.run + (size_t)m * sizeof(LatRun));
  b.ctr = align256(b.rem + (size_t)m * kShards * sizeof(ShardRem));
  b.q = align256(b.ctr + sizeof(BatchCounters));
  b.total = align256(b.q + (size_t)kShards * qn * sizeof(unsigned long long));
  return b;
}

// Host staging of one launch: caller-provided arrays of `cap` entries.
struct BatchStage {
  Lattice* lat;
  LatRun* run;
  int* idx;
  int cap;
};

// One persistent launch in flight: what batch_begin enqueued and batch_end
// needs to collect it.
struct BatchLaunch {
  sr_sim* const* sims = nullptr;
  int m = 0;                       // lattices in the launch (hs.idx[0..m))
  int32_t max_windows = -1;
  hipStream_t stream = nullptr;
  char* base = nullptr;            // device block of the launch
  bool owned = false;              // allocated by batch_begin (freed by batch_end)
  LatRun* drun = nullptr;
  BatchCounters* dctr = nullptr;
  bool fixed_mem = false;
  int restarted = 0;               // lattices the launch gave up on (set by batch_end)
};

// Launches in a row that may give up on one lattice before it fails.
constexpr int kMaxGiveUps = 3;

// Enqueue one persistent launch over the listed simulations (sr_batch_step)
// on `stream` and return without waiting: run records and counters prepared,
// queue cleared (the grid deals every lattice's first iteration itself), the
// kernel bracketed by the first lattice's timing events.  `dev` = nullptr:
// the launch's device memory is allocated here (and freed by batch_end);
// otherwise it is the caller's block of `dev_cap` bytes and nothing is
// allocated.  yield / notify: host-coherent words (or null), see BatchArgs.
// *bl.m = 0 on return means no listed simulation had windows left.
static int batch_begin(sr_sim* const* sims, int32_t n, int32_t max_windows, hipStream_t stream,
                       BatchStage& hs, void* dev, size_t dev_cap, const uint32_t* yield, uint32_t* notify,
                       BatchLaunch& bl) {
  bl = BatchLaunch();
  bl.sims = sims;
  bl.max_windows = max_windows;
  bl.stream = stream;
  bl.fixed_mem = dev != nullptr;
  if (!sims || n <= 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "sr_batch_run needs simulations");
  if (n > 4096) SR_FAIL(sims[0], SR_EINVAL, "at most 4096 lattices per batch");
  int m = 0;
  size_t lds = 16;
  uint64_t total = 0;
  bool all16 = true;   // every lattice 16x16 blocks without self-wrap
  for (int i = 0; i < n; ++i) {
    sr_sim* s = sims[i];
    if (!s) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "null simulation in batch");
    if (s->p.log_mode != SR_LOG_DIGEST) SR_FAIL(s, SR_EINVAL, "batched runs keep digests only (SR_LOG_DIGEST)");
    if (s->L.nsub >= (1 << 20)) SR_FAIL(s, SR_EINVAL, "too many subdomains for the batch queue");
    if (s->L.Lz > 1) SR_FAIL(s, SR_EINVAL, "batched runs take 2D lattices only");
    if (s->st.t_c >= s->H) continue;
    if (m >= hs.cap) SR_FAIL(s, SR_EINVAL, "at most %d lattices per batch here", hs.cap);
    hs.idx[m++] = i;
    all16 &= s->L.bx == 16 && s->L.by == 16 && s->L.nbx > 1 && s->L.nby > 1;
    lds = std::max(lds, relax_lds(s->L));
    total += (uint64_t)s->L.nsub;
  }
  if (m == 0) return SR_OK;
  sr_sim* s0 = sims[hs.idx[0]];
  int dev_id = 0, ncu = 0;
  HIP_OR_FAIL(s0, hipGetDevice(&dev_id));
  HIP_OR_FAIL(s0, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev_id));
  // the compile-time 16x16 body whenever every lattice can take it
  // (measured with six waves per SIMD: 512 lattices of 32..512, 2.93 s
  // against 3.07-3.26 s for the runtime-shape body; three 1024x1024
  // lattices, 1.05 s against 1.18 s)
  int shape = all16 ? kBatch16NoWrap : kBatchGeneric;
  if (const char* k = std::getenv("SR_BATCH_KERNEL")) {     // test knob: force one kernel
    if (!std::strcmp(k, "generic")) shape = kBatchGeneric;
    else if (!std::strcmp(k, "16x16") && all16) shape = kBatch16NoWrap;
  }
  int per_cu = batch_waves_per_cu(shape, lds);
  if (per_cu <= 0) SR_FAIL(s0, SR_EDEVICE, "cannot size the persistent grid");
  int waves = std::max(per_cu * ncu, kShards);   // every shard needs a wave
  // a shard's ring holds its share of every lattice's current iteration
  // (tasks are dealt round-robin, at most one extra per lattice) plus the
  // tickets its waves may hold ahead of production
  uint64_t qn = 1;
  while (qn < total / kShards + (uint64_t)m + (uint64_t)waves / kShards + 64) qn <<= 1;
  const BatchLayout lay = batch_layout(m, qn);
  char* base = (char*)dev;
  if (bl.fixed_mem) {
    if (lay.total > dev_cap)
      SR_FAIL(s0, SR_EINVAL, "this batch needs %zu bytes of launch memory, more than the %zu available "
              "(fewer lattices or subdomains per call)", lay.total, dev_cap);
  } else if (hipMalloc((void**)&base, lay.total) != hipSuccess) {
    SR_FAIL(s0, SR_ENOMEM, "cannot allocate the batch queue");
  }
  bl.base = base;
  bl.owned = !bl.fixed_mem;
  auto release = [&]() {
    if (bl.owned) (void)hipFree(bl.base);
    bl.owned = false;
  };
  Lattice* dlat = (Lattice*)(base + lay.lat);
  LatRun* drun = (LatRun*)(base + lay.run);
  ShardRem* drem = (ShardRem*)(base + lay.rem);
  BatchCounters* dctr = (BatchCounters*)(base + lay.ctr);
  unsigned long long* dq = (unsigned long long*)(base + lay.q);
  for (int k = 0; k < m; ++k) {
    sr_sim* s = sims[hs.idx[k]];
    hs.lat[k] = s->L;
    hs.lat[k].need = s->need;
    // (a kernel, not a memset: callers of the no-allocation form may be
    // capturing the stream into a graph)
    if (launch_zero(s->need, 2 * (size_t)need_stride(s->L.nsub), stream) != hipSuccess) {
      release();
      SR_FAIL(s0, SR_EDEVICE, "clearing run marks failed");
    }
    LatRun& r = hs.run[k];
    std::memset(&r, 0, sizeof(r));
    r.st = s->st;
    r.st.it = 0; r.st.fi = 0;
    r.st.t_end = std::min(s->st.t_c + s->W, s->H);
    r.H = s->H; r.W = s->W;
    r.max_iters = s->p.max_iters;
    r.status = kRunning;
    r.tune = s->tune ? 1 : 0;
    r.win_budget = max_windows > 0 ? max_windows : -1;
    r.Wmin = s->Wmin; r.Wmax = s->Wmax;
    // the first iteration's tasks, their per-shard counts and shards_left
    // are dealt by the kernel itself
  }
  BatchArgs args;
  args.ctr = dctr; args.q = dq; args.lat = dlat; args.run = drun; args.rem = drem;
  args.nlat = (uint32_t)m; args.qmask = (uint32_t)(qn - 1);
  args.yield = yield;
  args.notify = notify;
  if (launch_zero(base + lay.rem, lay.total - lay.rem, stream) != hipSuccess ||
      hipMemcpyAsync(dlat, hs.lat, m * sizeof(Lattice), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(drun, hs.run, m * sizeof(LatRun), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipEventRecord(s0->ev[0], stream) != hipSuccess || launch_batch(args, shape, waves, lds, stream) != hipSuccess ||
      hipEventRecord(s0->ev[1], stream) != hipSuccess) {
    (void)hipStreamSynchronize(stream);
    release();
    SR_FAIL(s0, SR_EDEVICE, "persistent batch launch failed: %s", hipGetErrorString(hipGetLastError()));
  }
  bl.m = m;
  bl.drun = drun;
  bl.dctr = dctr;
  bl.restarted = 0;
  return SR_OK;
}

// Has the launch ended (without waiting)?
static bool batch_done(const BatchLaunch& bl, BatchStage& hs) {
  if (bl.m == 0) return true;
  return hipEventQuery(bl.sims[hs.idx[0]]->ev[1]) != hipErrorNotReady;
}

// Wait for the launch, read back the run records, bring every simulation's
// host state up to date and release the launch memory.  Overflowed lattices
// are re-run from their last committed window with grown buffers (or, for a
// caller-provided block, reported as SR_EOVERFLOW since growing allocates).
static int batch_end(BatchLaunch& bl, BatchStage& hs) {
  if (bl.m == 0) return SR_OK;
  sr_sim* const* sims = bl.sims;
  const int m = bl.m;
  sr_sim* s0 = sims[hs.idx[0]];
  BatchCounters ctr;
  const hipError_t we = hipEventSynchronize(s0->ev[1]);
  const bool ok = we == hipSuccess &&
      hipMemcpyAsync(hs.run, bl.drun, m * sizeof(LatRun), hipMemcpyDeviceToHost, bl.stream) == hipSuccess &&
      hipMemcpyAsync(&ctr, bl.dctr, sizeof(ctr), hipMemcpyDeviceToHost, bl.stream) == hipSuccess &&
      hipStreamSynchronize(bl.stream) == hipSuccess;
  if (bl.owned) (void)hipFree(bl.base);
  bl.owned = false;
  bl.m = 0;
  if (!ok) SR_FAIL(s0, SR_EDEVICE, "persistent batch kernel failed: %s", hipGetErrorString(hipGetLastError()));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, s0->ev[0], s0->ev[1]);
  int rc = SR_OK, first_bad = -1;
  for (int k = 0; k < m; ++k) {
    sr_sim* s = sims[hs.idx[k]];
    const LatRun& r = hs.run[k];
    s->st.t_c = r.st.t_c;
    s->st.wp = r.st.wp;
    s->W = r.W;
    s->windows += r.windows;
    s->iterations += r.iterations;
    if (r.windows) s->last_g = r.last_g;
    s->relax_launches += 1;
    s->relax_ms += ms;
    s->batch_tasks += r.tasks;
    int one = SR_OK;
    if (r.status == kOverflow) {
      // the decider leaves that iteration's flags in the lattice record
      uint32_t bits = (r.fl.ovf_hist ? 1u : 0u) | (r.fl.ovf_log ? 2u : 0u);
      if (bl.fixed_mem) {
        // growing the buffers would allocate: the window stays uncommitted
        one = SR_EOVERFLOW;
        s->err = "a boundary list or window log overflowed (growing it needs an allocation)";
      } else {
        // grow what overflowed (or shorten the step at a capacity limit),
        // then run this step's windows alone from the last committed one
        one = on_overflow(s, bits ? bits : 3u, r.st.t_end - r.st.t_c);
        if (one == SR_OK) one = sr_run_window(s, bl.max_windows > 0 ? bl.max_windows : -1, nullptr, nullptr);
      }
    } else if (r.status == kNoConv) {
      one = SR_ENOCONV;
      s->err = "window did not converge within max_iters (batched run)";
    } else if (r.status == kRunning && ctr.abort && ++s->give_ups_in_row <= kMaxGiveUps) {
      // the launch gave up waiting for work before this lattice finished its
      // window; the window's work is discarded and its committed state (the
      // last converged window, whose time and parity the record holds) is
      // intact, so it continues from there in a later launch, with the same
      // results (the trajectory does not depend on how windows are run)
      s->gave_up = true;
      s->restarts++;
      bl.restarted++;
    } else if (r.status != kDone && r.status != kPaused) {
      one = SR_EDEVICE;
      s->err = "batched run ended early (status " + std::to_string(r.status) +
               (ctr.abort ? ", the persistent kernel gave up waiting for work)" : ")");
    }
    if (r.status == kDone || r.status == kPaused) s->give_ups_in_row = 0;
    s->failed = one;
    if (one != SR_OK && rc == SR_OK) { rc = one; first_bad = k; }
  }
  if (rc != SR_OK) {
    char b[320];
    sr_sim* bad = sims[hs.idx[first_bad]];
    std::snprintf(b, sizeof(b), "lattice %d of the batch (status %d): %s", hs.idx[first_bad],
                  hs.run[first_bad].status, bad->err.c_str());
    for (int k = 0; k < m; ++k) sims[hs.idx[k]]->err = b;
  }
  s0->last_batch_ms = ms;
  return rc;
}

// One synchronous persistent launch (sr_batch_step and its no-allocation
// variant).
// Lattices that a launch gave up on are launched again (listed in `retry`,
// room for every lattice one launch takes), within what is left of their
// window budget.
static int batch_core(sr_sim* const* sims, int32_t n, int32_t max_windows, hipStream_t stream,
                      BatchStage& hs, void* dev, size_t dev_cap, sr_sim** retry) {
  for (int32_t i = 0; i < n; ++i)
    if (sims[i]) { sims[i]->call_windows0 = sims[i]->windows; sims[i]->gave_up = false; }
  for (;;) {
    BatchLaunch bl;
    int rc = batch_begin(sims, n, max_windows, stream, hs, dev, dev_cap, nullptr, nullptr, bl);
    if (rc != SR_OK) return rc;
    rc = batch_end(bl, hs);
    if (rc != SR_OK || bl.restarted == 0) return rc;
    int32_t k = 0, left = max_windows;
    for (int32_t i = 0; i < n; ++i) {
      sr_sim* s = sims[i];
      if (!s || !s->gave_up) continue;
      s->gave_up = false;
      if (max_windows > 0) {
        const int64_t rest = max_windows - (s->windows - s->call_windows0);
        if (rest <= 0) continue;
        left = (int32_t)std::min<int64_t>(left, rest);
      }
      retry[k++] = s;
    }
    if (k == 0) return SR_OK;
    sims = retry;
    n = k;
    max_windows = left;
  }
}

extern "C" int sr_batch_step(sr_sim* const* sims, int32_t n, int32_t max_windows, void* stream_) {
  if (!sims || n <= 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "sr_batch_run needs simulations");
  std::vector<Lattice> lat((size_t)n);
  std::vector<LatRun> run((size_t)n);
  std::vector<int> idx((size_t)n);
  std::vector<sr_sim*> retry((size_t)n);
  BatchStage hs{lat.data(), run.data(), idx.data(), n};
  return batch_core(sims, n, max_windows, (hipStream_t)stream_, hs, nullptr, 0, retry.data());
}

// ------------------------------------------------------------ no-allocation batch step
// The launch memory of sr_batch_step_static: one array per GPU, kept for the
// life of the process.  In host code `scratch` names a host-side stand-in;
// its device address on the current GPU comes from hipGetSymbolAddress, taken
// once per device, and only that address is ever passed on.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
constexpr int kStaticMaxLattices = 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;                  // serialises sr_batch_step_static calls
static void* g_scratch_ptr[kMaxDevices];        // device address of `scratch`, per GPU
static Lattice g_static_lat[kStaticMaxLattices]; // host staging (no allocation per call)
static LatRun g_static_run[kStaticMaxLattices];
static int g_static_idx[kStaticMaxLattices];
static sr_sim* g_static_retry[kStaticMaxLattices];

extern "C" int sr_batch_step_static(sr_sim* const* sims, int32_t n, int32_t max_windows, void* stream_) {
  if (!sims || n <= 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "sr_batch_step_static needs simulations");
  std::lock_guard<std::mutex> guard(g_static_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    SR_FAIL(sims[0], SR_EDEVICE, "no usable current device");
  if (!g_scratch_ptr[dev]) {
    // first call on this GPU (current): the device address of its copy
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      SR_FAIL(sims[0], SR_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  BatchStage hs{g_static_lat, g_static_run, g_static_idx, kStaticMaxLattices};
  // (lattices launched again go to g_static_retry: only launched lattices
  // are, at most kStaticMaxLattices)
  return batch_core(sims, n, max_windows, (hipStream_t)stream_, hs, g_scratch_ptr[dev], kStaticScratchBytes,
                    g_static_retry);
}

// ------------------------------------------------------------ serving
// Continuous batching, driven by the caller.  sr_server_submit queues a
// request.  One persistent launch at a time runs every admitted lattice
// towards its horizon; it is left running between calls of sr_server_pump.
// When a request is waiting whose footprint fits the budget, or a lattice
// has reached its horizon, the pump raises a host-coherent yield word that
// every lattice's decider reads at its next window boundary: each lattice
// pauses there (committed time), the launch ends within about one window of
// work, and the next pump retires the finished lattices, admits waiting
// requests in arrival order while their device footprint fits, and starts
// the next launch over all admitted lattices.  A request therefore waits for
// the windows in flight, not for a round of fixed length.  A lattice's
// result does not depend on what it shares a launch with: random streams are
// keyed by the request's own seed and subdomains, the block comes from the
// request alone, and pausing at a window boundary changes nothing (the
// trajectory does not depend on the window).  All device work is on the
// server's stream; the caller's thread does all host work.
struct sr_server {
  size_t budget = 0, used = 0, peak_used = 0;
  int32_t wpr = 0;                 // windows per lattice and launch (<= 0: no limit)
  hipStream_t stream = nullptr;
  struct Pending {
    uint64_t id;
    sr_params p;
    std::vector<int8_t> spins;
    double t_arrive;
    size_t bytes;
  };
  struct Active {
    uint64_t id;
    sr_sim* s;
    double t_arrive, t_start;
    size_t bytes;
  };
  std::deque<Pending> pending;
  std::vector<Active> active;      // admitted, in the launch or waiting for the next
  std::deque<sr_result> done;
  uint64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  int64_t rounds = 0, completed = 0, failed = 0, submitted = 0;
  int32_t peak_active = 0;
  int32_t restarts = 0;            // lattices launched again after a launch gave up on them
  double busy_s = 0.0;
  // the launch in flight
  bool running = false;
  double t_launch = 0.0;
  BatchLaunch bl;
  std::vector<sr_sim*> launch_sims;
  std::vector<Lattice> st_lat;
  std::vector<LatRun> st_run;
  std::vector<int> st_idx;
  uint32_t* ctl = nullptr;         // pinned, host-coherent: [0] yield, [1] finished count
  bool yield_raised = false;
};

static double server_now(const sr_server* v) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - v->t0).count();
}

static void server_finish(sr_server* v, sr_server::Active& a, int status) {
  sr_result r;
  std::memset(&r, 0, sizeof(r));
  r.req_id = a.id;
  r.status = status;
  r.t_arrive = a.t_arrive;
  r.t_start = a.t_start;
  if (status == SR_OK) {
    sr_obs o;
    std::vector<uint64_t> dg(a.s->L.nsub);
    if (sr_observables(a.s, &o) == SR_OK && sr_get_digests(a.s, dg.data(), nullptr) == SR_OK) {
      for (uint64_t x : dg) r.digest += x;
      r.M = o.M; r.bond_sum = o.bond_sum; r.flips = o.flips;
      r.events_processed = o.events_processed;
      r.windows = o.windows; r.iterations = o.iterations;
      r.bx = o.bx; r.by = o.by;
    } else {
      r.status = SR_EDEVICE;
    }
  }
  sr_destroy(a.s);
  r.t_done = server_now(v);
  v->used -= a.bytes;
  if (r.status == SR_OK) v->completed++; else v->failed++;
  v->done.push_back(r);
}

extern "C" int sr_server_create(size_t hbm_budget, int32_t windows_per_round, void* hip_stream,
                                sr_server** out) {
  if (!out || hbm_budget == 0) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "sr_server_create needs a budget");
  sr_server* v = new sr_server();
  v->budget = hbm_budget;
  v->wpr = windows_per_round;
  v->stream = (hipStream_t)hip_stream;
  v->t0 = std::chrono::steady_clock::now();
  if (hipHostMalloc((void**)&v->ctl, 64, hipHostMallocCoherent) != hipSuccess) {
    delete v;
    SR_FAIL((sr_sim*)nullptr, SR_ENOMEM, "cannot allocate the server's control words");
  }
  v->ctl[0] = 0u;
  v->ctl[1] = 0u;
  *out = v;
  return SR_OK;
}

extern "C" int sr_server_submit(sr_server* v, const sr_params* pin, uint64_t* req_id) {
  if (!v || !pin) return SR_EINVAL;
  sr_params p = *pin;
  if (p.log_mode != SR_LOG_DIGEST) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "served requests keep digests only");
  if (p.Lz > 1) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "served requests are 2D lattices");
  bool tuned = false;
  std::string why;
  if (resolve(p, tuned, why) != SR_OK) SR_FAIL((sr_sim*)nullptr, SR_EINVAL, "%s", why.c_str());
  int64_t W = std::max<int64_t>(1, to_ticks(p.window, p.tick_bits));
  int64_t Wmax = tuned ? std::min(4 * W, to_ticks(4.0, p.tick_bits)) : W;
  size_t bytes = plan(p, std::max<int64_t>(W, Wmax)).bytes;
  if (bytes > v->budget) SR_FAIL((sr_sim*)nullptr, SR_ENOMEM, "request needs %zu bytes, more than the budget", bytes);
  sr_server::Pending q;
  q.p = *pin;                       // the request as given (tuning redone at creation)
  if (pin->init == SR_INIT_USER && pin->init_spins)
    q.spins.assign(pin->init_spins, pin->init_spins + (size_t)pin->Lx * pin->Ly);
  q.bytes = bytes;
  q.id = v->next_id++;
  q.t_arrive = server_now(v);
  v->submitted++;
  if (req_id) *req_id = q.id;
  v->pending.push_back(std::move(q));
  return SR_OK;
}

// Collect the ended launch: run records back, finished lattices retired.
static int server_collect(sr_server* v) {
  BatchStage hs{v->st_lat.data(), v->st_run.data(), v->st_idx.data(), (int)v->st_idx.size()};
  int rc = batch_end(v->bl, hs);
  // the reason of a failed launch outlives the simulations it finishes: it
  // becomes the calling thread's last error
  if (rc != SR_OK && rc != SR_ENOCONV)
    for (auto& a : v->active)
      if (!a.s->err.empty()) { g_create_err = "server launch: " + a.s->err; break; }
  v->running = false;
  v->busy_s += server_now(v) - v->t_launch;
  v->restarts += v->bl.restarted;
  std::vector<sr_server::Active> keep;
  for (auto& a : v->active) {
    if (a.s->failed != SR_OK) server_finish(v, a, a.s->failed);
    else if (rc != SR_OK && rc != SR_ENOCONV) server_finish(v, a, rc);
    else if (a.s->st.t_c >= a.s->H) server_finish(v, a, SR_OK);
    else keep.push_back(a);
  }
  v->active.swap(keep);
  return (rc == SR_OK || rc == SR_ENOCONV) ? SR_OK : rc;
}

extern "C" int sr_server_pump(sr_server* v, int32_t* n_open) {
  if (!v) return SR_EINVAL;
  int rc = SR_OK;
  if (v->running) {
    BatchStage hs{v->st_lat.data(), v->st_run.data(), v->st_idx.data(), (int)v->st_idx.size()};
    // wait a little for the launch to end, so that callers can spin on pump
    for (int i = 0; i < 20 && !batch_done(v->bl, hs); ++i) {
      if (!v->yield_raised) {
        const bool arrived = !v->pending.empty() && v->used + v->pending.front().bytes <= v->budget;
        const bool finished = __atomic_load_n(&v->ctl[1], __ATOMIC_ACQUIRE) != 0u;
        if (arrived || finished) {
          __atomic_store_n(&v->ctl[0], 1u, __ATOMIC_RELEASE);   // pause at the next window boundary
          v->yield_raised = true;
        }
      }
      struct timespec ts = {0, 50 * 1000};
      nanosleep(&ts, nullptr);
    }
    if (!batch_done(v->bl, hs)) {
      if (n_open) *n_open = (int32_t)(v->active.size() + v->pending.size());
      return SR_OK;
    }
    rc = server_collect(v);
  }
  while (!v->pending.empty() && v->used + v->pending.front().bytes <= v->budget) {
    sr_server::Pending q = std::move(v->pending.front());
    v->pending.pop_front();
    v->used += q.bytes;
    v->peak_used = std::max(v->peak_used, v->used);
    sr_params p = q.p;
    p.init_spins = q.spins.empty() ? nullptr : q.spins.data();
    sr_server::Active a{q.id, nullptr, q.t_arrive, server_now(v), q.bytes};
    int c = sr_create(&p, v->stream, &a.s);
    if (c != SR_OK) {
      sr_result r;
      std::memset(&r, 0, sizeof(r));
      r.req_id = q.id; r.status = c; r.t_arrive = q.t_arrive; r.t_start = a.t_start;
      r.t_done = server_now(v);
      v->used -= q.bytes;
      v->failed++;
      v->done.push_back(r);
      continue;
    }
    v->active.push_back(a);
  }
  if (!v->active.empty() && rc == SR_OK) {
    v->peak_active = std::max<int32_t>(v->peak_active, (int32_t)v->active.size());
    const size_t m = v->active.size();
    v->launch_sims.resize(m);
    for (size_t k = 0; k < m; ++k) v->launch_sims[k] = v->active[k].s;
    v->st_lat.resize(m);
    v->st_run.resize(m);
    v->st_idx.resize(m);
    BatchStage hs{v->st_lat.data(), v->st_run.data(), v->st_idx.data(), (int)m};
    __atomic_store_n(&v->ctl[0], 0u, __ATOMIC_RELEASE);
    __atomic_store_n(&v->ctl[1], 0u, __ATOMIC_RELEASE);
    v->yield_raised = false;
    v->t_launch = server_now(v);
    rc = batch_begin(v->launch_sims.data(), (int32_t)m, v->wpr, v->stream, hs, nullptr, 0, v->ctl, v->ctl + 1,
                     v->bl);
    if (rc == SR_OK) {
      v->rounds++;
      v->running = v->bl.m > 0;
    } else {
      for (auto& a : v->active)
        if (!a.s->err.empty()) { g_create_err = "server launch: " + a.s->err; break; }
      for (auto& a : v->active) server_finish(v, a, rc);
      v->active.clear();
    }
  }
  if (n_open) *n_open = (int32_t)(v->active.size() + v->pending.size());
  return rc;
}

extern "C" int sr_server_poll(sr_server* v, sr_result* out, int32_t cap, int32_t* n) {
  if (!v || !n) return SR_EINVAL;
  int32_t k = 0;
  while (k < cap && !v->done.empty()) {
    out[k++] = v->done.front();
    v->done.pop_front();
  }
  *n = k;
  return SR_OK;
}

extern "C" int sr_server_stats(sr_server* v, sr_server_info* o) {
  if (!v || !o) return SR_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->submitted = v->submitted;
  o->completed = v->completed;
  o->failed = v->failed;
  o->queued = (int64_t)v->pending.size();
  o->rounds = v->rounds;
  o->bytes_in_use = (int64_t)v->used;
  o->peak_bytes = (int64_t)v->peak_used;
  o->peak_active = v->peak_active;
  o->restarts = v->restarts;
  o->busy_s = v->busy_s;
  o->uptime_s = server_now(v);
  return SR_OK;
}

extern "C" void sr_server_destroy(sr_server* v) {
  if (!v) return;
  if (v->running) {
    // end the launch at the next window boundaries, then collect it
    __atomic_store_n(&v->ctl[0], 1u, __ATOMIC_RELEASE);
    BatchStage hs{v->st_lat.data(), v->st_run.data(), v->st_idx.data(), (int)v->st_idx.size()};
    (void)batch_end(v->bl, hs);
    v->running = false;
  }
  for (auto& a : v->active) sr_destroy(a.s);
  if (v->ctl) (void)hipHostFree(v->ctl);
  delete v;
}
