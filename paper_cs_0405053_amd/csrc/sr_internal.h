// sr_internal.h -- device-side data layout shared by the kernels and the
// host runtime of the synchronous-relaxation library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

constexpr int kClasses = 10;             // Sec. 3: 2 spin states x 5 up-counts
constexpr int kClasses3 = 14;            // 3D simple-cubic: 2 spin states x 7 up-counts
constexpr int kMaxClasses = 14;
constexpr uint32_t kRateOne = 1u << 28;  // rates are round(2^28 p)
constexpr int kRateBits = 28;
constexpr int64_t kTickInf = (int64_t)1 << 62;  // "no pending event"
constexpr int kEdges = 4;                // boundary lists: N, S, W, E
enum Edge { kN = 0, kS = 1, kW = 2, kE = 3 };
constexpr int kPosBits = 16;             // history entry = tick << 16 | position
constexpr int kMaxHistCap = 1024;        // entries per boundary list, at most
constexpr int kFaces3 = 6;               // 3D boundary lists: W, E, N, S, D, U
enum Face3 { kFW = 0, kFE = 1, kFN = 2, kFS = 3, kFD = 4, kFU = 5 };
constexpr int kMaxHistCap3 = 448;        // 3D: 18 lists of this length in LDS (< 64 KiB)

// Per-subdomain state at committed time (or at a working window end).
struct alignas(64) Carry {
  uint64_t j;        // index of the pending random pair
  int64_t anchor;    // tick of the last own event or break point
  uint64_t acc;      // hazard integrated over [anchor_0, anchor) (Q(28+tick_bits))
  uint64_t digest;   // order-free digest of committed events
  int64_t flips;     // committed flips
  int64_t wflips;    // flips of the working window (used by commit)
  int64_t nbound;    // own events on boundary sites in this run's window
  int64_t nbmax;     // the largest nbound over this window's runs: the
                     // paper's f (Sec. 6: boundary events of a PE in one
                     // iteration; a step's f is the largest over its
                     // iterations) for this subdomain
};

// Work counters of one subdomain (owned by the wave that runs it: read at the
// start of a run, written at its end; summed by the host on request).
struct SubStat {
  unsigned long long events;  // events simulated, re-simulations included
  unsigned long long runs;    // relaxation runs
};

// Snapshot of one subdomain's simulation state inside a window: the state
// after every event and break point with tick < T.  A later iteration whose
// inputs first differ at tick >= T resumes here instead of at the window
// start (same inputs before T give the same state at T).  Written by one
// wave with two full-line vector stores: the class words of its 64 lanes,
// then 32 metadata words from lanes 0..31 (layout kCk* below).
struct alignas(256) Ckpt {
  uint64_t cls[64];        // class nibbles, one word per lane
  uint64_t meta[32];
};
enum CkptWord {
  kCkCounts = 0,           // words 0..4: N_{2w} | N_{2w+1} << 32 (class counts)
  kCkT = 5,                // T
  kCkJ = 6,                // index of the pending random pair
  kCkAcc = 7,              // integrated hazard
  kCkAnchor = 8,
  kCkHalo = 9,             // words 9..12: N, S, W, E halo spins
  kCkDsum = 13,            // digest sum of the window-log entries flushed so far
  kCkNev = 14,             // window events so far | (of which on the boundary) << 32
  kCkOut01 = 15,           // own boundary-list lengths N | S << 32
  kCkOut23 = 16,           // W | E << 32
  kCkHead = 17,            // position in the merged neighbour-flip stream
  kCkWords = 18
};

// Per-iteration flags, cleared before every iteration.  Set with plain
// stores of the value 1 (idempotent, so no read-modify-write on one shared
// line by thousands of waves); visible to the next launch, or to the batched
// decider through its release / acquire fences.
struct IterFlags {
  uint32_t changed;      // some boundary history differs from the previous iteration
  uint32_t ovf_hist;     // some boundary list overflowed
  uint32_t ovf_log;      // some window log overflowed (or a run was cut short)
  uint32_t pad;
};

// Everything one relaxation iteration of one lattice needs.
struct Lattice {
  int32_t Lx, Ly, bx, by, nbx, nby, nsub;
  int32_t Lz, bz, nbz;    // 3D simple-cubic lattice when Lz > 1 (else 1, 1, 1)
  int32_t S;              // sites per lane (power of 2, 1..16)
  int32_t sshift;         // log2(S)
  int32_t tick_bits;
  uint32_t rate[kMaxClasses];  // 10 classes in 2D, 14 in 3D
  uint32_t seed_lo, seed_hi;
  int32_t hcap;           // entries per boundary list
  int32_t wcap;           // entries per subdomain window log
  int32_t wipe;           // step rule: 1 = every window start t_c > 0 drops
                          // the pending pair (wipe the slate, Sec. 5)
  // Double buffers are single allocations; buffer q starts at base + q * stride.
  int8_t* spins;          // 2 x Lx*Ly: committed lattice, by window parity
  Carry* carry;           // 2 x nsub: by window parity
  uint64_t* hist;         // 2 x [nsub][4][hcap]: two list slots per subdomain
  uint32_t* hcnt;         // 2 x [nsub][4]: list lengths, per slot
  uint8_t* slot;          // 2 x need_stride(nsub): slot holding a subdomain's
                          // latest lists, by iteration parity
  uint8_t* chg;           // 2 x need_stride(nsub): which of a subdomain's lists
                          // (bit per edge N, S, W, E) changed in that
                          // iteration, by parity
  int64_t* fct;           // 2 x [nsub][4]: per slot, first tick at which a list
                          // differs from its previous version (kTickInf: same)
  Ckpt* ck;               // [nsub][nck] checkpoints of each subdomain's last run
  uint32_t* ckn;          // [nsub] valid checkpoints of that run
  int32_t nck;            // checkpoints per subdomain and window
  int32_t ckint;          // events + break points between checkpoints
  uint8_t* need;          // batched form: 2 x need_stride(nsub) bytes, by
                          // iteration parity: 1 = the subdomain runs in
                          // that iteration (set by the runs of the one
                          // before, cleared by the subdomain's own run)
  SubStat* stat;          // [nsub]
  uint64_t* wlog;         // [nsub][wcap]: tick << 16 | local site
  uint32_t* wcnt;         // [nsub]
  IterFlags* flags;       // [kMaxBatch], one per queued iteration
};

constexpr int kMaxBatch = 64;   // iterations queued per host round trip

// Buffer q (0 or 1) of a double buffer.
template <class LT>
__host__ __device__ inline int8_t* spins_at(const LT& L, int q) {
  return L.spins + (int64_t)(q & 1) * ((int64_t)L.Lx * L.Ly * L.Lz);
}
template <class LT>
__host__ __device__ inline Carry* carry_at(const LT& L, int q) { return L.carry + (q & 1) * L.nsub; }
template <class LT>
__host__ __device__ inline uint64_t* hist_at(const LT& L, int q) {
  return L.hist + (int64_t)(q & 1) * ((int64_t)L.nsub * kEdges * L.hcap);
}
template <class LT>
__host__ __device__ inline uint32_t* hcnt_at(const LT& L, int q) {
  return L.hcnt + (q & 1) * (L.nsub * kEdges);
}
// Per-subdomain byte arrays (slot, change mask, run marks) are padded to a
// multiple of 64 subdomains, so that they can be copied 16 bytes at a time.
__host__ __device__ inline int need_stride(int nsub) { return (nsub + 63) & ~63; }
template <class LT>
__host__ __device__ inline uint8_t* slot_at(const LT& L, int q) { return L.slot + (q & 1) * need_stride(L.nsub); }
template <class LT>
__host__ __device__ inline uint8_t* chg_at(const LT& L, int q) { return L.chg + (q & 1) * need_stride(L.nsub); }
template <class LT>
__host__ __device__ inline uint8_t* need_at(const LT& L, int q) {
  return L.need + (q & 1) * need_stride(L.nsub);
}
template <class LT>
__host__ __device__ inline int64_t* fct_at(const LT& L, int q) {
  return L.fct + (q & 1) * (L.nsub * kEdges);
}

// Where a lattice stands in its window loop.
struct Step {
  int64_t t_c, t_end;     // window [t_c, t_end)
  int32_t wp;             // window parity: spins[wp], carry[wp] are committed
  int32_t it;             // iteration index within the window
  int32_t fi;             // this iteration's entry in Lattice::flags
  int32_t pad;
};

// Per-lattice state of the persistent batched kernel (device resident).
struct LatRun {
  Step st;                 // current window and iteration
  IterFlags fl;            // flags of the current iteration
  int64_t H, W;            // horizon and window (ticks)
  int32_t shards_left;     // shards still running tasks of the current iteration
  int32_t max_iters;
  int32_t status;          // kRunning, kDone, kOverflow, kNoConv
  int32_t last_g;
  int64_t windows, iterations, tasks;
  int32_t tune;            // adapt W after every window (see tune_window)
  int32_t win_budget;      // windows to commit in this launch (< 0: no limit)
  int64_t Wmin, Wmax;
};
enum { kRunning = 0, kDone = 1, kOverflow = 2, kNoConv = 3, kBad = 4, kPaused = 5 };

// Step size for the next window (Sec. 4 box: a step size is chosen at every
// step; the trajectory does not depend on it).  Aims at about `target`
// iterations per window, at most halving or doubling per window.  Shorter
// windows re-simulate less but pay the per-window cost more often, and that
// cost differs by executor: the plain form's host loop waits for every
// window, the persistent kernel's decider starts the next one on the device.
// Measured best on the 512-lattice batch: plain 12 (8 streams 16.7 s against
// 20.6 s at 6), persistent 6 (1.43 s per launch against 1.45 / 1.58 / 1.75 /
// 1.53 s at 8 / 10 / 12 / 5).
constexpr int kTargetGPlain = 12, kTargetGBatch = 6;
__host__ __device__ inline int64_t tune_window(int64_t W, int g, int64_t Wmin, int64_t Wmax, int target) {
  if (g < 1) g = 1;
  int64_t want = (int64_t)((double)W * target / g);
  int64_t nw = (W + want) / 2;                 // damped
  if (nw < W / 2) nw = W / 2;
  if (nw > 2 * W) nw = 2 * W;
  if (nw < Wmin) nw = Wmin;
  if (nw > Wmax) nw = Wmax;
  return nw < 1 ? 1 : nw;
}

// Device work queue of (lattice, subdomain) tasks, dealt over kShards shards.
// Every atomic on these counters is performed at the memory side, so a single
// shared ticket counter would serialise the whole grid: each shard is a ring
// with its own head / tail on its own cache line, and a wave serves one
// shard.  A slot holds (ticket + 1) << 32 | lattice << 20 | subdomain; a
// consumer owning ticket p of a shard waits until slot p & qmask of that
// shard's ring carries p + 1.
constexpr int kShards = 8;
struct alignas(128) ShardCtr {
  unsigned long long head;     // next ticket to hand to a consumer
  unsigned long long tail;     // next ticket to hand to a producer
};
struct BatchCounters {
  ShardCtr sh[kShards];
  alignas(128) uint32_t done;  // lattices finished
  uint32_t abort;              // set when a wave waited far too long
};
// Tasks of one lattice's current iteration still running in one shard (own
// cache line).  The last task of a shard then counts down the lattice's
// shards_left; the last shard's last task decides the iteration.
struct alignas(128) ShardRem {
  int32_t n;
};
// Persistent kernel instantiations (block shape class of a whole launch).
enum { kBatchGeneric = 0, kBatch16NoWrap = 1 };
struct BatchArgs {             // read-only for the kernel's lifetime
  BatchCounters* ctr;
  unsigned long long* q;       // kShards rings of qmask + 1 slots
  const Lattice* lat;
  LatRun* run;
  ShardRem* rem;               // [nlat][kShards]
  uint32_t nlat, qmask;
  // host-coherent pinned words (or null): `yield` != 0 asks every lattice to
  // pause at its next window boundary, so that the launch ends and the host
  // can admit and retire; `notify` counts lattices that reached their horizon
  const uint32_t* yield;
  uint32_t* notify;
};

}  // namespace sr
