// sr_internal.h -- device-side data layout shared by the kernels and the
// host runtime of the synchronous-relaxation library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

constexpr int kClasses = 10;             // Sec. 3: 2 spin states x 5 up-counts
constexpr uint32_t kRateOne = 1u << 28;  // rates are round(2^28 p)
constexpr int kRateBits = 28;
constexpr int64_t kTickInf = (int64_t)1 << 62;  // "no pending event"
constexpr int kEdges = 4;                // boundary lists: N, S, W, E
enum Edge { kN = 0, kS = 1, kW = 2, kE = 3 };
constexpr int kPosBits = 16;             // history entry = tick << 16 | position

// Per-subdomain state at committed time (or at a working window end).
struct alignas(64) Carry {
  uint64_t j;        // index of the pending random pair
  int64_t anchor;    // tick of the last own event or break point
  uint64_t acc;      // hazard integrated over [anchor_0, anchor) (Q(28+tick_bits))
  uint64_t digest;   // order-free digest of committed events
  int64_t flips;     // committed flips
  int64_t wflips;    // flips of the working window (used by commit)
  int64_t pad[2];
};

// Per-iteration flags, cleared before every iteration.
struct IterFlags {
  uint32_t changed;      // some boundary history differs from the previous iteration
  uint32_t overflow;     // some history / window-log buffer overflowed
  uint32_t fmax;         // max boundary-site events of one subdomain
  uint32_t pad0;
  unsigned long long events;  // events simulated in this iteration
};

// Everything one relaxation iteration of one lattice needs.
struct Lattice {
  int32_t Lx, Ly, bx, by, nbx, nby, nsub;
  int32_t S;              // sites per lane (power of 2, 1..16)
  int32_t sshift;         // log2(S)
  int32_t tick_bits;
  uint32_t rate[kClasses];
  uint32_t seed_lo, seed_hi;
  int32_t hcap;           // entries per boundary list
  int32_t wcap;           // entries per subdomain window log
  int8_t* spins[2];       // committed lattice, indexed by window parity
  Carry* carry[2];        // indexed by window parity
  uint64_t* hist[2];      // [nsub][4][hcap], indexed by iteration parity
  uint32_t* hcnt[2];      // [nsub][4]
  uint64_t* wlog;         // [nsub][wcap]: tick << 16 | local site
  uint32_t* wcnt;         // [nsub]
  IterFlags* flags;
};

// Where a lattice stands in its window loop (host mirror and device copy).
struct Step {
  int64_t t_c, t_end;     // window [t_c, t_end)
  int32_t wp;             // window parity: spins[wp], carry[wp] are committed
  int32_t it;             // iteration index within the window
};

}  // namespace sr
