// sr_device.h -- device helpers shared by the 2D and 3D relaxation kernels
// of the synchronous-relaxation library: wavefront primitives (ballots,
// lane reads, DPP scans), the random numbers of the presimulated list
// (Philox-4x32-10 and a fixed-point -ln), integer event times, the merged
// neighbour-flip stream in LDS, the end-of-run list comparison and the event
// digest mixer.  Not part of the C ABI.
#pragma once
#include "sr_internal.h"

namespace sr {

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ uint32_t rdl(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t rdl64(uint64_t v, int l) {
  return (uint64_t)rdl((uint32_t)v, l) | ((uint64_t)rdl((uint32_t)(v >> 32), l) << 32);
}
// v with lane L's word replaced by the uniform value x (two v_writelane;
// this compiler has no builtin for it, and the asm reads and writes only
// registers).
template <int L>
__device__ __forceinline__ uint64_t wrl64(uint64_t v, uint64_t x) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint32_t xl = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t xh = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  __asm__("v_writelane_b32 %0, %1, %2" : "+v"(lo) : "s"(xl), "i"(L));
  __asm__("v_writelane_b32 %0, %1, %2" : "+v"(hi) : "s"(xh), "i"(L));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
// The same for a lane chosen at run time (a uniform index).
__device__ __forceinline__ uint64_t wrl64_at(uint64_t v, uint64_t x, int l) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint32_t xl = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t xh = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  const int ls = __builtin_amdgcn_readfirstlane(l);
  // a VALU instruction reads one SGPR besides M0: the lane select goes in M0
  __asm__("s_mov_b32 m0, %4\n\ts_nop 0\n\tv_writelane_b32 %0, %2, m0\n\tv_writelane_b32 %1, %3, m0"
          : "+v"(lo), "+v"(hi) : "s"(xl), "s"(xh), "s"(ls) : "m0");
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ int ctz64(uint64_t m) { return __builtin_ctzll(m); }
__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }


template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp0(uint32_t x) {
  // lanes whose DPP source is outside the row (or whose row is masked off)
  // read 0
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xf, false);
}

// Inclusive prefix sum of 32-bit values over the 64 lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += dpp0<0x111, 0xf>(x);  // row_shr:1
  x += dpp0<0x112, 0xf>(x);  // row_shr:2
  x += dpp0<0x114, 0xf>(x);  // row_shr:4
  x += dpp0<0x118, 0xf>(x);  // row_shr:8
  x += dpp0<0x142, 0xa>(x);  // row_bcast:15 into rows 1, 3
  x += dpp0<0x143, 0xc>(x);  // row_bcast:31 into rows 2, 3
  return x;
}

// Inclusive prefix sum of 64-bit values within each row of 16 lanes, four
// Hillis-Steele steps (row_shr 1, 2, 4, 8).  Each step is one 64-bit add
// whose first operand is the row-shifted value: a carry-out add and a
// carry-in add with the DPP shift applied to them directly.  Lanes whose
// source lies outside the row are disabled by DPP (bound_ctrl off) and keep
// their value, which is what adding 0 gives.  A DPP read of a register that
// a VALU instruction just wrote needs two wait states: `s_nop 1` before each
// step.  The asm touches registers and VCC only.
__device__ __forceinline__ uint64_t row_incl_scan64(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  __asm__("s_nop 1\n\t"
          "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
          "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
          "s_nop 1\n\t"
          "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
          "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
          "s_nop 1\n\t"
          "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
          "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
          "s_nop 1\n\t"
          "v_add_co_u32_dpp %0, vcc, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
          "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc row_shr:8 row_mask:0xf bank_mask:0xf"
          : "+v"(lo), "+v"(hi) : : "vcc");
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// ------------------------------------------------------------ random numbers
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its
// published round function: multipliers 0xD2511F53 / 0xCD9E8D57, key
// increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ void philox4x32_10(uint32_t k0, uint32_t k1, uint32_t& c0,
                                              uint32_t& c1, uint32_t& c2, uint32_t& c3) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
}

// -ln(U), U = (u|1)/2^64, as an integer in units of 2^-(28+tick_bits):
// binary logarithm of the normalised mantissa by 32 repeated squarings of a
// truncated Q1.31 value, then one 64x64->128 product with floor(ln2 * 2^64).
__device__ __forceinline__ uint64_t neglog_fixed(uint64_t u, int tick_bits) {
  const uint64_t kLn2Q64 = 0xB17217F7D1CF79ABull;
  uint64_t m = u | 1ull;
  int c = __clzll((long long)m);
  int e = 63 - c;
  uint32_t z = (uint32_t)((m << c) >> 32);
  uint32_t frac = 0;
#pragma unroll 8
  for (int i = 0; i < 32; ++i) {
    uint64_t q = (uint64_t)z * (uint64_t)z;
    uint32_t bit = (uint32_t)(q >> 63);
    frac = (frac << 1) | bit;
    z = (uint32_t)(q >> (31 + bit));
  }
  uint64_t lq = ((uint64_t)(64 - e) << 32) - (uint64_t)frac;
  uint64_t lo = lq * kLn2Q64, hi = __umul64hi(lq, kLn2Q64);
  int sh = 96 - (kRateBits + tick_bits);  // 40 .. 64
  return sh >= 64 ? (hi >> (sh - 64)) : ((hi << (64 - sh)) | (lo >> sh));
}

// The 64 pairs (E_j, V_j), j = j0 + lane, of subdomain d.
__device__ __forceinline__ void draw_chunk(uint32_t k0, uint32_t k1, uint64_t j0, uint32_t d,
                                           int lane, int tick_bits, uint64_t& E, uint64_t& V) {
  uint64_t j = j0 + (uint64_t)lane;
  uint32_t c0 = (uint32_t)j, c1 = (uint32_t)(j >> 32), c2 = d, c3 = 0;
  philox4x32_10(k0, k1, c0, c1, c2, c3);
  V = (uint64_t)c2 | ((uint64_t)c3 << 32);
  E = neglog_fixed((uint64_t)c0 | ((uint64_t)c1 << 32), tick_bits);
}

// ------------------------------------------------------------ integer time
// floor(n / d) and ceil(n / d) for d >= 1, exact when the quotient is below
// 2^50: a double estimate from the hardware reciprocal refined by one Newton
// step (no IEEE division sequence), then exact integer correction.  Larger
// quotients are reported as 2^50, which callers treat as "beyond any
// horizon" (horizons are below 2^46 ticks, so an estimate near that bound
// that lands on either side gives the same behaviour).
__device__ __forceinline__ uint64_t udiv_floor(uint64_t n, uint64_t d, uint64_t* rem_nonzero) {
  const double dd = (double)d;
  double r = __builtin_amdgcn_rcp(dd);
  r = __builtin_fma(r, __builtin_fma(-dd, r, 1.0), r);
  const double qd = (double)n * r;
  if (qd >= 1125899906842624.0) { *rem_nonzero = 1; return 1ull << 50; }
  uint64_t q = (uint64_t)qd;
  uint64_t p = q * d;
  while (p > n) { q -= 1; p -= d; }
  while (n - p >= d) { q += 1; p += d; }
  *rem_nonzero = (n != p);
  return q;
}

// floor(n / d) for a quotient below 2^20 (the index of a site inside its
// class): a single-precision estimate, then exact integer correction.
__device__ __forceinline__ uint32_t udiv_small(uint64_t n, uint32_t d) {
  float qf = (float)n * __builtin_amdgcn_rcpf((float)d);
  uint32_t q = (uint32_t)qf;
  uint64_t p = (uint64_t)q * d;
  while (p > n) { q -= 1; p -= d; }
  while (n - p >= d) { q += 1; p += d; }
  return q;
}

// Tick of the pending event: anchor + max(1, ceil((E - acc) / lam)), or never
// when lam = 0 (eq. nextau, and eq. lambdataua after a break point).
__device__ __forceinline__ int64_t next_tick(int64_t anchor, uint64_t E, uint64_t acc, uint64_t lam) {
  if (lam == 0) return kTickInf;
  uint64_t nz;
  uint64_t q = udiv_floor(E - acc, lam, &nz);
  if (q >= (1ull << 50)) return kTickInf;
  q += nz;
  if (q < 1) q = 1;
  return anchor + (int64_t)q;
}

// ------------------------------------------------------------ lists
// The four neighbour lists of a subdomain are merged, once per run, into one
// stream sorted by (tick, edge) in LDS; an entry is tick << 18 | edge << 16 |
// position.  The event loop reads it through a 64-entry register window.
constexpr int kKeyShift = 18;

// Number of keys < k in the sorted LDS array a[0, n).
__device__ __forceinline__ int lds_lower_bound(const uint64_t* a, int n, uint64_t k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct Merged {
  const uint64_t* m;   // LDS
  int n, head;
  uint64_t chunk;
  int64_t ht;          // tick of the head entry, kTickInf when exhausted
};
// KS: bits below the tick in a key (18 in 2D: edge << 16 | position; 9 in
// 3D: face << 6 | position)
template <int KS = kKeyShift>
__device__ __forceinline__ void merged_open(Merged& s, const uint64_t* m, int n, int head, int lane) {
  s.m = m; s.n = n; s.head = head;
  int b = head & ~63;
  s.chunk = (b + lane < n) ? m[b + lane] : ~0ull;
  s.ht = head < n ? (int64_t)(rdl64(s.chunk, head & 63) >> KS) : kTickInf;
}
template <int KS = kKeyShift>
__device__ __forceinline__ uint64_t merged_pop(Merged& s, int lane) {
  uint64_t e = rdl64(s.chunk, s.head & 63);
  s.head++;
  if (s.head >= s.n) {
    s.ht = kTickInf;
  } else {
    if ((s.head & 63) == 0) s.chunk = (s.head + lane < s.n) ? s.m[s.head + lane] : ~0ull;
    s.ht = (int64_t)(rdl64(s.chunk, s.head & 63) >> KS);
  }
  return e;
}

// First tick at which the own list of this run (`cur`, n entries) differs
// from the previous iteration's (`prev`, np entries); both agree on their
// first n0 entries.  kTickInf if equal.  Both lists are in this wave's LDS.
__device__ __forceinline__ int64_t first_change(const uint64_t* cur, int n, const uint64_t* prev, int np,
                                                int n0, int lane) {
  const int m = n < np ? n : np;
  for (int b = n0 & ~63; b < m; b += 64) {
    int i = b + lane;
    bool diff = false;
    uint64_t x = 0, y = 0;
    if (i >= n0 && i < m) {
      x = cur[i];
      y = prev[i];
      diff = x != y;
    }
    uint64_t dm = ballot(diff);
    if (dm) {
      int f = ctz64(dm);
      uint64_t xf = rdl64(x, f), yf = rdl64(y, f);
      int64_t tx = (int64_t)(xf >> kPosBits), ty = (int64_t)(yf >> kPosBits);
      return tx < ty ? tx : ty;
    }
  }
  if (n == np) return kTickInf;
  // one list is a prefix of the other: the first extra entry
  const uint64_t e = n > np ? cur[m] : prev[m];
  return (int64_t)(e >> kPosBits);
}

// SplitMix64 finaliser (Steele, Lea & Flood 2014) for event digests.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, off, 64);
    uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), off, 64);
    x += ((uint64_t)hi << 32) | lo;
  }
  return x;
}

}  // namespace sr
