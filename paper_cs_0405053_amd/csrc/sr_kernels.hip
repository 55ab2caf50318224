// sr_kernels.hip -- gfx950 kernels of the synchronous-relaxation library.
//
// One 64-lane wavefront plays one of the paper's PEs: it owns one bx x by
// subdomain and, in one launch, produces that subdomain's history over the
// current window [t_c, t_end) (Sec. 4 box, step (a); Sec. 5).  The kernel
// boundary is the "synchronize" of steps (b)/(d); step (c) is done by every
// wave comparing its own new boundary lists with the ones it produced in the
// previous iteration (the neighbours' assumptions) and raising a change flag.
//
// Per-wave state lives in registers:
//   * classes of the owned sites as 4-bit nibbles, lane l owning the S
//     local sites l, l + 64, ..., l + 64(S-1) (row-major index) in nibbles
//     0..S-1, so the members of a class in ascending local order (Sec. 3
//     "linear order" of a class) are the set bits of the S per-nibble ballots
//     taken in turn;
//   * class counts N_k and rates r_k in lanes 0..9, the cumulative weights
//     C_k = sum_{i<=k} N_i r_i by a 16-lane DPP scan (eqs. biglambda, Wsum);
//   * the halo spins as four 64-bit masks;
//   * 64 presimulated (E, V) pairs, one per lane (Philox-4x32-10 + a fixed-point
//     -ln), refilled every 64 events (the "presimulated list" of Sec. 4);
//   * 64-entry chunks of the four neighbour boundary lists (break points of
//     Sec. 5), of the four own lists of the previous iteration (for the
//     comparison) and of the lists / event log being written (flushed with
//     coalesced stores).
// Nothing on the event chain touches HBM except chunk refills and flushes.
#include <vector>

#include "sr_device.h"

namespace sr {

// LDS bytes one relaxation wave needs: the halo tile, or the lists
// (whichever is larger): the four raw neighbour lists (reused for the own
// lists of the run once merged), the merged stream, and the four own lists of
// the previous iteration, up to hcap entries each.
// Bytes of the committed block each lane loads per round (all in flight).
constexpr int kTileStage = 8;

__host__ __device__ inline size_t relax_lds_bytes(int bx, int by, int hcap) {
  size_t tile = (size_t)(bx + 2) * (by + 2);
  size_t lists = (size_t)3 * 4 * hcap * sizeof(uint64_t);
  size_t b = tile > lists ? tile : lists;
  return (b + 15) & ~(size_t)15;
}

// Per-lattice descriptors are read through the constant address space: they
// do not change while the kernel runs, so the compiler may keep their fields
// in scalar registers or reload them instead of pinning ~100 values.
typedef const __attribute__((address_space(4))) Lattice CLattice;

// ------------------------------------------------------------ relaxation
// One subdomain (this wave) over one window, one iteration (Sec. 4 box, step
// (a) for one PE; Sec. 5 for the Ising specifics).
// log2 of the sites per lane of a bx x by block (a power of two).
constexpr int lane_shift(int nblk) {
  int sh = 0;
  while ((1 << sh) * 64 < nblk) sh++;
  return sh;
}

// BX, BY > 0: the block shape is a compile-time constant (the common shapes
// get their own instantiation: fewer live scalar registers and constant
// index arithmetic); 0: read from the lattice.  NW: the lattice has at least
// two subdomains in each direction, so no block wraps onto itself (the wrap
// selects on neighbour indices and edge pushes drop out at compile time).
// A store of a run's results.  COH: device-coherent (written through to the
// point where every XCD's reads meet, so the task publishes by waiting for
// its stores, with no L2 write-back); else an ordinary store (the plain
// kernels publish at the kernel boundary).
// A load of data other waves wrote in this launch.  COH: device-coherent
// (past this CU's L1, at the point device-coherent stores reach), so no
// acquire is needed before it; else an ordinary load.
template <bool COH, class T>
__device__ __forceinline__ T gget(const T* p) {
  if constexpr (COH) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    return *p;
  }
}

template <bool COH, class T, class U>
__device__ __forceinline__ void gput(T* p, U v) {
  if constexpr (COH) {
    __hip_atomic_store(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = (T)v;
  }
}

// COH: every store of the run's results is device-coherent (see gput).
template <int BX, int BY, bool NW = false, bool COH = false, class LT>
__device__ __forceinline__ void relax_subdomain(const LT& L, const Step& st, int d,
                                                int8_t* lds, IterFlags* fl) {
  static_assert((BX == 0) == (BY == 0), "both or neither block sides fixed");
  // the lane index, opaque to the compiler: per-lane offsets are then
  // computed in each run, not hoisted out of the persistent kernel's task
  // loop and kept in spilled registers
  int lane = lane_id();
  __asm__ volatile("" : "+v"(lane));
  lane &= 63;                            // (its range, for the compiler)
  const int bx = BX ? BX : L.bx, by = BY ? BY : L.by;
  const int sh = BX ? lane_shift(BX * BY) : L.sshift, S = 1 << sh;
  const int nbx = L.nbx, nby = L.nby;
  const int cx = d % nbx, cy = d / nbx;
  const int x0 = cx * bx, y0 = cy * by;
  const int nblk = bx * by;
  const bool wrapx = !NW && (nbx == 1), wrapy = !NW && (nby == 1);
  const bool first = (st.it == 0);
  const int hcap = L.hcap;
  const int dn = ((cy + nby - 1) % nby) * nbx + cx;
  const int ds = ((cy + 1) % nby) * nbx + cx;
  const int dw = cy * nbx + (cx + nbx - 1) % nbx;
  const int de = cy * nbx + (cx + 1) % nbx;
  const uint8_t* slot_prev = slot_at(L, (st.it + 1) & 1);
  const uint8_t* chg_prev = chg_at(L, (st.it + 1) & 1);
  const Carry* cin = &carry_at(L, st.wp)[d];
  const uint32_t k0 = L.seed_lo, k1 = L.seed_hi;
  auto clampn = [&](uint32_t n) { return (int)(n < (uint32_t)hcap ? n : (uint32_t)hcap); };

  uint32_t rate = 0;
#pragma unroll
  for (int k = 0; k < kClasses; ++k)
    if (lane == k) rate = L.rate[k];

  // ---- setup loads in three dependent rounds, each a gather with one lane
  // per value (a run then waits for three memory round trips, not one per
  // value): (1) the slot and change bytes of this subdomain and of its four
  // neighbours, its checkpoint count and ticks, its carry and work counters;
  // (2) the facing lists' first-change ticks and lengths and its own lists'
  // lengths, which pick the checkpoint to resume from (the latest one whose
  // state only depends on input entries that did not change); (3) that
  // checkpoint or the committed block, and the list entries.
  // facing list q (0..3) is the list of neighbour dn, ds, dw, de on its
  // edge kS, kN, kE, kW
  const bool none[4] = {first || wrapy, first || wrapy, first || wrapx, first || wrapx};
  const Ckpt* cks = L.ck + (size_t)d * L.nck;
  uint32_t g8 = 0;                         // lane 0: own slot; 1..4: facing slots; 5..8: their change masks
  uint32_t nck_v = 0;
  uint64_t ckt = 0, ckv = 0;               // lane k < nck: tick and window event count of checkpoint k
  if (!first) {
    const int ql = (lane - 1) & 3;
    const int el = lane == 0 ? d : ql == 0 ? dn : ql == 1 ? ds : ql == 2 ? dw : de;
    if (lane < 9) g8 = gget<COH>((lane < 5 ? slot_prev : chg_prev) + el);
    nck_v = gget<COH>(&L.ckn[d]);
    if (lane < L.nck) {
      ckt = gget<COH>(&cks[lane].meta[kCkT]);
      ckv = gget<COH>(&cks[lane].meta[kCkNev]);
    }
  }
  // lanes 0..4: j, anchor, acc, digest, flips of the committed carry; 5: the
  // largest boundary-event count of this window's earlier runs; 6, 7: work
  // counters
  uint64_t cv = 0;
  if (lane < 8 && (lane != 5 || !first)) {
    const uint64_t* cp = lane < 5 ? reinterpret_cast<const uint64_t*>(cin) + lane
                         : lane == 5 ? reinterpret_cast<const uint64_t*>(&carry_at(L, st.wp ^ 1)[d].nbmax)
                                     : reinterpret_cast<const uint64_t*>(&L.stat[d]) + (lane - 6);
    cv = gget<COH>(cp);
  }

  int sprev = 0, sl[4] = {0, 0, 0, 0}, ni[4] = {0, 0, 0, 0}, np[4] = {0, 0, 0, 0};
  int ck = -1;
  if (!first) {
    sprev = (int)rdl(g8, 0);
    uint32_t cm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sl[q] = none[q] ? 0 : (int)rdl(g8, 1 + q);
      cm[q] = rdl(g8, 5 + q);
    }
    // lanes 0..3: facing list q's first-change tick (if it changed) and
    // length; lanes 4..7: own list e's length in the previous run
    const int ql = lane & 3;
    const int eq = ql == 0 ? dn : ql == 1 ? ds : ql == 2 ? dw : de;
    const int edq = ql == 0 ? kS : ql == 1 ? kN : ql == 2 ? kE : kW;
    const int slq = ql == 0 ? sl[0] : ql == 1 ? sl[1] : ql == 2 ? sl[2] : sl[3];
    const uint32_t cmq = ql == 0 ? cm[0] : ql == 1 ? cm[1] : ql == 2 ? cm[2] : cm[3];
    const bool nq = ql < 2 ? wrapy : wrapx;
    uint64_t f = (uint64_t)kTickInf;
    uint32_t hc = 0;
    if (lane < 4) {
      if (!nq) {
        if ((cmq >> edq) & 1u) f = (uint64_t)gget<COH>(&fct_at(L, slq)[eq * kEdges + edq]);
        hc = gget<COH>(&hcnt_at(L, slq)[eq * kEdges + edq]);
      }
    } else if (lane < 8) {
      hc = gget<COH>(&hcnt_at(L, sprev)[d * kEdges + (lane - 4)]);
    }
    int64_t tau = kTickInf;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t fq = (int64_t)rdl64(f, q);
      tau = fq < tau ? fq : tau;
      ni[q] = clampn(rdl(hc, q));
      np[q] = clampn(rdl(hc, 4 + q));
    }
    const uint64_t m = ballot(lane < (int)nck_v && (int64_t)ckt <= tau);
    if (m) ck = 63 - __builtin_clzll(m);
  }
  const int sout = first ? 0 : 1 - sprev;

  // neighbour histories of the previous iteration (break points), each in
  // the slot its owner last wrote, and this subdomain's own lists of its
  // previous run; the first iteration assumes none (canonical assumption).
  // The first 64 entries of each concatenation are gathered now, beside the
  // checkpoint or block loads, and go to LDS once the tile's LDS is free.
  const int o1 = ni[0], o2 = o1 + ni[1], o3 = o2 + ni[2], tot = o3 + ni[3];
  const int p1 = np[0], p2 = p1 + np[1], p3 = p2 + np[2], totp = p3 + np[3];
  const uint64_t* pb = hist_at(L, sprev) + (size_t)d * kEdges * hcap;
  auto nb_src = [&](int i, int& q, int& k) -> const uint64_t* {
    q = i < o1 ? 0 : i < o2 ? 1 : i < o3 ? 2 : 3;
    k = i - (q == 0 ? 0 : q == 1 ? o1 : q == 2 ? o2 : o3);
    const int e = q == 0 ? dn : q == 1 ? ds : q == 2 ? dw : de;
    const int eg = q == 0 ? kS : q == 1 ? kN : q == 2 ? kE : kW;
    const int s = q == 0 ? sl[0] : q == 1 ? sl[1] : q == 2 ? sl[2] : sl[3];
    return hist_at(L, s) + ((size_t)e * kEdges + eg) * hcap + k;
  };
  auto own_at = [&](int i) -> int {       // offset of own entry i in the per-edge layout
    const int e = i < p1 ? 0 : i < p2 ? 1 : i < p3 ? 2 : 3;
    return e * hcap + i - (e == 0 ? 0 : e == 1 ? p1 : e == 2 ? p2 : p3);
  };
  uint64_t xn = 0, xo = 0;
  if (lane < tot) { int q, k; xn = gget<COH>(nb_src(lane, q, k)); }
  if (lane < totp) xo = gget<COH>(&pb[own_at(lane)]);

  uint64_t cls, hN, hS, hW, hE, j, acc, dtot;
  uint32_t ncnt;
  int64_t anchor;
  int nev, nbound, n0[4], h0;
  uint64_t lbuf = 0;                       // window log entries of the unfinished 64-chunk
  uint64_t* wl = L.wlog + (size_t)d * L.wcap;
  const int wcap = L.wcap;
  if (ck >= 0) {
    const Ckpt* c = cks + ck;
    cls = gget<COH>(&c->cls[lane]);
    const uint64_t mw = lane < kCkWords ? gget<COH>(&c->meta[lane]) : 0ull;
    {
      const int nv = (int)rdl64(ckv, ck) & ~63;
      const int nevc = (int)(uint32_t)rdl64(ckv, ck);
      if (nv + lane < nevc && nv + lane < wcap) lbuf = gget<COH>(&wl[nv + lane]);
    }
    const uint64_t pair = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(mw >> 32), lane >> 1, 64) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)mw, lane >> 1, 64);
    ncnt = lane < kClasses ? (uint32_t)(pair >> (32 * (lane & 1))) : 0u;
    hN = rdl64(mw, kCkHalo + 0); hS = rdl64(mw, kCkHalo + 1);
    hW = rdl64(mw, kCkHalo + 2); hE = rdl64(mw, kCkHalo + 3);
    j = rdl64(mw, kCkJ); acc = rdl64(mw, kCkAcc); anchor = (int64_t)rdl64(mw, kCkAnchor);
    dtot = rdl64(mw, kCkDsum);
    nev = (int)rdl(mw, kCkNev); nbound = (int)rdl((uint32_t)(mw >> 32), kCkNev);
    n0[0] = (int)rdl(mw, kCkOut01); n0[1] = (int)rdl((uint32_t)(mw >> 32), kCkOut01);
    n0[2] = (int)rdl(mw, kCkOut23); n0[3] = (int)rdl((uint32_t)(mw >> 32), kCkOut23);
    h0 = (int)rdl(mw, kCkHead);
  } else {
    // committed block + one-site halo -> LDS (internal wrap falls out of the
    // periodic global index when the block spans the torus), loaded in
    // stages of kTileStage bytes per lane, all in flight together
    int8_t* tile = lds;
    const int8_t* sp = spins_at(L, st.wp);
    const int tw = bx + 2, ntile = (by + 2) * tw;
    const int ln = lane;
    for (int b0 = 0; b0 < ntile; b0 += 64 * kTileStage) {
      int8_t tv[kTileStage];
#pragma unroll
      for (int k = 0; k < kTileStage; ++k) {
        const int i = b0 + 64 * k + ln;
        tv[k] = 0;
        if (i < ntile) {
          const int ty = i / tw, tx = i - ty * tw;
          int gy = y0 + ty - 1, gx = x0 + tx - 1;
          gy = gy < 0 ? gy + L.Ly : (gy >= L.Ly ? gy - L.Ly : gy);
          gx = gx < 0 ? gx + L.Lx : (gx >= L.Lx ? gx - L.Lx : gx);
          tv[k] = gget<COH>(&sp[(int64_t)gy * L.Lx + gx]);
        }
      }
#pragma unroll
      for (int k = 0; k < kTileStage; ++k) {
        const int i = b0 + 64 * k + ln;
        if (i < ntile) tile[i] = tv[k];
      }
    }
    __syncthreads();
    // classes of owned sites, 4 bits each; unused nibbles hold 0xF
    cls = ~0ull;
    for (int i = 0; i < S; ++i) {
      int v = lane + 64 * i;
      if (v < nblk) {
        int ly = v / bx, lx = v - ly * bx;
        int tp = (ly + 1) * tw + lx + 1;
        int up = (tile[tp - 1] > 0) + (tile[tp + 1] > 0) + (tile[tp - tw] > 0) + (tile[tp + tw] > 0);
        int k = (tile[tp] < 0 ? 5 : 0) + up;
        cls = (cls & ~(0xFull << (4 * i))) | ((uint64_t)k << (4 * i));
      }
    }
    // halo spins (bit p set = up) of the four external directions
    hN = ballot(lane < bx && tile[lane + 1] > 0);
    hS = ballot(lane < bx && tile[(by + 1) * tw + lane + 1] > 0);
    hW = ballot(lane < by && tile[(lane + 1) * tw] > 0);
    hE = ballot(lane < by && tile[(lane + 1) * tw + bx + 1] > 0);
    // class counts N_k in lane k: each lane counts its own sites per class
    // in 12-bit fields (at most 1024 sites in a block), classes 0..4 in one
    // word and 5..9 in another, and two wave sums add the lanes up (unused
    // nibbles hold 0xF and count nowhere)
    {
      uint64_t p0 = 0, p1 = 0;
      for (int i = 0; i < S; ++i) {
        const uint32_t k = (uint32_t)(cls >> (4 * i)) & 15u;
        p0 += k < 5 ? 1ull << (12 * k) : 0ull;
        p1 += k - 5u < 5u ? 1ull << (12 * (k - 5u)) : 0ull;
      }
      p0 = wave_sum64(p0);
      p1 = wave_sum64(p1);
      const uint64_t pk = lane < 5 ? p0 >> (12 * lane) : p1 >> (12 * (lane - 5));
      ncnt = lane < kClasses ? (uint32_t)(pk & 0xFFF) : 0u;
    }
    j = rdl64(cv, 0); anchor = (int64_t)rdl64(cv, 1); acc = rdl64(cv, 2); dtot = 0;
    if (L.wipe && st.t_c > 0) {
      // wipe the slate (Sec. 5): the pending pair is dropped, the next one
      // starts its hazard at the window start
      j += 1; acc = 0; anchor = st.t_c;
    }
    nev = 0; nbound = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) n0[e] = 0;
    h0 = 0;
    __syncthreads();                     // the tile's LDS is reused below
  }
  const int nev0 = nev;

  // ---- the list entries to LDS: the facing lists merged into one stream
  // (break points), this subdomain's previous lists beside them (the
  // end-of-run comparison then reads no global memory: a load there would
  // wait for every store the run issued)
  uint64_t* raw = reinterpret_cast<uint64_t*>(lds);
  uint64_t* mrg = raw + 4 * hcap;
  uint64_t* lprev = raw + 8 * hcap;
  uint64_t* lcur = raw;                  // own lists of this run, once merged
  auto nb_key = [&](uint64_t x, int q) {
    return ((x >> kPosBits) << kKeyShift) | ((uint64_t)q << 16) | (x & 0xFFFF);
  };
  if (lane < tot) { int q, k; nb_src(lane, q, k); raw[lane] = nb_key(xn, q); }
  if (lane < totp) lprev[own_at(lane)] = xo;
  for (int i = 64 + lane; i < tot; i += 64) { int q, k; const uint64_t x = gget<COH>(nb_src(i, q, k)); raw[i] = nb_key(x, q); }
  for (int i = 64 + lane; i < totp; i += 64) lprev[own_at(i)] = gget<COH>(&pb[own_at(i)]);
  // committed digest and flip count of this subdomain, needed at the end;
  // the largest boundary-event count of its earlier runs in this window
  const uint64_t dig_in = rdl64(cv, 3);
  const int64_t flips_in = (int64_t)rdl64(cv, 4);
  const int64_t nbmax_in = first ? 0 : (int64_t)rdl64(cv, 5);
  const unsigned long long ev_in = rdl64(cv, 6), runs_in = rdl64(cv, 7);
  __syncthreads();
  if (tot > 0) {
    for (int i = lane; i < tot; i += 64) {
      const int q = i < o1 ? 0 : i < o2 ? 1 : i < o3 ? 2 : 3;
      const int oq = q == 0 ? 0 : q == 1 ? o1 : q == 2 ? o2 : o3;
      const uint64_t key = raw[i];
      int rank = i - oq;
      if (q != 0) rank += lds_lower_bound(raw, ni[0], key);
      if (q != 1) rank += lds_lower_bound(raw + o1, ni[1], key);
      if (q != 2) rank += lds_lower_bound(raw + o2, ni[2], key);
      if (q != 3) rank += lds_lower_bound(raw + o3, ni[3], key);
      mrg[rank] = key;
    }
    __syncthreads();
  }
  Merged in;
  merged_open(in, mrg, tot, h0, lane);

  // ---- own lists of this iteration, built in LDS (when resuming, the
  // previous version's first n0 entries, which the same inputs reproduce)
  // and stored to the other slot at the end of the run
  uint64_t* ob = hist_at(L, sout) + (size_t)d * kEdges * hcap;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    for (int i = lane; i < n0[e]; i += 64) lcur[e * hcap + i] = lprev[e * hcap + i];
  int nN = n0[0], nS = n0[1], nW = n0[2], nE = n0[3];
  auto push = [&](int e, int& n, uint64_t x) {
    if (lane == 0 && n < hcap) lcur[e * hcap + n] = x;
    n++;
  };

  // presimulated randoms of the current 64-chunk
  uint64_t Eb, Vb;
  draw_chunk(k0, k1, j & ~63ull, (uint32_t)d, lane, L.tick_bits, Eb, Vb);
  uint64_t E = rdl64(Eb, (int)(j & 63)), V = rdl64(Vb, (int)(j & 63));
  uint64_t C = row_incl_scan64((uint64_t)ncnt * rate);
  uint64_t lam = rdl64(C, kClasses - 1);
  int64_t next = next_tick(anchor, E, acc, lam);

  // window event log (tick << 16 | local site), buffered 64 at a time
  auto log_flush = [&](int k) {          // k buffered entries in lanes 0..k-1
    int at = nev - k + lane;
    uint64_t dsum = 0;
    if (lane < k) {
      if (at < wcap) gput<COH>(&wl[at], lbuf);
      int v = (int)(lbuf & 0xFFFF);
      int ly = v / bx, lx = v - ly * bx;
      int64_t g = (int64_t)(y0 + ly) * L.Lx + x0 + lx;
      dsum = mix64(mix64(lbuf >> kPosBits) + (uint64_t)g);
    }
    dtot += wave_sum64(dsum);
  };

  // move site u (local) by `delta` classes
  auto change = [&](int u, int delta) {
    int o = u & 63, sl = (u >> 6) * 4;
    uint64_t w = rdl64(cls, o);
    int a = (int)((w >> sl) & 15);
    int b = a + delta;
    if (lane == o) cls += (uint64_t)(int64_t)delta * (1ull << sl);
    ncnt += (uint32_t)((lane == b) - (lane == a));
  };

  const int64_t t_end = st.t_end;
  // hard bound on the loop: a window log far beyond its capacity means the
  // window is re-run with more room anyway
  const int nev_limit = 4 * wcap + 64;
  bool runaway = false;
  Ckpt* ckbase = L.ck + (size_t)d * L.nck;
  int ckc = ck + 1;                      // next checkpoint slot
  int since = 0;                         // items since the last checkpoint
  int64_t last_t = -1;                   // tick of the last processed item
  for (;;) {
    if (nev >= nev_limit) { runaway = true; break; }
    const int64_t tb = in.ht;
    const int64_t tn = min64(next, tb);
    if (tn >= t_end) break;
    if (since >= L.ckint && ckc < L.nck && tn > last_t) {
      // state after every item with tick < tn: a place to resume from
      Ckpt* c = ckbase + ckc;
      gput<COH>(&c->cls[lane], cls);
      // metadata word `lane` (dsum: the log entries flushed so far)
      const uint32_t clo = (uint32_t)__shfl((int)ncnt, (2 * lane) & 63, 64);
      const uint32_t chi = (uint32_t)__shfl((int)ncnt, (2 * lane + 1) & 63, 64);
      uint64_t w = (uint64_t)clo | ((uint64_t)chi << 32);
      // the scalar words go in with lane writes (no per-lane selects, so no
      // lane masks kept live across the event loop)
      w = wrl64<kCkT>(w, (uint64_t)tn);
      w = wrl64<kCkJ>(w, j);
      w = wrl64<kCkAcc>(w, acc);
      w = wrl64<kCkAnchor>(w, (uint64_t)anchor);
      w = wrl64<kCkHalo + 0>(w, hN);
      w = wrl64<kCkHalo + 1>(w, hS);
      w = wrl64<kCkHalo + 2>(w, hW);
      w = wrl64<kCkHalo + 3>(w, hE);
      w = wrl64<kCkDsum>(w, dtot);
      w = wrl64<kCkNev>(w, (uint64_t)(uint32_t)nev | ((uint64_t)(uint32_t)nbound << 32));
      w = wrl64<kCkOut01>(w, (uint64_t)(uint32_t)nN | ((uint64_t)(uint32_t)nS << 32));
      w = wrl64<kCkOut23>(w, (uint64_t)(uint32_t)nW | ((uint64_t)(uint32_t)nE << 32));
      w = wrl64<kCkHead>(w, (uint64_t)(uint32_t)in.head);
      if (lane < 32) gput<COH>(&c->meta[lane], lane < kCkWords ? w : 0ull);
      ckc++;
      since = 0;
    }
    since++;
    if (next <= tb) {
      // ---- own event (first on a tie: it chooses from the pre-tick state)
      const int64_t t = next;
      last_t = t;
      // class: first k with C_k > target (eqs. Wsum, Wstop)
      uint64_t target = __umul64hi(V, lam);
      // lanes kClasses..15 hold C = lam and higher rows 0: mask the ballot
      uint64_t gt = ballot(C > target) & ((1ull << kClasses) - 1);
      int ks = ctz64(gt);
      uint64_t below = ks ? rdl64(C, ks - 1) : 0ull;
      uint32_t rk = rdl(rate, ks);
      // uniform: kept on the scalar unit for the comparisons below
      const uint32_t idx = (uint32_t)__builtin_amdgcn_readfirstlane((int)udiv_small(target - below, rk));
      // site: the idx-th member of class ks in ascending local order
      // (eqs. nores, vindex).  Members in nibble i are the set bits of
      // ballot i; the nibble holding member idx is the last one whose count
      // of members in lower nibbles is <= idx (scalar unit), the lane the
      // one with exactly that many fewer members in the lanes below it.
      uint64_t msel = 0;
      uint32_t seen = 0, before = 0;
      int isel = 0;
      for (int i = 0; i < S; ++i) {
        const uint64_t m = ballot(((uint32_t)(cls >> (4 * i)) & 15u) == (uint32_t)ks);
        const bool here = idx >= seen;
        msel = here ? m : msel;
        isel = here ? i : isel;
        before = here ? seen : before;
        seen += (uint32_t)__popcll(m);
      }
      const uint32_t nth = idx - before;
      const uint32_t nlow = __builtin_amdgcn_mbcnt_hi((uint32_t)(msel >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)msel, 0u));
      const int v = isel * 64 + ctz64(ballot(nlow == nth) & msel);
      // flip v and re-class it and its in-block neighbours (Sec. 3, O(1))
      const int ly = v / bx, lx = v - ly * bx;
      const int kv = (int)((rdl64(cls, v & 63) >> ((v >> 6) * 4)) & 15);
      const bool now_up = kv >= 5;
      const int dup = now_up ? 1 : -1;
      if constexpr (BX == 16 && BY == 16 && NW) {
        // 16x16 block, no wrap: the five sites sit in five different lanes
        // (their index differences 1, 2, 15, 16, 17, 32 are never multiples
        // of 64), so each class word is read, moved on the scalar unit and
        // written back to its lane
        const int dv = now_up ? -5 : 5;
        uint32_t inc = (uint32_t)(lane == kv + dv), dec = (uint32_t)(lane == kv);
        cls = wrl64_at(cls, rdl64(cls, v & 63) + ((uint64_t)(int64_t)dv << ((v >> 6) * 4)), v & 63);
        const int nbr[4] = {lx > 0 ? v - 1 : -1, lx < 15 ? v + 1 : -1, ly > 0 ? v - 16 : -1,
                            ly < 15 ? v + 16 : -1};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = nbr[q];
          if (u < 0) continue;
          const int o = u & 63, sl = (u >> 6) * 4;
          const uint64_t w = rdl64(cls, o);
          const int a = (int)((w >> sl) & 15);
          cls = wrl64_at(cls, w + ((uint64_t)(int64_t)dup << sl), o);
          inc += (uint32_t)(lane == a + dup);
          dec += (uint32_t)(lane == a);
        }
        ncnt += inc - dec;
      } else if ((bx >= 3 || !wrapx) && (by >= 3 || !wrapy)) {
        // the flipped site and its in-block neighbours are five distinct
        // sites: read every old class from the words before the flip and
        // apply all the moves at once (no chain through the class words)
        const int nbr[4] = {lx > 0 ? v - 1 : (wrapx ? v + bx - 1 : -1),
                            lx < bx - 1 ? v + 1 : (wrapx ? v - bx + 1 : -1),
                            ly > 0 ? v - bx : (wrapy ? v + (by - 1) * bx : -1),
                            ly < by - 1 ? v + bx : (wrapy ? v - (by - 1) * bx : -1)};
        const int dv = now_up ? -5 : 5;
        uint64_t add = lane == (v & 63) ? (uint64_t)(int64_t)dv << ((v >> 6) * 4) : 0ull;
        uint32_t inc = (uint32_t)(lane == kv + dv), dec = (uint32_t)(lane == kv);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = nbr[q];
          if (u < 0) continue;
          const int o = u & 63, sl = (u >> 6) * 4;
          const int a = (int)((rdl64(cls, o) >> sl) & 15);
          add += lane == o ? (uint64_t)(int64_t)dup << sl : 0ull;
          inc += (uint32_t)(lane == a + dup);
          dec += (uint32_t)(lane == a);
        }
        cls += add;
        ncnt += inc - dec;
      } else {
        // a 2-wide block wrapping onto itself: both horizontal (or vertical)
        // neighbours are the same site, so the moves must chain
        change(v, now_up ? -5 : 5);
        if (lx > 0) change(v - 1, dup); else if (wrapx) change(v + bx - 1, dup);
        if (lx < bx - 1) change(v + 1, dup); else if (wrapx) change(v - bx + 1, dup);
        if (ly > 0) change(v - bx, dup); else if (wrapy) change(v + (by - 1) * bx, dup);
        if (ly < by - 1) change(v + bx, dup); else if (wrapy) change(v - (by - 1) * bx, dup);
      }
      // record
      const uint64_t tk = (uint64_t)t << kPosBits;
      if (lane == (nev & 63)) lbuf = tk | (uint64_t)v;
      nev++;
      if ((nev & 63) == 0) log_flush(64);
      bool onb = false;
      if (!wrapy && ly == 0) { push(kN, nN, tk | (uint64_t)lx); onb = true; }
      if (!wrapy && ly == by - 1) { push(kS, nS, tk | (uint64_t)lx); onb = true; }
      if (!wrapx && lx == 0) { push(kW, nW, tk | (uint64_t)ly); onb = true; }
      if (!wrapx && lx == bx - 1) { push(kE, nE, tk | (uint64_t)ly); onb = true; }
      nbound += onb;
      // next pair from the presimulated list
      j += 1; anchor = t; acc = 0;
      if ((j & 63) == 0) draw_chunk(k0, k1, j, (uint32_t)d, lane, L.tick_bits, Eb, Vb);
      E = rdl64(Eb, (int)(j & 63)); V = rdl64(Vb, (int)(j & 63));
      C = row_incl_scan64((uint64_t)ncnt * rate);
      lam = rdl64(C, kClasses - 1);
      next = next_tick(anchor, E, acc, lam);
    } else {
      // ---- break point: a neighbour flip changes our halo (Sec. 5)
      const int64_t t = tb;
      last_t = t;
      const uint64_t key = merged_pop(in, lane);
      const int q = (int)((key >> 16) & 3);
      const int p = (int)(key & 0xFFFF);
      if (q == 0) {
        hN ^= 1ull << p;
        change(p, ((hN >> p) & 1) ? 1 : -1);
      } else if (q == 1) {
        hS ^= 1ull << p;
        change((by - 1) * bx + p, ((hS >> p) & 1) ? 1 : -1);
      } else if (q == 2) {
        hW ^= 1ull << p;
        change(p * bx, ((hW >> p) & 1) ? 1 : -1);
      } else {
        hE ^= 1ull << p;
        change(p * bx + bx - 1, ((hE >> p) & 1) ? 1 : -1);
      }
      // integrate the hazard up to the break point with the old rate
      // (eqs. lambdataua, breaksum, bsubk), then re-aim with the new one
      acc += lam * (uint64_t)(t - anchor);
      anchor = t;
      C = row_incl_scan64((uint64_t)ncnt * rate);
      lam = rdl64(C, kClasses - 1);
      next = next_tick(anchor, E, acc, lam);
    }
  }
  if (nev & 63) log_flush(nev & 63);

  // end-of-window block -> working lattice (the other window parity): one
  // byte per owned site; nibble i of the 64 lanes is 64 consecutive sites
  int8_t* so = spins_at(L, st.wp ^ 1);
  for (int i = 0; i < S; ++i) {
    const int v = lane + 64 * i;
    if (v < nblk) {
      const int ly = v / bx, lx = v - ly * bx;
      gput<COH>(&so[(int64_t)(y0 + ly) * L.Lx + x0 + lx], ((cls >> (4 * i)) & 15) < 5 ? (int8_t)1 : (int8_t)-1);
    }
  }
  // compare step (c): own lists against the previous iteration's, then the
  // own lists to their slot (coalesced)
  const int nn[4] = {nN, nS, nW, nE};
  int64_t fc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int n = clampn((uint32_t)nn[e]);
    const uint64_t* cur = lcur + e * hcap;
    fc[e] = first ? (n > 0 ? (int64_t)(cur[0] >> kPosBits) : kTickInf)
                  : first_change(cur, n, lprev + e * hcap, np[e], n0[e], lane);
    for (int i = lane; i < n; i += 64) gput<COH>(&ob[e * hcap + i], cur[i]);
  }
  uint32_t* cnt_out = hcnt_at(L, sout) + d * kEdges;
  int64_t* fct_out = fct_at(L, sout) + d * kEdges;
  if (lane == 0) {
    uint32_t emask = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      gput<COH>(&cnt_out[e], (uint32_t)nn[e]);
      gput<COH>(&fct_out[e], fc[e]);
      emask |= fc[e] != kTickInf ? 1u << e : 0u;
    }
    Carry* co = &carry_at(L, st.wp ^ 1)[d];
    gput<COH>(&co->j, j); gput<COH>(&co->anchor, anchor); gput<COH>(&co->acc, acc);
    gput<COH>(&co->digest, dig_in + dtot);
    gput<COH>(&co->flips, flips_in + nev);
    gput<COH>(&co->wflips, nev);
    gput<COH>(&co->nbound, nbound);
    gput<COH>(&co->nbmax, nbound > nbmax_in ? nbound : nbmax_in);
    gput<COH>(&L.stat[d].events, ev_in + (unsigned long long)(nev - nev0));
    gput<COH>(&L.stat[d].runs, runs_in + 1ull);
    gput<COH>(&L.wcnt[d], (uint32_t)nev);
    gput<COH>(&L.ckn[d], (uint32_t)ckc);
    gput<COH>(&slot_at(L, st.it & 1)[d], (uint8_t)sout);
    gput<COH>(&chg_at(L, st.it & 1)[d], (uint8_t)emask);
    uint32_t ovf = ((nN > hcap || nS > hcap || nW > hcap || nE > hcap) ? 1u : 0u) |
                   ((nev > wcap || runaway) ? 2u : 0u);
    if (emask) gput<COH>(&fl->changed, 1u);
    if (L.need) {
      // batched form: this run consumed its own "runs now" mark; the
      // neighbour facing each changed edge runs in the next iteration
      // (plain byte stores of 0 / 1: one subdomain per byte, and the
      // fences of the batched form order them)
      gput<COH>(&need_at(L, st.it & 1)[d], (uint8_t)0);
      uint8_t* nb = need_at(L, (st.it + 1) & 1);
      const int facing[4] = {dn, ds, dw, de};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (emask & (1u << e)) gput<COH>(&nb[facing[e]], (uint8_t)1);
    }
    if (ovf & 1u) gput<COH>(&fl->ovf_hist, 1u);
    if (ovf & 2u) gput<COH>(&fl->ovf_log, 1u);
  }
}

// Does subdomain d have to run in iteration st.it (> 0)?  Only if one of its
// external neighbours' lists changed in the previous iteration: the same
// inputs give the same outputs.
template <class LT>
__device__ __forceinline__ bool inputs_changed(const LT& L, int it, int d) {
  const int nbx = L.nbx, nby = L.nby;
  const int cx = d % nbx, cy = d / nbx;
  // only the list of each neighbour's edge that faces d is an input of d
  const uint8_t* c = chg_at(L, (it + 1) & 1);
  bool need = false;
  if (nby > 1)
    need |= ((c[((cy + nby - 1) % nby) * nbx + cx] >> kS) & 1) | ((c[((cy + 1) % nby) * nbx + cx] >> kN) & 1);
  if (nbx > 1)
    need |= ((c[cy * nbx + (cx + nbx - 1) % nbx] >> kE) & 1) | ((c[cy * nbx + (cx + 1) % nbx] >> kW) & 1);
  return need;
}

template <int BX, int BY, bool NW>
__global__ __launch_bounds__(64) void relax_kernel(Lattice L, Step st) {
  extern __shared__ int8_t tile[];
  const int d = blockIdx.x;
  if (d >= L.nsub) return;
  if (st.fi > 0) {
    // queued behind an iteration that already converged (or overflowed):
    // nothing to do
    const IterFlags* fp = L.flags + st.fi - 1;
    if (fp->changed == 0 || fp->ovf_hist != 0 || fp->ovf_log != 0) return;
  }
  if (st.it > 0 && !inputs_changed(L, st.it, d)) {
    // keep the previous outputs (lists, window state, log): skip the run
    if (lane_id() == 0) {
      slot_at(L, st.it & 1)[d] = slot_at(L, (st.it + 1) & 1)[d];
      chg_at(L, st.it & 1)[d] = 0;
    }
    return;
  }
  // the descriptor is read in place from the kernel arguments (constant
  // address space), so rarely used fields need not stay in registers
  relax_subdomain<BX, BY, NW>(*(CLattice*)__builtin_amdgcn_kernarg_segment_ptr(), st, d, tile, L.flags + st.fi);
}

// Graph form of the plain iteration: the window descriptor lives in device
// memory (written by the host before each replay) and node i of the graph is
// iteration st.it + i.
template <int BX, int BY, bool NW>
__global__ __launch_bounds__(64) void relax_graph_kernel(Lattice L, const Step* stp, int i) {
  extern __shared__ int8_t tile[];
  const int d = blockIdx.x;
  if (d >= L.nsub) return;
  typedef const __attribute__((address_space(4))) Step CStep;
  CStep& cs = *(CStep*)stp;
  Step st;
  st.t_c = cs.t_c; st.t_end = cs.t_end; st.wp = cs.wp; st.it = cs.it + i; st.fi = i; st.pad = 0;
  if (i > 0) {
    const IterFlags* fp = L.flags + i - 1;
    if (fp->changed == 0 || fp->ovf_hist != 0 || fp->ovf_log != 0) return;
  }
  if (st.it > 0 && !inputs_changed(L, st.it, d)) {
    if (lane_id() == 0) {
      slot_at(L, st.it & 1)[d] = slot_at(L, (st.it + 1) & 1)[d];
      chg_at(L, st.it & 1)[d] = 0;
    }
    return;
  }
  relax_subdomain<BX, BY, NW>(*(CLattice*)__builtin_amdgcn_kernarg_segment_ptr(), st, d, tile, L.flags + i);
}

// Clears the first n iteration flags (a kernel, so that graphs hold no
// memset nodes).
__global__ void clear_flags_kernel(IterFlags* f, int n) {
  int i = threadIdx.x;
  if (i < n) {
    f[i].changed = 0; f[i].ovf_hist = 0; f[i].ovf_log = 0; f[i].pad = 0;
  }
}

// ------------------------------------------------------------ batched form

// The 128-byte per-lattice record, one 32-bit word per lane (lanes 0..31),
// fetched with one load instead of one dependent load per field.
static_assert(sizeof(LatRun) == 128, "LatRun is read as 32 words");
struct RunView {
  uint32_t w;
  __device__ __forceinline__ uint32_t u32(size_t off) const { return rdl(w, (int)(off / 4)); }
  __device__ __forceinline__ int64_t i64(size_t off) const {
    return (int64_t)(((uint64_t)rdl(w, (int)(off / 4) + 1) << 32) | rdl(w, (int)(off / 4)));
  }
};
__device__ __forceinline__ RunView load_run(const LatRun* run, int lane) {
  RunView v;
  v.w = lane < 32 ? gget<true>(&reinterpret_cast<const uint32_t*>(run)[lane]) : 0u;
  return v;
}
__device__ __forceinline__ Step step_of(const RunView& v) {
  Step st;
  st.t_c = v.i64(offsetof(LatRun, st) + offsetof(Step, t_c));
  st.t_end = v.i64(offsetof(LatRun, st) + offsetof(Step, t_end));
  st.wp = (int32_t)v.u32(offsetof(LatRun, st) + offsetof(Step, wp));
  st.it = (int32_t)v.u32(offsetof(LatRun, st) + offsetof(Step, it));
  st.fi = (int32_t)v.u32(offsetof(LatRun, st) + offsetof(Step, fi));
  st.pad = 0;
  return st;
}

// Wave-cooperative enqueue of the subdomains of lattice `lat` that run in
// iteration `it`: all of them when it == 0, else those whose facing input
// lists changed in iteration it - 1 (their "runs now" bytes).  The
// others keep their lists: the slot array is copied forward and the change
// masks cleared before anything is published.  Sets the per-shard counts
// and shards_left before publishing any task.
// Ordering between the tasks of one lattice.  Everything the batched form
// writes for other waves (a run's results, the decider's run record, slot
// and change arrays, counts) goes out with device-coherent stores, written
// through to the point where every XCD's reads meet, and everything it reads
// that other waves wrote in this launch comes in with device-coherent loads
// (past this CU's L1; the compiled kernel has no other vector load).  So
// publishing is a wait for the stores, and a task needs no acquire: its
// loads are issued after the queue slot that named the task was read, and
// that slot was written after the producer's stores completed.  (Measured
// alternatives: a device-scope release per task writes the whole L2 back and
// the L2 serialises it, over half of the batched form's time; a device-scope
// acquire per task drops the L2's copies of other XCDs' lines; the
// workgroup-scope L1 invalidate left stale L1 lines outside threadgroup-split
// mode, seen as wrong trajectories.)
__device__ __forceinline__ void publish_wait() { __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory"); }

// Device-coherent load and store of 16 bytes (two 8-byte accesses).
__device__ __forceinline__ uint4 gget16(const uint4* p) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long a = gget<true>(q), b = gget<true>(q + 1);
  return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
}
__device__ __forceinline__ void gput16(uint4* p, const uint4& v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  gput<true>(q, ((unsigned long long)v.y << 32) | v.x);
  gput<true>(q + 1, ((unsigned long long)v.w << 32) | v.z);
}

__device__ uint32_t enqueue_iteration(const BatchArgs& B, int lat, LatRun* run, CLattice& L, int it,
                                      int lane) {
  const int nsub = L.nsub;
  const int nw = (nsub + 63) / 64;              // 64 subdomains per lane and pass
  const uint8_t* nb = need_at(L, it & 1);
  // the 64 "runs now" bytes of group w as a bit mask (bytes are 0 or 1):
  // four 16-byte loads, then the gather
  auto group_mask = [&](int w) -> unsigned long long {
    if (it == 0) {
      const int left = nsub - w * 64;
      return left >= 64 ? ~0ull : ((1ull << left) - 1);
    }
    // the four 16-byte loads in flight together (one round trip on the
    // decider's path instead of four)
    const unsigned long long* p = reinterpret_cast<const unsigned long long*>(nb + (size_t)w * 64);
    unsigned long long xs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) xs[k] = gget<true>(&p[k]);
    unsigned long long m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned long long lo = xs[2 * k], hi = xs[2 * k + 1];
      m |= (((lo & 0x0101010101010101ull) * 0x0102040810204080ull) >> 56) << (16 * k);
      m |= (((hi & 0x0101010101010101ull) * 0x0102040810204080ull) >> 56) << (16 * k + 8);
    }
    return m;
  };
  if (it > 0) {
    // subdomains that do not run keep their lists: carry their slot
    // forward and clear the change masks, 16 bytes per lane and step
    const uint4* sp = reinterpret_cast<const uint4*>(slot_at(L, (it + 1) & 1));
    uint4* sn = reinterpret_cast<uint4*>(slot_at(L, it & 1));
    uint4* cn = reinterpret_cast<uint4*>(chg_at(L, it & 1));
    const int n16 = need_stride(nsub) / 16;
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll 4
    for (int i = lane; i < n16; i += 64) {
      gput16(&sn[i], gget16(&sp[i]));
      gput16(&cn[i], zero);
    }
  }
  uint32_t count = 0;
  unsigned long long m_first = 0;               // the first pass's masks, kept
  for (int w = 0; w < nw; w += 64) {
    if (w + lane < nw) {
      const unsigned long long m = group_mask(w + lane);
      if (w == 0) m_first = m;
      count += (uint32_t)__popcll(m);
    }
  }
  count = (uint32_t)wave_sum64(count);
  if (count == 0) return 0;                     // caller turns this into an error
  // task i of the iteration goes to shard (off + i) % kShards, the
  // (i / kShards)-th of that shard; lane s < kShards handles shard s
  const int off = lat % kShards;
  const int ls = (lane - off + kShards) % kShards;         // first task index of shard `lane`
  const uint32_t ns = lane < kShards ? (count > (uint32_t)ls ? (count - 1 - ls) / kShards + 1 : 0u) : 0u;
  // the counts are set with returning memory-side atomics, not stores: the
  // tasks count them down with memory-side atomics, and a store still on its
  // way there could land after a fast task's decrement and undo it (the
  // shard would then never reach zero and the lattice would stall)
  // (the returned old values are kept live, so that the atomics return and
  // the wait below waits until they were performed)
  int32_t old_n = 0, old_s = 0;
  if (lane < kShards) old_n = atomicExch(&B.rem[(size_t)lat * kShards + lane].n, (int32_t)ns);
  if (lane == 0) {
    old_s = atomicExch(&run->shards_left, (int32_t)(count < (uint32_t)kShards ? count : (uint32_t)kShards));
    gput<true>(&run->tasks, gget<true>(&run->tasks) + count);
  }
  publish_wait();
  __asm__ volatile("" ::"v"(old_n), "v"(old_s));
  unsigned long long sbase = 0;
  if (lane < kShards && ns) sbase = atomicAdd(&B.ctr->sh[lane].tail, (unsigned long long)ns);
  unsigned long long bases[kShards];           // wave-uniform, read before the divergent walk
#pragma unroll
  for (int k = 0; k < kShards; ++k) bases[k] = rdl64(sbase, k);
  const size_t qn = (size_t)B.qmask + 1;
  if (it == 0) {
    // every subdomain runs: task i is subdomain i, in shard (off + i) mod
    // kShards at position i / kShards; 64 is a multiple of kShards, so a
    // lane's shard is the same in every round
    const int sh = (off + lane) % kShards;
    unsigned long long base = bases[0];
#pragma unroll
    for (int k = 1; k < kShards; ++k) base = sh == k ? bases[k] : base;
    unsigned long long* qs = B.q + (size_t)sh * qn;
    for (int d = lane; d < nsub; d += 64) {
      const unsigned long long at = base + (unsigned)d / kShards;
      __hip_atomic_store(&qs[at & B.qmask], ((at + 1) << 32) | ((unsigned long long)lat << 20) | (unsigned)d,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return count;
  }
  // lane-major walk: 64 subdomains per lane, set marks in ascending order
  uint32_t done_before = 0;
  for (int w0 = 0; w0 < nw; w0 += 64) {
    unsigned long long m = 0;
    if (w0 + lane < nw) m = w0 == 0 ? m_first : group_mask(w0 + lane);
    const uint32_t c = (uint32_t)__popcll(m);
    const uint32_t incl = wave_incl_scan(c);
    uint32_t i = done_before + incl - c;       // task index of this lane's first bit
    while (m) {
      const int bit = ctz64(m);
      m &= m - 1;
      const int d = (w0 + lane) * 64 + bit;
      const int sh = (int)((off + i) % kShards);
      unsigned long long base = bases[0];
#pragma unroll
      for (int k = 1; k < kShards; ++k) base = sh == k ? bases[k] : base;
      const unsigned long long at = base + i / kShards;
      const unsigned long long v = ((at + 1) << 32) | ((unsigned long long)lat << 20) | (unsigned)d;
      __hip_atomic_store(&B.q[(size_t)sh * qn + (at & B.qmask)], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      i++;
    }
    done_before += rdl(incl, 63);
  }
  return count;
}

// Device-coherent store of a run record's step.
__device__ __forceinline__ void put_step(Step* p, const Step& st) {
  gput<true>(&p->t_c, st.t_c); gput<true>(&p->t_end, st.t_end);
  gput<true>(&p->wp, st.wp); gput<true>(&p->it, st.it); gput<true>(&p->fi, st.fi);
}

// The last task of an iteration of lattice `lat`: compare step (c) of the
// Sec. 4 box for the whole lattice, then the next iteration, the next
// window (committed time advances), or completion.
__device__ void decide(const BatchArgs& B, int lat, int lane) {
  CLattice& L = ((CLattice*)B.lat)[lat];
  LatRun* run = &B.run[lat];
  const RunView rv = load_run(run, lane);
  IterFlags f;
  f.changed = rv.u32(offsetof(LatRun, fl) + offsetof(IterFlags, changed));
  f.ovf_hist = rv.u32(offsetof(LatRun, fl) + offsetof(IterFlags, ovf_hist));
  f.ovf_log = rv.u32(offsetof(LatRun, fl) + offsetof(IterFlags, ovf_log));
  f.pad = 0;
  Step st = step_of(rv);
  const int32_t max_iters = (int32_t)rv.u32(offsetof(LatRun, max_iters));
  const int32_t tune = (int32_t)rv.u32(offsetof(LatRun, tune));
  const int32_t win_budget = (int32_t)rv.u32(offsetof(LatRun, win_budget));
  const int64_t H = rv.i64(offsetof(LatRun, H));
  bool finish = false;
  if (lane == 0) gput<true>(&run->iterations, rv.i64(offsetof(LatRun, iterations)) + 1);
  int next_it = -1;
  if (f.ovf_hist || f.ovf_log) {
    if (lane == 0) gput<true>(&run->status, (int32_t)kOverflow);
    finish = true;
  } else if (f.changed) {
    if (st.it + 1 >= max_iters) {
      if (lane == 0) gput<true>(&run->status, (int32_t)kNoConv);
      finish = true;
    } else {
      next_it = st.it + 1;
    }
  } else {
    // converged: the working outputs become committed (parity flip)
    st.wp ^= 1;
    st.t_c = st.t_end;
    const int64_t wins = rv.i64(offsetof(LatRun, windows)) + 1;
    if (lane == 0) {
      gput<true>(&run->windows, wins);
      gput<true>(&run->last_g, st.it + 1);
    }
    int64_t W = rv.i64(offsetof(LatRun, W));
    if (tune) {
      W = tune_window(W, st.it + 1, rv.i64(offsetof(LatRun, Wmin)), rv.i64(offsetof(LatRun, Wmax)), kTargetGBatch);
      if (lane == 0) gput<true>(&run->W, W);
    }
    if (st.t_c >= H) {
      if (lane == 0) {
        gput<true>(&run->status, (int32_t)kDone);
        put_step(&run->st, st);
        if (B.notify) __hip_atomic_fetch_add(B.notify, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      finish = true;
    } else if ((win_budget >= 0 && wins >= win_budget) ||
               (B.yield && __hip_atomic_load(B.yield, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u)) {
      // this launch's share of windows is done, or the host asked the launch
      // to end: pause at committed time
      if (lane == 0) { gput<true>(&run->status, (int32_t)kPaused); put_step(&run->st, st); }
      finish = true;
    } else {
      st.t_end = min64(st.t_c + W, H);
      next_it = 0;
    }
  }
  if (finish) {
    publish_wait();
    if (lane == 0) atomicAdd(&B.ctr->done, 1u);
    return;
  }
  st.it = next_it;
  st.fi = 0;
  if (lane == 0) {
    put_step(&run->st, st);
    gput<true>(&run->fl.changed, 0u); gput<true>(&run->fl.ovf_hist, 0u); gput<true>(&run->fl.ovf_log, 0u);
  }
  if (enqueue_iteration(B, lat, run, L, next_it, lane) == 0) {
    // a changed iteration must schedule some subdomain; never wait forever
    if (lane == 0) gput<true>(&run->status, (int32_t)kBad);
    publish_wait();
    if (lane == 0) atomicAdd(&B.ctr->done, 1u);
  }
}

// Empty polls of one queue slot, with no task finished anywhere in the grid
// meanwhile, before the kernel gives up (tens of seconds at the longest
// back-off; a task takes microseconds to milliseconds).  Progress is the sum of the shards' ticket
// counters (every finished task takes a ticket), read every kProgressEvery
// polls; a wave whose shard has no work while others do keeps waiting.
constexpr uint32_t kSpinBudget = 20u << 20;
constexpr uint32_t kProgressEvery = 4096;

// Wave w serves shard w % kShards (the dispatcher places workgroup w on XCD
// w % kShards, so each shard's counters are hit from one XCD).  Per task:
// wait for the slot of the ticket held, relax, publish (wait for the run's
// stores), count the task down while taking the next ticket.
// A held ticket whose task is not produced yet blocks no one: tasks are
// produced by deciders, and a wave finishes its current task before it waits.
// Registers are capped so that six waves share a SIMD (80 VGPRs, no
// spills): more waves hide more of each task's latency chain.
// BX, BY, NW as for the plain kernels: <16, 16, true> (constant index
// arithmetic, no wrap handling) for launches whose lattices all have 16x16
// blocks and two or more subdomains per direction, <0, 0, false> otherwise;
// WPE caps the waves per SIMD (registers per wave).
template <int BX, int BY, bool NW, int WPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void batch_kernel(BatchArgs B) {
  extern __shared__ int8_t tile[];
  const int lane = lane_id();
  CLattice* lats = (CLattice*)B.lat;
  const int g = (int)(blockIdx.x % kShards);
  ShardCtr* sc = &B.ctr->sh[g];
  const unsigned long long* qg = B.q + (size_t)g * ((size_t)B.qmask + 1);
  // the first iteration of every lattice (all its subdomains) is dealt by
  // the grid before any wave takes a ticket; tasks are taken as they appear
  for (int k = blockIdx.x; k < (int)B.nlat; k += gridDim.x)
    enqueue_iteration(B, k, &B.run[k], lats[k], 0, lane);
  unsigned long long t = 0;
  if (lane == 0) t = atomicAdd(&sc->head, 1ull);
  t = ((uint64_t)rdl((uint32_t)(t >> 32), 0) << 32) | rdl((uint32_t)t, 0);
  for (;;) {
    const uint32_t want = (uint32_t)(t + 1);
    unsigned long long v;
    uint32_t spins = 0, polls = 0;
    unsigned long long seen = 0;
    for (;;) {
      v = __hip_atomic_load(&qg[t & B.qmask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32)) == want) break;
      if ((++polls & 7) == 0) {
        if (__hip_atomic_load(&B.ctr->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= B.nlat) return;
        if (__hip_atomic_load(&B.ctr->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
      }
      if (++spins % kProgressEvery == 0) {
        unsigned long long prog = 0;
#pragma unroll
        for (int k = 0; k < kShards; ++k)
          prog += __hip_atomic_load(&B.ctr->sh[k].head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prog = ((uint64_t)rdl((uint32_t)(prog >> 32), 0) << 32) | rdl((uint32_t)prog, 0);
        if (prog != seen) { seen = prog; spins = 0; }
      }
      if (spins > kSpinBudget) {
        // no task finished anywhere for far longer than any task takes: give
        // up rather than hang
        if (lane == 0) __hip_atomic_store(&B.ctr->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
      // back off: with few lattices most waves wait for the next iteration's
      // tasks, and their polls would compete with the running tasks' memory
      // traffic (a slot still empty after a few polls waits for a decider,
      // microseconds away)
      if (polls < 4) __builtin_amdgcn_s_sleep(1);
      else if (polls < 32) __builtin_amdgcn_s_sleep(8);
      else __builtin_amdgcn_s_sleep(32);
    }
    // the task is wave-uniform: keep it (and all that derives from it) scalar
    const uint32_t pay = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int lat = (int)((pay >> 20) & 0xFFF);
    const int d = (int)(pay & 0xFFFFF);
    LatRun* run = &B.run[lat];
    const Step st = step_of(load_run(run, lane));
    relax_subdomain<BX, BY, NW, true>(lats[lat], st, d, tile, &run->fl);
    // the run's stores are device-coherent: publishing waits for them only
    // (convergent no-ops around it keep one wait, executed by the whole wave,
    // instead of one in each lane-0 region the compiler would merge it into)
    __builtin_amdgcn_wave_barrier();
    publish_wait();
    __builtin_amdgcn_wave_barrier();
    // count this task down and take the next ticket: both memory-side
    // atomics are in flight together
    int last = 0;
    unsigned long long tn = 0;
    if (lane == 0) {
      const int32_t left = atomicSub(&B.rem[(size_t)lat * kShards + g].n, 1);
      tn = atomicAdd(&sc->head, 1ull);
      if (left == 1) last = (atomicSub(&run->shards_left, 1) == 1);
    }
    last = (int)rdl((uint32_t)last, 0);
    t = ((uint64_t)rdl((uint32_t)(tn >> 32), 0) << 32) | rdl((uint32_t)tn, 0);
    if (last) decide(B, lat, lane);
  }
}

// ------------------------------------------------------------ init / observables
__global__ void init_random_kernel(int8_t* s, int64_t n, uint32_t k0, uint32_t k1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)((uint64_t)i >> 32), c2 = 0, c3 = 1;
    philox4x32_10(k0, k1, c0, c1, c2, c3);
    s[i] = (c0 & 1u) ? (int8_t)1 : (int8_t)-1;
  }
}

__global__ void fill_kernel(int8_t* s, int64_t n, int8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s[i] = v;
}

// out[0] += sum s, out[1] += sum s (s_right + s_down).  Blocks stride over
// rows (no per-element index division); each block reduces in LDS and adds
// its two totals once (device-scope atomics are served at the memory side,
// so one per wave on a single address would serialise the whole grid).
__global__ __launch_bounds__(256) void observables_kernel(const int8_t* s, int Lx, int Ly,
                                                          unsigned long long* out) {
  __shared__ long long red[2][4];
  long long m = 0, b = 0;
  for (int y = blockIdx.x; y < Ly; y += gridDim.x) {
    const int8_t* row = s + (int64_t)y * Lx;
    const int8_t* below = s + (int64_t)(y + 1 == Ly ? 0 : y + 1) * Lx;
    for (int x = threadIdx.x; x < Lx; x += blockDim.x) {
      const int v = row[x];
      const int r = row[x + 1 == Lx ? 0 : x + 1];
      m += v;
      b += v * (r + below[x]);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    m += __shfl_xor(m, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = m; red[1][w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], (unsigned long long)(red[0][0] + red[0][1] + red[0][2] + red[0][3]));
    atomicAdd(&out[1], (unsigned long long)(red[1][0] + red[1][1] + red[1][2] + red[1][3]));
  }
}

// ------------------------------------------------------------ launchers
// 3D lattices (sr_kernels3d.hip)
hipError_t launch_relax3d(const Lattice& L, const Step& st, hipStream_t stream);
const void* relax3d_graph_kernel_ptr();
size_t relax3d_lds(const Lattice& L);

// The instantiation for a lattice's block shape and wrap: 16x16 and 32x32
// blocks have their own, split by whether a block can wrap onto itself.
static bool no_wrap(const Lattice& L) { return L.nbx > 1 && L.nby > 1; }
static const void* relax_kernel_for(const Lattice& L) {
  const bool nw = no_wrap(L);
  if (L.bx == 16 && L.by == 16) return nw ? (const void*)relax_kernel<16, 16, true> : (const void*)relax_kernel<16, 16, false>;
  if (L.bx == 32 && L.by == 32) return nw ? (const void*)relax_kernel<32, 32, true> : (const void*)relax_kernel<32, 32, false>;
  return (const void*)relax_kernel<0, 0, false>;
}
static const void* relax_graph_kernel_for(const Lattice& L) {
  if (L.Lz > 1) return relax3d_graph_kernel_ptr();
  const bool nw = no_wrap(L);
  if (L.bx == 16 && L.by == 16)
    return nw ? (const void*)relax_graph_kernel<16, 16, true> : (const void*)relax_graph_kernel<16, 16, false>;
  if (L.bx == 32 && L.by == 32)
    return nw ? (const void*)relax_graph_kernel<32, 32, true> : (const void*)relax_graph_kernel<32, 32, false>;
  return (const void*)relax_graph_kernel<0, 0, false>;
}

size_t relax_lds(const Lattice& L) {
  return L.Lz > 1 ? relax3d_lds(L) : relax_lds_bytes(L.bx, L.by, L.hcap);
}

hipError_t launch_relax(const Lattice& L, const Step& st, hipStream_t stream) {
  if (L.Lz > 1) return launch_relax3d(L, st, stream);
  size_t lds = relax_lds_bytes(L.bx, L.by, L.hcap);
  Lattice Lc = L;
  Step sc = st;
  void* args[] = {&Lc, &sc};
  return hipLaunchKernel(relax_kernel_for(L), dim3(L.nsub), dim3(64), args, lds, stream);
}

// Entry points of the graph form (the host runtime builds the window graphs
// from them).
const void* clear_flags_kernel_ptr() { return (const void*)clear_flags_kernel; }
const void* relax_graph_kernel_ptr(const Lattice& L) { return relax_graph_kernel_for(L); }

// Zeroes `bytes` (a multiple of 16) at a 16-byte aligned address: a kernel,
// so that no memset is issued for the batch queue.
__global__ void zero_kernel(uint4* p, size_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = z;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (uint4*)p, n16);
  return hipGetLastError();
}

// Both instantiations run six waves per SIMD (80 VGPRs, no spills); more
// or fewer waves per SIMD were slower (512-lattice batch 1.42 s at six
// against 1.68 / 1.44 / 1.53 s at four / seven / eight).
static const void* batch_kernel_for(int shape) {
  return shape == kBatch16NoWrap ? (const void*)batch_kernel<16, 16, true, 6> : (const void*)batch_kernel<0, 0, false, 6>;
}

hipError_t launch_batch(const BatchArgs& B, int shape, int waves, size_t lds, hipStream_t stream) {
  BatchArgs Bc = B;
  void* args[] = {&Bc};
  const hipError_t e = hipLaunchKernel(batch_kernel_for(shape), dim3(waves), dim3(64), args, lds, stream);
  return e != hipSuccess ? e : hipGetLastError();
}


int batch_waves_per_cu(int shape, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel_for(shape), 64, lds) != hipSuccess) return 0;
  return n;
}

hipError_t launch_init_random(int8_t* s, int64_t n, uint64_t seed, hipStream_t stream) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(init_random_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, s, n,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_fill(int8_t* s, int64_t n, int8_t v, hipStream_t stream) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, s, n, v);
  return hipGetLastError();
}

hipError_t launch_observables(const int8_t* s, int Lx, int Ly, unsigned long long* out,
                              hipStream_t stream) {
  const int blocks = Ly < 512 ? Ly : 512;      // one or more rows per block
  hipLaunchKernelGGL(observables_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, s, Lx, Ly,
                     out);
  return hipGetLastError();
}

}  // namespace sr
