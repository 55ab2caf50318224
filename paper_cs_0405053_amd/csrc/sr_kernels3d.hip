// sr_kernels3d.hip -- gfx950 relaxation kernel for the 3D simple-cubic
// lattice (the generalisation to more dimensions and neighbours that Secs. 3
// and 5 of the paper point to).
//
// One 64-lane wavefront plays one PE: a bx x by x bz block, local site
// v = (lz*by + ly)*bx + lx, lane l owning sites l, l+64, ... in 4-bit class
// nibbles, class k = 7*[s = -1] + (up neighbours among six), 14 classes.  The
// neighbour state outside the block is six halo faces kept as 64-bit masks
// (each face holds at most 64 sites): W/E indexed lz*by + ly, N/S lz*bx + lx,
// D/U ly*bx + lx.  A run reads the six facing boundary histories of its
// neighbours' previous iteration, merged by (tick, face) into one stream in
// LDS (break points, Sec. 5), writes its own six face lists, and compares
// them with its previous ones (step (c) over "more atoms", Sec. 5).  Runs
// always start at the window start (no mid-window checkpoints); subdomains
// whose facing inputs did not change keep their outputs.
#include "sr_device.h"

namespace sr {

constexpr int kKeyShift3 = 9;   // merged key: tick << 9 | face << 6 | position

__host__ __device__ inline size_t relax3d_lds_bytes(int bx, int by, int bz, int hcap) {
  size_t tile = (size_t)(bx + 2) * (by + 2) * (bz + 2);
  size_t lists = (size_t)3 * kFaces3 * hcap * sizeof(uint64_t);
  size_t b = tile > lists ? tile : lists;
  return (b + 15) & ~(size_t)15;
}

template <class LT>
__device__ __forceinline__ uint64_t* hist3_at(const LT& L, int q) {
  return L.hist + (int64_t)(q & 1) * ((int64_t)L.nsub * kFaces3 * L.hcap);
}
template <class LT>
__device__ __forceinline__ uint32_t* hcnt3_at(const LT& L, int q) {
  return L.hcnt + (q & 1) * (L.nsub * kFaces3);
}
template <class LT>
__device__ __forceinline__ int64_t* fct3_at(const LT& L, int q) {
  return L.fct + (q & 1) * (L.nsub * kFaces3);
}

typedef const __attribute__((address_space(4))) Lattice CLattice3;

// The six neighbouring subdomains of d, indexed by the face they border.
struct Nbr3 {
  int n[6];
};
template <class LT>
__device__ __forceinline__ Nbr3 neighbours3(const LT& L, int d) {
  const int nbx = L.nbx, nby = L.nby, nbz = L.nbz;
  const int cx = d % nbx, cy = (d / nbx) % nby, cz = d / (nbx * nby);
  Nbr3 r;
  r.n[kFW] = (cz * nby + cy) * nbx + (cx + nbx - 1) % nbx;
  r.n[kFE] = (cz * nby + cy) * nbx + (cx + 1) % nbx;
  r.n[kFN] = (cz * nby + (cy + nby - 1) % nby) * nbx + cx;
  r.n[kFS] = (cz * nby + (cy + 1) % nby) * nbx + cx;
  r.n[kFD] = (((cz + nbz - 1) % nbz) * nby + cy) * nbx + cx;
  r.n[kFU] = (((cz + 1) % nbz) * nby + cy) * nbx + cx;
  return r;
}

// One subdomain over one window, one iteration (Sec. 4 box step (a) for
// one PE, in 3D).
template <class LT>
__device__ __forceinline__ void relax3d_subdomain(const LT& L, const Step& st, int d, int8_t* lds,
                                                  IterFlags* fl) {
  const int lane = lane_id();
  const int bx = L.bx, by = L.by, bz = L.bz, bxy = bx * by;
  const int nblk = bxy * bz;
  const int S = 1 << L.sshift;
  const int nbx = L.nbx, nby = L.nby;
  const int cx = d % nbx, cy = (d / nbx) % nby, cz = d / (nbx * nby);
  const int x0 = cx * bx, y0 = cy * by, z0 = cz * bz;
  const bool wx = L.nbx == 1, wy = L.nby == 1, wz = L.nbz == 1;   // block spans the torus
  const bool first = (st.it == 0);
  const int hcap = L.hcap;
  const Nbr3 nb = neighbours3(L, d);
  const uint8_t* slot_prev = slot_at(L, (st.it + 1) & 1);
  const int sprev = first ? 0 : slot_prev[d];
  const int sout = first ? 0 : 1 - sprev;
  const Carry* cin = &carry_at(L, st.wp)[d];
  const uint32_t k0 = L.seed_lo, k1 = L.seed_hi;
  auto clampn = [&](uint32_t n) { return (int)(n < (uint32_t)hcap ? n : (uint32_t)hcap); };

  uint32_t rate = 0;
#pragma unroll
  for (int k = 0; k < kClasses3; ++k)
    if (lane == k) rate = L.rate[k];

  // ---- committed block + one-site halo shell -> LDS, then classes
  const int tw = bx + 2, th = by + 2, tl = tw * th;
  {
    const int8_t* sp = spins_at(L, st.wp);
    const int tsz = tl * (bz + 2);
    for (int i = lane; i < tsz; i += 64) {
      const int tz = i / tl, r = i - tz * tl, ty = r / tw, tx = r - ty * tw;
      int gx = x0 + tx - 1, gy = y0 + ty - 1, gz = z0 + tz - 1;
      gx = gx < 0 ? gx + L.Lx : (gx >= L.Lx ? gx - L.Lx : gx);
      gy = gy < 0 ? gy + L.Ly : (gy >= L.Ly ? gy - L.Ly : gy);
      gz = gz < 0 ? gz + L.Lz : (gz >= L.Lz ? gz - L.Lz : gz);
      lds[i] = sp[((int64_t)gz * L.Ly + gy) * L.Lx + gx];
    }
  }
  __syncthreads();
  const int8_t* tile = lds;
  uint64_t cls = ~0ull;
  for (int i = 0; i < S; ++i) {
    const int v = lane + 64 * i;
    if (v < nblk) {
      const int lx = v % bx, t = v / bx, ly = t % by, lz = t / by;
      const int tp = ((lz + 1) * th + ly + 1) * tw + lx + 1;
      const int up = (tile[tp - 1] > 0) + (tile[tp + 1] > 0) + (tile[tp - tw] > 0) + (tile[tp + tw] > 0) +
                     (tile[tp - tl] > 0) + (tile[tp + tl] > 0);
      const int k = (tile[tp] < 0 ? 7 : 0) + up;
      cls = (cls & ~(0xFull << (4 * i))) | ((uint64_t)k << (4 * i));
    }
  }
  // halo faces (bit p = the halo site at face position p is up)
  uint64_t hW, hE, hN, hS, hD, hU;
  {
    const int pw = lane < by * bz ? lane : 0, pn = lane < bx * bz ? lane : 0, pd = lane < bxy ? lane : 0;
    const int wly = pw % by, wlz = pw / by;
    const int nlx = pn % bx, nlz = pn / bx;
    const int dlx = pd % bx, dly = pd / bx;
    hW = ballot(lane < by * bz && tile[((wlz + 1) * th + wly + 1) * tw] > 0);
    hE = ballot(lane < by * bz && tile[((wlz + 1) * th + wly + 1) * tw + bx + 1] > 0);
    hN = ballot(lane < bx * bz && tile[((nlz + 1) * th) * tw + nlx + 1] > 0);
    hS = ballot(lane < bx * bz && tile[((nlz + 1) * th + by + 1) * tw + nlx + 1] > 0);
    hD = ballot(lane < bxy && tile[(dly + 1) * tw + dlx + 1] > 0);
    hU = ballot(lane < bxy && tile[((bz + 1) * th + dly + 1) * tw + dlx + 1] > 0);
  }
  uint32_t ncnt = 0;
  for (int k = 0; k < kClasses3; ++k) {
    const uint64_t x = cls ^ (0x1111111111111111ull * (uint64_t)k);
    const uint64_t nz = (x | (x >> 1) | (x >> 2) | (x >> 3)) & 0x1111111111111111ull;
    const uint32_t c = (uint32_t)__popcll(~nz & 0x1111111111111111ull);
    const uint32_t tot = rdl(wave_incl_scan(c), 63);
    if (lane == k) ncnt = tot;
  }
  uint64_t j = cin->j, acc = cin->acc;
  int64_t anchor = cin->anchor;
  if (L.wipe && st.t_c > 0) {
    // wipe the slate (Sec. 5): drop the pending pair, hazard from t_c
    j += 1; acc = 0; anchor = st.t_c;
  }
  uint64_t dtot = 0;
  int nev = 0, nbound = 0;
  __syncthreads();                               // the tile's LDS is reused below

  // ---- the neighbours' facing lists of the previous iteration, merged by
  // (tick, face); the own lists of the previous iteration for the compare
  uint64_t* raw = reinterpret_cast<uint64_t*>(lds);
  uint64_t* mrg = raw + kFaces3 * hcap;
  uint64_t* lprev = raw + 2 * kFaces3 * hcap;
  uint64_t* lcur = raw;
  int ni[6], oi[7];
  const uint64_t* li[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const bool none = first || (f < 2 ? wx : f < 4 ? wy : wz);
    const int e = nb.n[f];
    const int sl = none ? 0 : slot_prev[e];
    li[f] = hist3_at(L, sl) + ((size_t)e * kFaces3 + (f ^ 1)) * hcap;   // its face that borders ours
    ni[f] = none ? 0 : clampn(hcnt3_at(L, sl)[e * kFaces3 + (f ^ 1)]);
  }
  oi[0] = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f) oi[f + 1] = oi[f] + ni[f];
  const int tot = oi[6];
#pragma unroll
  for (int f = 0; f < 6; ++f)
    for (int i = lane; i < ni[f]; i += 64) {
      const uint64_t x = li[f][i];
      raw[oi[f] + i] = ((x >> kPosBits) << kKeyShift3) | ((uint64_t)f << 6) | (x & 63);
    }
  const uint64_t* pb = hist3_at(L, sprev) + (size_t)d * kFaces3 * hcap;
  int np[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    np[f] = first ? 0 : clampn(hcnt3_at(L, sprev)[d * kFaces3 + f]);
    for (int i = lane; i < np[f]; i += 64) lprev[f * hcap + i] = pb[f * hcap + i];
  }
  const uint64_t dig_in = rdl64(cin->digest, 0);
  const int64_t flips_in = (int64_t)rdl64((uint64_t)cin->flips, 0);
  const int64_t nbmax_in = first ? 0 : (int64_t)rdl64((uint64_t)carry_at(L, st.wp ^ 1)[d].nbmax, 0);
  const unsigned long long ev_in = rdl64(L.stat[d].events, 0), runs_in = rdl64(L.stat[d].runs, 0);
  __syncthreads();
  if (tot > 0) {
    for (int i = lane; i < tot; i += 64) {
      int q = 0;
#pragma unroll
      for (int f = 1; f < 6; ++f) q = i >= oi[f] ? f : q;
      const uint64_t key = raw[i];
      int rank = 0;
#pragma unroll
      for (int f = 0; f < 6; ++f)
        rank += f == q ? i - oi[f] : lds_lower_bound(raw + oi[f], ni[f], key);
      mrg[rank] = key;
    }
    __syncthreads();
  }
  Merged in;
  merged_open<kKeyShift3>(in, mrg, tot, 0, lane);

  uint64_t* ob = hist3_at(L, sout) + (size_t)d * kFaces3 * hcap;
  int nW = 0, nE = 0, nN = 0, nS = 0, nD = 0, nU = 0;
  auto push = [&](int f, int& n, uint64_t x) {
    if (lane == 0 && n < hcap) lcur[f * hcap + n] = x;
    n++;
  };

  uint64_t Eb, Vb;
  draw_chunk(k0, k1, j & ~63ull, (uint32_t)d, lane, L.tick_bits, Eb, Vb);
  uint64_t E = rdl64(Eb, (int)(j & 63)), V = rdl64(Vb, (int)(j & 63));
  uint64_t C = row_incl_scan64((uint64_t)ncnt * rate);
  uint64_t lam = rdl64(C, kClasses3 - 1);
  int64_t next = next_tick(anchor, E, acc, lam);

  uint64_t* wl = L.wlog + (size_t)d * L.wcap;
  const int wcap = L.wcap;
  uint64_t lbuf = 0;
  auto log_flush = [&](int k) {
    const int at = nev - k + lane;
    uint64_t dsum = 0;
    if (lane < k) {
      if (at < wcap) wl[at] = lbuf;
      const int v = (int)(lbuf & 0xFFFF);
      const int lx = v % bx, t = v / bx, ly = t % by, lz = t / by;
      const int64_t g = ((int64_t)(z0 + lz) * L.Ly + (y0 + ly)) * L.Lx + x0 + lx;
      dsum = mix64(mix64(lbuf >> kPosBits) + (uint64_t)g);
    }
    dtot += wave_sum64(dsum);
  };
  auto change = [&](int u, int delta) {
    const int o = u & 63, sl = (u >> 6) * 4;
    const uint64_t w = rdl64(cls, o);
    const int a = (int)((w >> sl) & 15);
    const int b = a + delta;
    if (lane == o) cls += (uint64_t)(int64_t)delta * (1ull << sl);
    ncnt += (uint32_t)((lane == b) - (lane == a));
  };
  // in each direction the two neighbours of a site are distinct unless the
  // block wraps onto itself with side 2
  const bool distinct = (bx >= 3 || !wx) && (by >= 3 || !wy) && (bz >= 3 || !wz);

  const int64_t t_end = st.t_end;
  const int nev_limit = 4 * wcap + 64;
  bool runaway = false;
  for (;;) {
    if (nev >= nev_limit) { runaway = true; break; }
    const int64_t tb = in.ht;
    const int64_t tn = min64(next, tb);
    if (tn >= t_end) break;
    if (next <= tb) {
      // ---- own event (first on a tie)
      const int64_t t = next;
      const uint64_t target = __umul64hi(V, lam);
      const uint64_t gt = ballot(C > target) & ((1ull << kClasses3) - 1);
      const int ks = ctz64(gt);
      const uint64_t below = ks ? rdl64(C, ks - 1) : 0ull;
      const uint32_t rk = rdl(rate, ks);
      const uint32_t idx = (uint32_t)__builtin_amdgcn_readfirstlane((int)udiv_small(target - below, rk));
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
      const int lx = v % bx, vt = v / bx, ly = vt % by, lz = vt / by;
      const int kv = (int)((rdl64(cls, v & 63) >> ((v >> 6) * 4)) & 15);
      const bool now_up = kv >= 7;
      const int dup = now_up ? 1 : -1;
      const int nbr[6] = {lx > 0 ? v - 1 : (wx ? v + bx - 1 : -1),
                          lx < bx - 1 ? v + 1 : (wx ? v - bx + 1 : -1),
                          ly > 0 ? v - bx : (wy ? v + (by - 1) * bx : -1),
                          ly < by - 1 ? v + bx : (wy ? v - (by - 1) * bx : -1),
                          lz > 0 ? v - bxy : (wz ? v + (bz - 1) * bxy : -1),
                          lz < bz - 1 ? v + bxy : (wz ? v - (bz - 1) * bxy : -1)};
      if (distinct) {
        // seven distinct sites: old classes from the words before the flip,
        // all moves at once
        const int dv = now_up ? -7 : 7;
        uint64_t add = lane == (v & 63) ? (uint64_t)(int64_t)dv << ((v >> 6) * 4) : 0ull;
        uint32_t inc = (uint32_t)(lane == kv + dv), dec = (uint32_t)(lane == kv);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
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
        change(v, now_up ? -7 : 7);
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (nbr[q] >= 0) change(nbr[q], dup);
      }
      const uint64_t tk = (uint64_t)t << kPosBits;
      if (lane == (nev & 63)) lbuf = tk | (uint64_t)v;
      nev++;
      if ((nev & 63) == 0) log_flush(64);
      bool onb = false;
      if (!wx && lx == 0) { push(kFW, nW, tk | (uint64_t)(lz * by + ly)); onb = true; }
      if (!wx && lx == bx - 1) { push(kFE, nE, tk | (uint64_t)(lz * by + ly)); onb = true; }
      if (!wy && ly == 0) { push(kFN, nN, tk | (uint64_t)(lz * bx + lx)); onb = true; }
      if (!wy && ly == by - 1) { push(kFS, nS, tk | (uint64_t)(lz * bx + lx)); onb = true; }
      if (!wz && lz == 0) { push(kFD, nD, tk | (uint64_t)(ly * bx + lx)); onb = true; }
      if (!wz && lz == bz - 1) { push(kFU, nU, tk | (uint64_t)(ly * bx + lx)); onb = true; }
      nbound += onb;
      j += 1; anchor = t; acc = 0;
      if ((j & 63) == 0) draw_chunk(k0, k1, j, (uint32_t)d, lane, L.tick_bits, Eb, Vb);
      E = rdl64(Eb, (int)(j & 63)); V = rdl64(Vb, (int)(j & 63));
      C = row_incl_scan64((uint64_t)ncnt * rate);
      lam = rdl64(C, kClasses3 - 1);
      next = next_tick(anchor, E, acc, lam);
    } else {
      // ---- break point: a neighbour's flip on one of our halo faces
      const int64_t t = tb;
      const uint64_t key = merged_pop<kKeyShift3>(in, lane);
      const int q = (int)((key >> 6) & 7);
      const int p = (int)(key & 63);
      int u;
      bool up;
      if (q == kFW) { hW ^= 1ull << p; up = (hW >> p) & 1; u = p * bx; }
      else if (q == kFE) { hE ^= 1ull << p; up = (hE >> p) & 1; u = p * bx + bx - 1; }
      else if (q == kFN) { hN ^= 1ull << p; up = (hN >> p) & 1; u = (p / bx) * bxy + p % bx; }
      else if (q == kFS) { hS ^= 1ull << p; up = (hS >> p) & 1; u = (p / bx) * bxy + (by - 1) * bx + p % bx; }
      else if (q == kFD) { hD ^= 1ull << p; up = (hD >> p) & 1; u = p; }
      else { hU ^= 1ull << p; up = (hU >> p) & 1; u = (bz - 1) * bxy + p; }
      change(u, up ? 1 : -1);
      acc += lam * (uint64_t)(t - anchor);
      anchor = t;
      C = row_incl_scan64((uint64_t)ncnt * rate);
      lam = rdl64(C, kClasses3 - 1);
      next = next_tick(anchor, E, acc, lam);
    }
  }
  if (nev & 63) log_flush(nev & 63);

  int8_t* so = spins_at(L, st.wp ^ 1);
  for (int i = 0; i < S; ++i) {
    const int v = lane + 64 * i;
    if (v < nblk) {
      const int lx = v % bx, t = v / bx, ly = t % by, lz = t / by;
      so[((int64_t)(z0 + lz) * L.Ly + (y0 + ly)) * L.Lx + x0 + lx] =
          ((cls >> (4 * i)) & 15) < 7 ? (int8_t)1 : (int8_t)-1;
    }
  }
  const int nn[6] = {nW, nE, nN, nS, nD, nU};
  int64_t fc[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int n = clampn((uint32_t)nn[f]);
    const uint64_t* cur = lcur + f * hcap;
    fc[f] = first ? (n > 0 ? (int64_t)(cur[0] >> kPosBits) : kTickInf)
                  : first_change(cur, n, lprev + f * hcap, np[f], 0, lane);
    for (int i = lane; i < n; i += 64) ob[f * hcap + i] = cur[i];
  }
  if (lane == 0) {
    uint32_t* cnt_out = hcnt3_at(L, sout) + d * kFaces3;
    int64_t* fct_out = fct3_at(L, sout) + d * kFaces3;
    uint32_t emask = 0;
    bool ovf_h = false;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      cnt_out[f] = (uint32_t)nn[f];
      fct_out[f] = fc[f];
      emask |= fc[f] != kTickInf ? 1u << f : 0u;
      ovf_h |= nn[f] > hcap;
    }
    Carry* co = &carry_at(L, st.wp ^ 1)[d];
    co->j = j; co->anchor = anchor; co->acc = acc;
    co->digest = dig_in + dtot;
    co->flips = flips_in + nev;
    co->wflips = nev;
    co->nbound = nbound;
    co->nbmax = nbound > nbmax_in ? nbound : nbmax_in;
    L.stat[d].events = ev_in + (unsigned long long)nev;
    L.stat[d].runs = runs_in + 1ull;
    L.wcnt[d] = (uint32_t)nev;
    slot_at(L, st.it & 1)[d] = (uint8_t)sout;
    chg_at(L, st.it & 1)[d] = (uint8_t)emask;
    if (emask) fl->changed = 1u;
    if (ovf_h) fl->ovf_hist = 1u;
    if (nev > wcap || runaway) fl->ovf_log = 1u;
  }
}

// Does subdomain d run in iteration it (> 0)?  Only if a face list of a
// neighbour that borders it changed in the previous iteration.
template <class LT>
__device__ __forceinline__ bool inputs_changed3(const LT& L, int it, int d) {
  const uint8_t* c = chg_at(L, (it + 1) & 1);
  const Nbr3 nb = neighbours3(L, d);
  bool need = false;
  if (L.nbx > 1) need |= ((c[nb.n[kFW]] >> kFE) & 1) | ((c[nb.n[kFE]] >> kFW) & 1);
  if (L.nby > 1) need |= ((c[nb.n[kFN]] >> kFS) & 1) | ((c[nb.n[kFS]] >> kFN) & 1);
  if (L.nbz > 1) need |= ((c[nb.n[kFD]] >> kFU) & 1) | ((c[nb.n[kFU]] >> kFD) & 1);
  return need;
}

__global__ __launch_bounds__(64) void relax3d_kernel(Lattice L, Step st) {
  extern __shared__ int8_t tile[];
  const int d = blockIdx.x;
  if (d >= L.nsub) return;
  if (st.fi > 0) {
    const IterFlags* fp = L.flags + st.fi - 1;
    if (fp->changed == 0 || fp->ovf_hist != 0 || fp->ovf_log != 0) return;
  }
  if (st.it > 0 && !inputs_changed3(L, st.it, d)) {
    if (lane_id() == 0) {
      slot_at(L, st.it & 1)[d] = slot_at(L, (st.it + 1) & 1)[d];
      chg_at(L, st.it & 1)[d] = 0;
    }
    return;
  }
  relax3d_subdomain(*(CLattice3*)__builtin_amdgcn_kernarg_segment_ptr(), st, d, tile, L.flags + st.fi);
}

__global__ __launch_bounds__(64) void relax3d_graph_kernel(Lattice L, const Step* stp, int i) {
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
  if (st.it > 0 && !inputs_changed3(L, st.it, d)) {
    if (lane_id() == 0) {
      slot_at(L, st.it & 1)[d] = slot_at(L, (st.it + 1) & 1)[d];
      chg_at(L, st.it & 1)[d] = 0;
    }
    return;
  }
  relax3d_subdomain(*(CLattice3*)__builtin_amdgcn_kernarg_segment_ptr(), st, d, tile, L.flags + i);
}

// out[0] += sum s, out[1] += sum s (s_{+x} + s_{+y} + s_{+z}); one block per
// group of (z, y) rows, LDS reduction, two atomics per block.
__global__ __launch_bounds__(256) void observables3d_kernel(const int8_t* s, int Lx, int Ly, int Lz,
                                                            unsigned long long* out) {
  __shared__ long long red[2][4];
  long long m = 0, b = 0;
  const int rows = Ly * Lz;
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const int z = r / Ly, y = r - z * Ly;
    const int8_t* row = s + (int64_t)r * Lx;
    const int8_t* south = s + ((int64_t)z * Ly + (y + 1 == Ly ? 0 : y + 1)) * Lx;
    const int8_t* up = s + ((int64_t)(z + 1 == Lz ? 0 : z + 1) * Ly + y) * Lx;
    for (int x = threadIdx.x; x < Lx; x += blockDim.x) {
      const int v = row[x];
      m += v;
      b += v * (row[x + 1 == Lx ? 0 : x + 1] + south[x] + up[x]);
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
size_t relax3d_lds(const Lattice& L) { return relax3d_lds_bytes(L.bx, L.by, L.bz, L.hcap); }

hipError_t launch_relax3d(const Lattice& L, const Step& st, hipStream_t stream) {
  Lattice Lc = L;
  Step sc = st;
  void* args[] = {&Lc, &sc};
  return hipLaunchKernel((const void*)relax3d_kernel, dim3(L.nsub), dim3(64), args, relax3d_lds(L), stream);
}

const void* relax3d_graph_kernel_ptr() { return (const void*)relax3d_graph_kernel; }

hipError_t launch_observables3d(const int8_t* s, int Lx, int Ly, int Lz, unsigned long long* out,
                                hipStream_t stream) {
  const int rows = Ly * Lz;
  const int blocks = rows < 1024 ? rows : 1024;
  hipLaunchKernelGGL(observables3d_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, s, Lx, Ly, Lz, out);
  return hipGetLastError();
}

}  // namespace sr
