/*
 * sr_oracle3d.c -- CPU oracle for synchronous relaxation of the n-fold way
 * Ising simulation on a 3D simple-cubic lattice (the generalisation to more
 * dimensions and neighbours the paper names in Secs. 3 and 5).
 *
 * TEST INFRASTRUCTURE ONLY, like sr_oracle.c: only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * shares no code with it.  Plain single-threaded C99, written for reading.
 * It reuses this library's own Philox-4x32-10, fixed-point -ln and event
 * digest (sr_oracle.c), and follows the same integer conventions as the 2D
 * oracle, with these 3D readings:
 *  - lattice Lx x Ly x Lz, periodic, six nearest neighbours; global site
 *    index (z*Ly + y)*Lx + x; energy of eq. hamil with every bond counted
 *    once (a direction of length 2 links a pair by two bonds, one each way);
 *  - classes of Sec. 3: spin (2 states) times up neighbours (0..6), i.e.
 *    k = 7*[s = -1] + n_up, 14 classes; flipping s changes the energy by
 *    dE = 2 s (J (2 n_up - 6) + h);
 *  - subdomains bx x by x bz, id (cz*nby + cy)*nbx + cx; a site's local index
 *    (lz*by + ly)*bx + lx orders the members of a class;
 *  - boundary histories per face (Sec. 4 step (c) "more dimensions, more
 *    neighbours"): W (x = 0 layer), E, N (y = 0), S, D (z = 0), U, each entry
 *    (tick, position in the face): W/E by lz*by + ly, N/S by lz*bx + lx,
 *    D/U by ly*bx + lx;
 *  - random pairs: subdomain d, event index j, counter (j lo, j hi, d, 0);
 *    initial spins: counter (site lo, site hi, 0, 1), up iff word 0 is odd.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "sr_oracle.h"

#define NC3 14
#define RATE_ONE3 (1u << 28)
#define TICK_INF3 INT64_MAX

/* Rates of the 14 classes (eqs. hamil, pMin / pglauber), round(2^28 p). */
int orc3_rate_table(double J, double h, double T, int rule, uint32_t out[NC3]) {
  if (!(T > 0.0) || (rule != ORC_METROPOLIS && rule != ORC_GLAUBER)) return -1;
  for (int k = 0; k < NC3; ++k) {
    int s = (k < 7) ? 1 : -1;
    int nup = k % 7;
    double x = -(2.0 * s * (J * (2 * nup - 6) + h)) / T; /* -dE / T */
    double p;
    if (rule == ORC_METROPOLIS) {
      double theta = exp(x);
      p = theta < 1.0 ? theta : 1.0;
    } else {
      p = 1.0 / (1.0 + exp(-x));
    }
    double q = nearbyint(ldexp(p, 28));
    if (q > (double)RATE_ONE3) q = (double)RATE_ONE3;
    out[k] = (uint32_t)q;
  }
  return 0;
}

typedef struct {
  int Lx, Ly, Lz, bx, by, bz, nbx, nby, nbz, nsub;
  uint32_t rate[NC3];
  uint64_t seed;
  int tick_bits;
} lat3_t;

static int lat3_init(lat3_t* L, const orc3_params* p) {
  if (p->Lx < 2 || p->Ly < 2 || p->Lz < 2 || p->bx < 1 || p->by < 1 || p->bz < 1) return -1;
  if (p->Lx % p->bx || p->Ly % p->by || p->Lz % p->bz) return -1;
  if (p->tick_bits < 1 || p->tick_bits > 28) return -1;
  if (p->window_ticks < 1 || p->horizon_ticks < 0) return -1;
  if (p->step_rule != ORC_STEP_CONTINUE && p->step_rule != ORC_STEP_WIPE) return -1;
  if ((int64_t)p->bx * p->by * p->bz > 4096) return -1;
  L->Lx = p->Lx; L->Ly = p->Ly; L->Lz = p->Lz;
  L->bx = p->bx; L->by = p->by; L->bz = p->bz;
  L->nbx = p->Lx / p->bx; L->nby = p->Ly / p->by; L->nbz = p->Lz / p->bz;
  L->nsub = L->nbx * L->nby * L->nbz;
  L->seed = p->seed;
  L->tick_bits = p->tick_bits;
  return orc3_rate_table(p->J, p->h, p->T, p->rule, L->rate);
}

static int wrap3(int a, int n) { return ((a % n) + n) % n; }

static int64_t gidx(const lat3_t* L, int x, int y, int z) {
  return ((int64_t)wrap3(z, L->Lz) * L->Ly + wrap3(y, L->Ly)) * L->Lx + wrap3(x, L->Lx);
}

static int sub3_of_site(const lat3_t* L, int x, int y, int z) {
  x = wrap3(x, L->Lx); y = wrap3(y, L->Ly); z = wrap3(z, L->Lz);
  return ((z / L->bz) * L->nby + (y / L->by)) * L->nbx + (x / L->bx);
}

static void sub3_origin(const lat3_t* L, int d, int* x0, int* y0, int* z0) {
  *x0 = (d % L->nbx) * L->bx;
  *y0 = ((d / L->nbx) % L->nby) * L->by;
  *z0 = (d / (L->nbx * L->nby)) * L->bz;
}

static int init3_spins(const lat3_t* L, const orc3_params* p, int8_t* s) {
  int64_t n = (int64_t)L->Lx * L->Ly * L->Lz;
  if (p->init == ORC_INIT_USER) {
    if (!p->init_spins) return -1;
    for (int64_t i = 0; i < n; ++i) {
      if (p->init_spins[i] != 1 && p->init_spins[i] != -1) return -1;
      s[i] = p->init_spins[i];
    }
  } else if (p->init == ORC_INIT_ALL_UP) {
    for (int64_t i = 0; i < n; ++i) s[i] = 1;
  } else if (p->init == ORC_INIT_RANDOM) {
    uint32_t key[2] = {(uint32_t)L->seed, (uint32_t)(L->seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
      uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 1u};
      uint32_t o[4];
      orc_philox4x32_10(key, ctr, o);
      s[i] = (o[0] & 1u) ? 1 : -1;
    }
  } else {
    return -1;
  }
  return 0;
}

static void draw3(const lat3_t* L, int d, uint64_t j, uint64_t* E, uint64_t* V) {
  uint32_t key[2] = {(uint32_t)L->seed, (uint32_t)(L->seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), (uint32_t)d, 0u};
  uint32_t o[4];
  orc_philox4x32_10(key, ctr, o);
  *V = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
  *E = orc_expq((uint64_t)o[0] | ((uint64_t)o[1] << 32), L->tick_bits);
}

static int64_t next3(int64_t anchor, uint64_t E, uint64_t acc, uint64_t lam) {
  if (lam == 0) return TICK_INF3;
  uint64_t rem = E - acc;
  uint64_t q = rem / lam + (rem % lam != 0);
  if (q < 1) q = 1;
  if (q > (uint64_t)(TICK_INF3 - anchor)) return TICK_INF3;
  return anchor + (int64_t)q;
}

/* M and the bond sum over +x, +y, +z bonds, from scratch. */
static void observe3(const lat3_t* L, const int8_t* s, int64_t* M, int64_t* bond) {
  int64_t m = 0, b = 0;
  for (int z = 0; z < L->Lz; ++z)
    for (int y = 0; y < L->Ly; ++y)
      for (int x = 0; x < L->Lx; ++x) {
        int v = s[gidx(L, x, y, z)];
        m += v;
        b += v * (s[gidx(L, x + 1, y, z)] + s[gidx(L, x, y + 1, z)] + s[gidx(L, x, y, z + 1)]);
      }
  *M = m;
  *bond = b;
}

static int nbr_sum3(const lat3_t* L, const int8_t* s, int x, int y, int z) {
  return s[gidx(L, x + 1, y, z)] + s[gidx(L, x - 1, y, z)] + s[gidx(L, x, y + 1, z)]
       + s[gidx(L, x, y - 1, z)] + s[gidx(L, x, y, z + 1)] + s[gidx(L, x, y, z - 1)];
}

static int class3_of(const lat3_t* L, const int8_t* s, int x, int y, int z) {
  int up = (s[gidx(L, x + 1, y, z)] > 0) + (s[gidx(L, x - 1, y, z)] > 0)
         + (s[gidx(L, x, y + 1, z)] > 0) + (s[gidx(L, x, y - 1, z)] > 0)
         + (s[gidx(L, x, y, z + 1)] > 0) + (s[gidx(L, x, y, z - 1)] > 0);
  return 7 * (s[gidx(L, x, y, z)] < 0) + up;
}

static uint64_t sub3_lambda(const lat3_t* L, const int8_t* s, int d, int64_t N[NC3]) {
  int x0, y0, z0;
  sub3_origin(L, d, &x0, &y0, &z0);
  for (int k = 0; k < NC3; ++k) N[k] = 0;
  for (int lz = 0; lz < L->bz; ++lz)
    for (int ly = 0; ly < L->by; ++ly)
      for (int lx = 0; lx < L->bx; ++lx) N[class3_of(L, s, x0 + lx, y0 + ly, z0 + lz)]++;
  uint64_t lam = 0;
  for (int k = 0; k < NC3; ++k) lam += (uint64_t)N[k] * L->rate[k];
  return lam;
}

/* Class, then site (eqs. Wsum, Wstop, nores, vindex); global site index. */
static int64_t select3_site(const lat3_t* L, const int8_t* s, int d, uint64_t V) {
  int64_t N[NC3];
  uint64_t lam = sub3_lambda(L, s, d, N);
  uint64_t target = (uint64_t)(((unsigned __int128)V * lam) >> 64);
  uint64_t below = 0;
  int ks = -1;
  for (int k = 0; k < NC3; ++k) {
    uint64_t w = (uint64_t)N[k] * L->rate[k];
    if (below + w > target) { ks = k; break; }
    below += w;
  }
  if (ks < 0) return -1;
  uint64_t idx = (target - below) / L->rate[ks];
  int x0, y0, z0;
  sub3_origin(L, d, &x0, &y0, &z0);
  uint64_t seen = 0;
  for (int lz = 0; lz < L->bz; ++lz)
    for (int ly = 0; ly < L->by; ++ly)
      for (int lx = 0; lx < L->bx; ++lx)
        if (class3_of(L, s, x0 + lx, y0 + ly, z0 + lz) == ks) {
          if (seen == idx) return gidx(L, x0 + lx, y0 + ly, z0 + lz);
          seen++;
        }
  return -1;
}

int orc3_select_site(const orc3_params* p, const int8_t* spins, int d, uint64_t V, int64_t* site_out) {
  lat3_t L;
  if (lat3_init(&L, p) != 0 || d < 0 || d >= L.nsub) return -1;
  int64_t v = select3_site(&L, spins, d, V);
  if (v < 0) return -2;
  *site_out = v;
  return 0;
}

int orc3_subdomain_lambda(const orc3_params* p, const int8_t* spins, int d, uint64_t* lam_out) {
  lat3_t L;
  int64_t N[NC3];
  if (lat3_init(&L, p) != 0 || d < 0 || d >= L.nsub) return -1;
  *lam_out = sub3_lambda(&L, spins, d, N);
  return 0;
}

/* ======================================================================== */
/* DES: all subdomains' event streams merged in global tick order.  The     */
/* next subdomain is found by a linear scan (the 3D lattices tested here    */
/* are small).                                                              */
/* ======================================================================== */
typedef struct {
  uint64_t j, acc, E, V, lam;
  int64_t anchor, next;
} sub3_t;

static int cmp3_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

int orc3_des_run(const orc3_params* p, orc_result* r) {
  lat3_t L;
  if (lat3_init(&L, p) != 0) return -1;
  int8_t* s = r->spins;
  if (!s) return -1;
  if (init3_spins(&L, p, s) != 0) return -1;
  int nsub = L.nsub;
  sub3_t* sub = (sub3_t*)calloc((size_t)nsub, sizeof(sub3_t));
  int* S = (int*)malloc(sizeof(int) * nsub);
  int64_t* vsel = (int64_t*)malloc(sizeof(int64_t) * nsub);
  int* aff = (int*)malloc(sizeof(int) * 7 * nsub);
  char* inS = (char*)calloc((size_t)nsub, 1);
  if (!sub || !S || !vsel || !aff || !inS) return -2;
  for (int d = 0; d < nsub; ++d) {
    int64_t N[NC3];
    draw3(&L, d, 0, &sub[d].E, &sub[d].V);
    sub[d].lam = sub3_lambda(&L, s, d, N);
    sub[d].next = next3(0, sub[d].E, 0, sub[d].lam);
    if (r->sub_flips) r->sub_flips[d] = 0;
    if (r->sub_digest) r->sub_digest[d] = 0;
  }
  int64_t M, bond;
  observe3(&L, s, &M, &bond);
  int64_t nwin = p->horizon_ticks == 0 ? 0 : (p->horizon_ticks + p->window_ticks - 1) / p->window_ticks;
  int64_t snap = 0, nev = 0;
  double iM = 0, iM2 = 0, iabsM = 0, ibond = 0, iE2 = 0, iM4 = 0;
  int64_t t_last = p->burn_ticks;
  int64_t next_wipe = p->window_ticks;
  const int64_t stop = p->horizon_ticks;
  for (;;) {
    int64_t t = TICK_INF3;
    for (int d = 0; d < nsub; ++d) if (sub[d].next < t) t = sub[d].next;
    /* wipe rule (Sec. 5 alternate approach): every step start before the
     * next event drops every pending event */
    if (p->step_rule == ORC_STEP_WIPE && next_wipe < stop && next_wipe <= t) {
      for (int d = 0; d < nsub; ++d) {
        sub[d].j += 1;
        sub[d].anchor = next_wipe;
        sub[d].acc = 0;
        draw3(&L, d, sub[d].j, &sub[d].E, &sub[d].V);
        sub[d].next = next3(next_wipe, sub[d].E, 0, sub[d].lam);
      }
      next_wipe += p->window_ticks;
      continue;
    }
    int64_t t_eff = t < stop ? t : stop;
    while (snap <= nwin) {                     /* state after flips < k W */
      int64_t tc = snap * p->window_ticks;
      if (tc > stop) tc = stop;
      if (tc > t_eff) break;
      if (r->snap_M) { int64_t m2, b2; observe3(&L, s, &m2, &b2); r->snap_M[snap] = m2; r->snap_bond[snap] = b2; }
      snap++;
    }
    if (t_eff > t_last) {
      double dt = (double)(t_eff - t_last);
      double e = -p->J * (double)bond - p->h * (double)M;
      iM += dt * M; iM2 += dt * (double)M * M; iabsM += dt * (M < 0 ? -M : M);
      ibond += dt * bond; iE2 += dt * e * e; iM4 += dt * (double)M * M * (double)M * M;
      t_last = t_eff;
    }
    if (t >= stop) break;
    int nS = 0;
    for (int d = 0; d < nsub; ++d) if (sub[d].next == t) S[nS++] = d;   /* ascending id */
    for (int a = 0; a < nS; ++a) {                /* all choose before any flips */
      vsel[a] = select3_site(&L, s, S[a], sub[S[a]].V);
      if (vsel[a] < 0) return -3;
    }
    int naff = 0;
    for (int a = 0; a < nS; ++a) {
      int d = S[a];
      int64_t v = vsel[a];
      int x = (int)(v % L.Lx), y = (int)((v / L.Lx) % L.Ly), z = (int)(v / ((int64_t)L.Lx * L.Ly));
      int old = s[v];
      s[v] = (int8_t)(-old);
      M += -2 * old;
      bond += -2 * old * nbr_sum3(&L, s, x, y, z);
      if (nev < r->log_cap) { r->log_tick[nev] = t; r->log_site[nev] = v; r->log_sub[nev] = d; }
      nev++;
      if (r->sub_flips) r->sub_flips[d]++;
      if (r->sub_digest) r->sub_digest[d] += orc_event_digest(t, v);
      aff[naff++] = d;
      aff[naff++] = sub3_of_site(&L, x + 1, y, z);
      aff[naff++] = sub3_of_site(&L, x - 1, y, z);
      aff[naff++] = sub3_of_site(&L, x, y + 1, z);
      aff[naff++] = sub3_of_site(&L, x, y - 1, z);
      aff[naff++] = sub3_of_site(&L, x, y, z + 1);
      aff[naff++] = sub3_of_site(&L, x, y, z - 1);
    }
    for (int a = 0; a < nS; ++a) inS[S[a]] = 1;
    qsort(aff, (size_t)naff, sizeof(int), cmp3_int);
    for (int a = 0; a < naff; ++a) {
      int e = aff[a];
      if (a > 0 && aff[a - 1] == e) continue;
      int64_t N[NC3];
      if (inS[e]) {                         /* own event: next pair */
        sub[e].j += 1; sub[e].anchor = t; sub[e].acc = 0;
        draw3(&L, e, sub[e].j, &sub[e].E, &sub[e].V);
      } else {                              /* break point: fold the hazard */
        sub[e].acc += sub[e].lam * (uint64_t)(t - sub[e].anchor);
        sub[e].anchor = t;
      }
      sub[e].lam = sub3_lambda(&L, s, e, N);
      sub[e].next = next3(sub[e].anchor, sub[e].E, sub[e].acc, sub[e].lam);
    }
    for (int a = 0; a < nS; ++a) inS[S[a]] = 0;
  }
  r->n_events = nev;
  r->M = M; r->bond = bond;
  r->int_M = iM; r->int_M2 = iM2; r->int_absM = iabsM; r->int_bond = ibond;
  r->int_E2 = iE2; r->int_M4 = iM4;
  r->int_ticks = (p->horizon_ticks > p->burn_ticks) ? (p->horizon_ticks - p->burn_ticks) : 0;
  if (r->carry)
    for (int d = 0; d < nsub; ++d) {
      r->carry[4 * d + 0] = (int64_t)sub[d].j;
      r->carry[4 * d + 1] = sub[d].anchor;
      r->carry[4 * d + 2] = (int64_t)sub[d].acc;
      r->carry[4 * d + 3] = sub[d].next;
    }
  {
    int64_t m2, b2;
    observe3(&L, s, &m2, &b2);
    if (m2 != M || b2 != bond) return -4;
  }
  free(sub); free(S); free(vsel); free(aff); free(inS);
  return 0;
}

/* ======================================================================== */
/* Literal synchronous relaxation in 3D (Sec. 4 box): each subdomain alone  */
/* over [t_c, t_end) from the committed state, its six halo faces flipped   */
/* by the neighbours' face histories of the previous iteration.             */
/* ======================================================================== */
enum { FW = 0, FE = 1, FN = 2, FS = 3, FD = 4, FU = 5 };

typedef struct { int64_t* tick; int32_t* pos; int64_t n, cap; } hl3_t;

static int hl3_push(hl3_t* h, int64_t t, int32_t pos) {
  if (h->n == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 16;
    int64_t* nt = (int64_t*)realloc(h->tick, sizeof(int64_t) * nc);
    if (!nt) return -1;
    h->tick = nt;
    int32_t* np = (int32_t*)realloc(h->pos, sizeof(int32_t) * nc);
    if (!np) return -1;
    h->pos = np;
    h->cap = nc;
  }
  h->tick[h->n] = t; h->pos[h->n] = pos; h->n++;
  return 0;
}
static int hl3_equal(const hl3_t* a, const hl3_t* b) {
  if (a->n != b->n) return 0;
  for (int64_t i = 0; i < a->n; ++i)
    if (a->tick[i] != b->tick[i] || a->pos[i] != b->pos[i]) return 0;
  return 1;
}

/* One subdomain's view: its block and six halo faces.  A direction in which
 * the block spans the torus wraps inside the block and has no halo. */
typedef struct {
  const lat3_t* L;
  int wrap[3];
  int8_t* blk;               /* bz*by*bx */
  int8_t* face[6];           /* halo layers beyond each face */
} loc3_t;

static int face_pos(const lat3_t* L, int f, int lx, int ly, int lz) {
  if (f == FW || f == FE) return lz * L->by + ly;
  if (f == FN || f == FS) return lz * L->bx + lx;
  return ly * L->bx + lx;
}

static int l3_spin(const loc3_t* B, int lx, int ly, int lz) {
  const lat3_t* L = B->L;
  if (lx < 0 || lx >= L->bx) {
    if (B->wrap[0]) lx = wrap3(lx, L->bx);
    else return B->face[lx < 0 ? FW : FE][face_pos(L, FW, 0, ly, lz)];
  }
  if (ly < 0 || ly >= L->by) {
    if (B->wrap[1]) ly = wrap3(ly, L->by);
    else return B->face[ly < 0 ? FN : FS][face_pos(L, FN, lx, 0, lz)];
  }
  if (lz < 0 || lz >= L->bz) {
    if (B->wrap[2]) lz = wrap3(lz, L->bz);
    else return B->face[lz < 0 ? FD : FU][face_pos(L, FD, lx, ly, 0)];
  }
  return B->blk[(lz * L->by + ly) * L->bx + lx];
}
static int l3_class(const loc3_t* B, int lx, int ly, int lz) {
  int up = (l3_spin(B, lx + 1, ly, lz) > 0) + (l3_spin(B, lx - 1, ly, lz) > 0)
         + (l3_spin(B, lx, ly + 1, lz) > 0) + (l3_spin(B, lx, ly - 1, lz) > 0)
         + (l3_spin(B, lx, ly, lz + 1) > 0) + (l3_spin(B, lx, ly, lz - 1) > 0);
  return 7 * (l3_spin(B, lx, ly, lz) < 0) + up;
}
static uint64_t l3_lambda(const loc3_t* B) {
  const lat3_t* L = B->L;
  int64_t N[NC3] = {0};
  for (int lz = 0; lz < L->bz; ++lz)
    for (int ly = 0; ly < L->by; ++ly)
      for (int lx = 0; lx < L->bx; ++lx) N[l3_class(B, lx, ly, lz)]++;
  uint64_t lam = 0;
  for (int k = 0; k < NC3; ++k) lam += (uint64_t)N[k] * L->rate[k];
  return lam;
}
static int l3_select(const loc3_t* B, uint64_t V) {
  const lat3_t* L = B->L;
  int64_t N[NC3] = {0};
  for (int lz = 0; lz < L->bz; ++lz)
    for (int ly = 0; ly < L->by; ++ly)
      for (int lx = 0; lx < L->bx; ++lx) N[l3_class(B, lx, ly, lz)]++;
  uint64_t lam = 0;
  for (int k = 0; k < NC3; ++k) lam += (uint64_t)N[k] * L->rate[k];
  uint64_t target = (uint64_t)(((unsigned __int128)V * lam) >> 64);
  uint64_t below = 0;
  int ks = -1;
  for (int k = 0; k < NC3; ++k) {
    uint64_t w = (uint64_t)N[k] * L->rate[k];
    if (below + w > target) { ks = k; break; }
    below += w;
  }
  if (ks < 0) return -1;
  uint64_t idx = (target - below) / L->rate[ks], seen = 0;
  for (int lz = 0; lz < L->bz; ++lz)
    for (int ly = 0; ly < L->by; ++ly)
      for (int lx = 0; lx < L->bx; ++lx)
        if (l3_class(B, lx, ly, lz) == ks) {
          if (seen == idx) return (lz * L->by + ly) * L->bx + lx;
          seen++;
        }
  return -1;
}

typedef struct { uint64_t j, acc; int64_t anchor; } carry3_t;
typedef struct { int64_t n, cap, nbound; int64_t* tick; int64_t* site; } ev3_t;

static int ev3_push(ev3_t* e, int64_t t, int64_t v) {
  if (e->n == e->cap) {
    int64_t nc = e->cap ? 2 * e->cap : 64;
    int64_t* nt = (int64_t*)realloc(e->tick, sizeof(int64_t) * nc);
    if (!nt) return -1;
    e->tick = nt;
    int64_t* ns = (int64_t*)realloc(e->site, sizeof(int64_t) * nc);
    if (!ns) return -1;
    e->site = ns;
    e->cap = nc;
  }
  e->tick[e->n] = t; e->site[e->n] = v; e->n++;
  return 0;
}

static int sr3_local(const lat3_t* L, int d, const int8_t* committed, int64_t t_end, carry3_t cin,
                     const hl3_t* in[6], int8_t* blk_out, carry3_t* cout, hl3_t out[6], ev3_t* ev) {
  loc3_t B;
  int x0, y0, z0;
  sub3_origin(L, d, &x0, &y0, &z0);
  B.L = L;
  B.wrap[0] = L->nbx == 1; B.wrap[1] = L->nby == 1; B.wrap[2] = L->nbz == 1;
  B.blk = blk_out;
  int8_t fbuf[6][4096];
  for (int f = 0; f < 6; ++f) B.face[f] = fbuf[f];
  for (int lz = 0; lz < L->bz; ++lz)
    for (int ly = 0; ly < L->by; ++ly)
      for (int lx = 0; lx < L->bx; ++lx) {
        B.blk[(lz * L->by + ly) * L->bx + lx] = committed[gidx(L, x0 + lx, y0 + ly, z0 + lz)];
        if (lx == 0) {
          fbuf[FW][face_pos(L, FW, lx, ly, lz)] = committed[gidx(L, x0 - 1, y0 + ly, z0 + lz)];
          fbuf[FE][face_pos(L, FE, lx, ly, lz)] = committed[gidx(L, x0 + L->bx, y0 + ly, z0 + lz)];
        }
        if (ly == 0) {
          fbuf[FN][face_pos(L, FN, lx, ly, lz)] = committed[gidx(L, x0 + lx, y0 - 1, z0 + lz)];
          fbuf[FS][face_pos(L, FS, lx, ly, lz)] = committed[gidx(L, x0 + lx, y0 + L->by, z0 + lz)];
        }
        if (lz == 0) {
          fbuf[FD][face_pos(L, FD, lx, ly, lz)] = committed[gidx(L, x0 + lx, y0 + ly, z0 - 1)];
          fbuf[FU][face_pos(L, FU, lx, ly, lz)] = committed[gidx(L, x0 + lx, y0 + ly, z0 + L->bz)];
        }
      }
  for (int f = 0; f < 6; ++f) out[f].n = 0;
  ev->n = 0; ev->nbound = 0;
  uint64_t j = cin.j, acc = cin.acc, E, V;
  int64_t anchor = cin.anchor;
  draw3(L, d, j, &E, &V);
  uint64_t lam = l3_lambda(&B);
  int64_t next = next3(anchor, E, acc, lam);
  int64_t head[6] = {0, 0, 0, 0, 0, 0};
  for (;;) {
    int64_t tb = TICK_INF3;
    for (int f = 0; f < 6; ++f)
      if (in[f] && head[f] < in[f]->n && in[f]->tick[head[f]] < tb) tb = in[f]->tick[head[f]];
    if (next <= tb) {                           /* own event first on a tie */
      if (next >= t_end) break;
      int64_t t = next;
      int lv = l3_select(&B, V);
      if (lv < 0) return -3;
      int lx = lv % L->bx, ly = (lv / L->bx) % L->by, lz = lv / (L->bx * L->by);
      B.blk[lv] = (int8_t)(-B.blk[lv]);
      if (ev3_push(ev, t, gidx(L, x0 + lx, y0 + ly, z0 + lz))) return -2;
      int onb = 0;
      if (!B.wrap[0] && lx == 0)          { if (hl3_push(&out[FW], t, face_pos(L, FW, lx, ly, lz))) return -2; onb = 1; }
      if (!B.wrap[0] && lx == L->bx - 1)  { if (hl3_push(&out[FE], t, face_pos(L, FE, lx, ly, lz))) return -2; onb = 1; }
      if (!B.wrap[1] && ly == 0)          { if (hl3_push(&out[FN], t, face_pos(L, FN, lx, ly, lz))) return -2; onb = 1; }
      if (!B.wrap[1] && ly == L->by - 1)  { if (hl3_push(&out[FS], t, face_pos(L, FS, lx, ly, lz))) return -2; onb = 1; }
      if (!B.wrap[2] && lz == 0)          { if (hl3_push(&out[FD], t, face_pos(L, FD, lx, ly, lz))) return -2; onb = 1; }
      if (!B.wrap[2] && lz == L->bz - 1)  { if (hl3_push(&out[FU], t, face_pos(L, FU, lx, ly, lz))) return -2; onb = 1; }
      ev->nbound += onb;
      j += 1; anchor = t; acc = 0;
      draw3(L, d, j, &E, &V);
      lam = l3_lambda(&B);
      next = next3(anchor, E, acc, lam);
    } else {                                    /* a neighbour's face flip */
      if (tb >= t_end) break;
      int64_t t = tb;
      for (int f = 0; f < 6; ++f)
        if (in[f] && head[f] < in[f]->n && in[f]->tick[head[f]] == t) {
          int32_t pos = in[f]->pos[head[f]];
          B.face[f][pos] = (int8_t)(-B.face[f][pos]);
          head[f]++;
          break;
        }
      acc += lam * (uint64_t)(t - anchor);
      anchor = t;
      lam = l3_lambda(&B);
      next = next3(anchor, E, acc, lam);
    }
  }
  cout->j = j; cout->acc = acc; cout->anchor = anchor;
  return 0;
}

int orc3_sr_run(const orc3_params* p, orc_result* r, int32_t* g_out, int32_t* f_out, int32_t max_iters) {
  lat3_t L;
  if (lat3_init(&L, p) != 0) return -1;
  int8_t* s = r->spins;
  if (init3_spins(&L, p, s) != 0) return -1;
  int nsub = L.nsub;
  int64_t nblk = (int64_t)L.bx * L.by * L.bz;
  carry3_t* carry = (carry3_t*)calloc((size_t)nsub, sizeof(carry3_t));
  carry3_t* cwork = (carry3_t*)calloc((size_t)nsub, sizeof(carry3_t));
  int8_t* blk = (int8_t*)malloc((size_t)(nsub * nblk));
  hl3_t* lists[2];
  lists[0] = (hl3_t*)calloc((size_t)nsub * 6, sizeof(hl3_t));
  lists[1] = (hl3_t*)calloc((size_t)nsub * 6, sizeof(hl3_t));
  ev3_t* ev = (ev3_t*)calloc((size_t)nsub, sizeof(ev3_t));
  hl3_t empty = {0, 0, 0, 0};
  if (!carry || !cwork || !blk || !lists[0] || !lists[1] || !ev) return -2;
  if (max_iters <= 0) max_iters = 10000;
  int64_t nev = 0;
  for (int d = 0; d < nsub; ++d) {
    if (r->sub_flips) r->sub_flips[d] = 0;
    if (r->sub_digest) r->sub_digest[d] = 0;
  }
  int64_t nwin = p->horizon_ticks == 0 ? 0 : (p->horizon_ticks + p->window_ticks - 1) / p->window_ticks;
  if (r->snap_M) observe3(&L, s, &r->snap_M[0], &r->snap_bond[0]);
  /* the face of neighbour e that borders my face f */
  const int opposite[6] = {FE, FW, FS, FN, FU, FD};
  for (int64_t w = 0; w < nwin; ++w) {
    int64_t t_c = w * p->window_ticks;
    int64_t t_end = t_c + p->window_ticks;
    if (t_end > p->horizon_ticks) t_end = p->horizon_ticks;
    if (p->step_rule == ORC_STEP_WIPE && t_c > 0)
      for (int d = 0; d < nsub; ++d) { carry[d].j += 1; carry[d].anchor = t_c; carry[d].acc = 0; }
    int it, converged = 0, fmax = 0;
    for (it = 0; it < max_iters; ++it) {
      int cur = it & 1, prev = cur ^ 1;
      for (int d = 0; d < nsub; ++d) {
        int cx = d % L.nbx, cy = (d / L.nbx) % L.nby, cz = d / (L.nbx * L.nby);
        int nb[6];
        nb[FW] = (cz * L.nby + cy) * L.nbx + wrap3(cx - 1, L.nbx);
        nb[FE] = (cz * L.nby + cy) * L.nbx + wrap3(cx + 1, L.nbx);
        nb[FN] = (cz * L.nby + wrap3(cy - 1, L.nby)) * L.nbx + cx;
        nb[FS] = (cz * L.nby + wrap3(cy + 1, L.nby)) * L.nbx + cx;
        nb[FD] = (wrap3(cz - 1, L.nbz) * L.nby + cy) * L.nbx + cx;
        nb[FU] = (wrap3(cz + 1, L.nbz) * L.nby + cy) * L.nbx + cx;
        const hl3_t* in[6];
        for (int f = 0; f < 6; ++f) {
          int dim = f / 2;
          int wraps = dim == 0 ? L.nbx == 1 : dim == 1 ? L.nby == 1 : L.nbz == 1;
          if (wraps) in[f] = NULL;
          else in[f] = it == 0 ? &empty : &lists[prev][6 * nb[f] + opposite[f]];
        }
        int rc = sr3_local(&L, d, s, t_end, carry[d], in, blk + d * nblk, &cwork[d], &lists[cur][6 * d], &ev[d]);
        if (rc) return rc;
        if (ev[d].nbound > fmax) fmax = (int)ev[d].nbound;
      }
      int changed = 0;
      for (int q = 0; q < 6 * nsub && !changed; ++q) {
        const hl3_t* old = it == 0 ? &empty : &lists[prev][q];
        if (!hl3_equal(&lists[cur][q], old)) changed = 1;
      }
      if (!changed) { converged = 1; break; }
    }
    if (!converged) return -5;
    if (g_out) g_out[w] = it + 1;
    if (f_out) f_out[w] = fmax;
    for (int d = 0; d < nsub; ++d) {
      int x0, y0, z0;
      sub3_origin(&L, d, &x0, &y0, &z0);
      for (int lz = 0; lz < L.bz; ++lz)
        for (int ly = 0; ly < L.by; ++ly)
          for (int lx = 0; lx < L.bx; ++lx)
            s[gidx(&L, x0 + lx, y0 + ly, z0 + lz)] = blk[d * nblk + (lz * L.by + ly) * L.bx + lx];
      carry[d] = cwork[d];
    }
    {
      int64_t* hd = (int64_t*)calloc((size_t)nsub, sizeof(int64_t));
      for (;;) {
        int best = -1;
        for (int d = 0; d < nsub; ++d)
          if (hd[d] < ev[d].n && (best < 0 || ev[d].tick[hd[d]] < ev[best].tick[hd[best]])) best = d;
        if (best < 0) break;
        int64_t t = ev[best].tick[hd[best]], v = ev[best].site[hd[best]];
        if (nev < r->log_cap) { r->log_tick[nev] = t; r->log_site[nev] = v; r->log_sub[nev] = best; }
        nev++;
        if (r->sub_flips) r->sub_flips[best]++;
        if (r->sub_digest) r->sub_digest[best] += orc_event_digest(t, v);
        hd[best]++;
      }
      free(hd);
    }
    if (r->snap_M) observe3(&L, s, &r->snap_M[w + 1], &r->snap_bond[w + 1]);
  }
  r->n_events = nev;
  observe3(&L, s, &r->M, &r->bond);
  if (r->carry)
    for (int d = 0; d < nsub; ++d) {
      uint64_t E, V;
      int64_t N[NC3];
      draw3(&L, d, carry[d].j, &E, &V);
      uint64_t lam = sub3_lambda(&L, s, d, N);
      r->carry[4 * d + 0] = (int64_t)carry[d].j;
      r->carry[4 * d + 1] = carry[d].anchor;
      r->carry[4 * d + 2] = (int64_t)carry[d].acc;
      r->carry[4 * d + 3] = next3(carry[d].anchor, E, carry[d].acc, lam);
    }
  for (int q = 0; q < 6 * nsub; ++q) {
    free(lists[0][q].tick); free(lists[0][q].pos);
    free(lists[1][q].tick); free(lists[1][q].pos);
  }
  for (int d = 0; d < nsub; ++d) { free(ev[d].tick); free(ev[d].site); }
  free(lists[0]); free(lists[1]); free(ev); free(carry); free(cwork); free(blk);
  return 0;
}
