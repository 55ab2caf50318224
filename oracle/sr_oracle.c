/*
 * sr_oracle.c -- CPU oracle for synchronous relaxation (SR) of the
 * continuous-time n-fold way Ising simulation (Lubachevsky & Weiss,
 * "Synchronous relaxation for parallel Ising spin simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * shares no code with it: no headers, no helpers, no tables, no constant
 * generators.  Everything here is plain single-threaded C99, written for
 * reading rather than speed.
 *
 * What it computes.  By the paper's consistency argument (Sec. 4: the
 * iteration stops only when every PE's assumed neighbour history equals the
 * generated one, and then the histories are the correct ones; random numbers
 * are treated as a presimulated list and reused), the converged result of
 * SR is the trajectory of a plain sequential discrete-event simulation (DES)
 * that merges all subdomains' n-fold-way event streams in global time order.
 * `orc_des_run` is that DES.  `orc_sr_run` is a literal CPU rendering of the
 * Sec. 4 iteration box (Jacobi: every subdomain reads its neighbours'
 * previous-iteration boundary histories, canonical "no change" assumption in
 * iteration 0, repeat until no history changes, then advance committed
 * time), used to pin the DES against the paper's iteration and to give the
 * exact iteration counts g of every window.
 *
 * Integer conventions (the paper works with real numbers; these readings make
 * "identical trajectory" well defined):
 *  - time in ticks of 2^-tick_bits (attempt rate lambda = 1, k_B = 1);
 *  - rates r_k = round(2^28 p_k) for the 10 classes of Sec. 3 (class
 *    k = 5*[s=-1] + number of up neighbours), p from eq. pMin (Metropolis) or
 *    eq. pglauber (Glauber), energy change from eq. hamil with every
 *    nearest-neighbour bond counted once;
 *  - Lambda = sum_k N_k r_k (eq. biglambda, in units of 2^-28 per time unit);
 *  - -log U of eq. nextau as a Q(28+tick_bits) integer E (fixed-point binary
 *    logarithm by repeated squaring, times ln 2);
 *  - eq. lambdataua solved exactly on the tick grid: the event falls on the
 *    first tick t at which the integrated hazard sum_{u<t} Lambda(u) reaches E,
 *    Lambda(u) being the rate in force during tick u (after all flips at
 *    ticks <= u);
 *  - class and site choice (eqs. Wsum, Wstop, nores, vindex) as one integer
 *    target = floor(V * Lambda / 2^64) in [0, Lambda): the class is the first
 *    k whose cumulative weight exceeds the target, the site is the
 *    floor((target - C_{k-1}) / r_k)-th member of that class in ascending
 *    local row-major order;
 *  - random pairs (U_i, V_i) of subdomain d, event index i, from Philox-4x32-10
 *    (Salmon, Moraes, Dror, Shaw, SC'11) with key = seed and counter
 *    (i mod 2^32, i >> 32, d, 0); initial spins from counter (site, 0, 1);
 *  - simultaneous events (same tick, different subdomains) all choose their
 *    site from the state before that tick;
 *  - windows are half open [t_c, t_c + W); the window edge is not a break
 *    point: the pending draw and its integrated hazard carry over (Sec. 5,
 *    "Subsequent steps"), so the trajectory does not depend on W;
 *  - or, with ORC_STEP_WIPE (Sec. 5, "An alternate approach to subsequent
 *    steps"), every step start t_c > 0 empties every subdomain's pending
 *    event: the pending pair is discarded, the next pair of the subdomain's
 *    list (one later than any used so far) is drawn, and its hazard starts
 *    at t_c.  Poisson memorylessness keeps this unbiased; the trajectory
 *    then depends on W.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "sr_oracle.h"

#define NCLS 10
#define RATE_ONE (1u << 28)
#define TICK_INF INT64_MAX

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10, from its published definition (Salmon et al., SC'11):     */
/* ten rounds of two 32x32->64 multiplications with the round function        */
/* (c0,c1,c2,c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,       */
/* lo(M0*c0)), the key bumped by the Weyl constants between rounds.           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t key_in[2], const uint32_t ctr_in[4],
                       uint32_t out[4]) {
  uint32_t k0 = key_in[0], k1 = key_in[1];
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* -log U in fixed point.  U = m / 2^64 with m = u | 1 (so U is in (0,1)).    */
/* log2 m = e + log2 y, y = m / 2^e in [1,2).  The bits of log2 y come from   */
/* repeated squaring: y^2 >= 2 gives a 1 bit and y <- y^2/2, else a 0 bit.    */
/* y is carried as a Q1.31 integer, truncated after every squaring.           */
/* -log2 U = (64 - e) - frac/2^32 as a Q32 integer Lq; then -ln U = Lq ln 2,  */
/* returned in units of 2^-(28+tick_bits) (the hazard unit).                  */
/* ------------------------------------------------------------------------ */
#define LN2_Q64 0xB17217F7D1CF79ABull /* floor(ln 2 * 2^64) */

uint64_t orc_expq(uint64_t u, int tick_bits) {
  uint64_t m = u | 1u;
  int c = 0;
  while (((m << c) >> 63) == 0) c++;           /* leading zeros */
  int e = 63 - c;
  uint32_t z = (uint32_t)((m << c) >> 32);     /* Q1.31, in [2^31, 2^32) */
  uint64_t frac = 0;
  for (int i = 0; i < 32; ++i) {
    uint64_t q = (uint64_t)z * (uint64_t)z;    /* Q2.62 */
    if (q >= (1ull << 63)) {
      frac = (frac << 1) | 1u;
      z = (uint32_t)(q >> 32);
    } else {
      frac = frac << 1;
      z = (uint32_t)(q >> 31);
    }
  }
  uint64_t lq = ((uint64_t)(64 - e) << 32) - frac;
  unsigned __int128 prod = (unsigned __int128)lq * (unsigned __int128)LN2_Q64;
  int shift = 96 - (28 + tick_bits);
  return (uint64_t)(prod >> shift);
}

/* ------------------------------------------------------------------------ */
/* Rate table, eqs. hamil / pMin / pglauber.  Class k = 5*[s=-1] + n_up.      */
/* Flipping s changes E by dE = 2 s (J sum_nn s' + h), sum_nn s' = 2 n_up - 4.*/
/* ------------------------------------------------------------------------ */
int orc_rate_table(double J, double h, double T, int rule, uint32_t out[NCLS]) {
  if (!(T > 0.0) || (rule != ORC_METROPOLIS && rule != ORC_GLAUBER)) return -1;
  for (int k = 0; k < NCLS; ++k) {
    int s = (k < 5) ? 1 : -1;
    int nup = k % 5;
    double x = -(2.0 * s * (J * (2 * nup - 4) + h)) / T; /* -dE / T */
    double p;
    if (rule == ORC_METROPOLIS) {
      double theta = exp(x);
      p = theta < 1.0 ? theta : 1.0;
    } else {
      p = 1.0 / (1.0 + exp(-x));              /* theta / (1 + theta) */
    }
    double q = nearbyint(ldexp(p, 28));
    if (q > (double)RATE_ONE) q = (double)RATE_ONE;
    out[k] = (uint32_t)q;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers (shared by the DES and the literal SR below).             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int Lx, Ly, bx, by, nbx, nby, nsub;
  uint32_t rate[NCLS];
  uint64_t seed;
  int tick_bits;
} lat_t;

static int lat_init(lat_t* L, const orc_params* p) {
  if (p->Lx < 2 || p->Ly < 2 || p->bx < 1 || p->by < 1) return -1;
  if (p->Lx % p->bx || p->Ly % p->by) return -1;
  if (p->tick_bits < 1 || p->tick_bits > 28) return -1;
  if (p->window_ticks < 1 || p->horizon_ticks < 0) return -1;
  if (p->step_rule != ORC_STEP_CONTINUE && p->step_rule != ORC_STEP_WIPE) return -1;
  if ((int64_t)p->bx * p->by > 4096) return -1;
  L->Lx = p->Lx; L->Ly = p->Ly; L->bx = p->bx; L->by = p->by;
  L->nbx = p->Lx / p->bx; L->nby = p->Ly / p->by;
  L->nsub = L->nbx * L->nby;
  L->seed = p->seed;
  L->tick_bits = p->tick_bits;
  return orc_rate_table(p->J, p->h, p->T, p->rule, L->rate);
}

static int wrapi(int a, int n) { return ((a % n) + n) % n; }

static int sub_of_site(const lat_t* L, int x, int y) {
  return (y / L->by) * L->nbx + (x / L->bx);
}

/* Initial spins: Philox counter (site lo, site hi, 0, 1), s = +1 iff x0 odd. */
static int init_spins(const lat_t* L, const orc_params* p, int8_t* s) {
  int64_t n = (int64_t)L->Lx * L->Ly;
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

/* The (E, V) pair of subdomain d, event index j. */
static void draw(const lat_t* L, int d, uint64_t j, uint64_t* E, uint64_t* V) {
  uint32_t key[2] = {(uint32_t)L->seed, (uint32_t)(L->seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), (uint32_t)d, 0u};
  uint32_t o[4];
  orc_philox4x32_10(key, ctr, o);
  uint64_t u = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
  *V = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
  *E = orc_expq(u, L->tick_bits);
}

/* next tick = anchor + max(1, ceil((E - acc) / lam)), or never if lam = 0. */
static int64_t next_tick(int64_t anchor, uint64_t E, uint64_t acc, uint64_t lam) {
  if (lam == 0) return TICK_INF;
  uint64_t rem = E - acc;
  uint64_t q = rem / lam + (rem % lam != 0);
  if (q < 1) q = 1;
  if (q > (uint64_t)(TICK_INF - anchor)) return TICK_INF;
  return anchor + (int64_t)q;
}

/* Digest of one committed event: order-free sum of a 64-bit mix (SplitMix64
 * finaliser, Steele, Lea & Flood 2014) of (tick, global site). */
uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t orc_event_digest(int64_t tick, int64_t site) {
  return orc_mix64(orc_mix64((uint64_t)tick) + (uint64_t)site);
}

/* Whole-lattice observables from scratch: M = sum s, bond = sum over right
 * and down bonds of s s'. */
static void observe(const lat_t* L, const int8_t* s, int64_t* M, int64_t* bond) {
  int64_t m = 0, b = 0;
  for (int y = 0; y < L->Ly; ++y)
    for (int x = 0; x < L->Lx; ++x) {
      int v = s[(int64_t)y * L->Lx + x];
      m += v;
      b += v * s[(int64_t)y * L->Lx + wrapi(x + 1, L->Lx)];
      b += v * s[(int64_t)wrapi(y + 1, L->Ly) * L->Lx + x];
    }
  *M = m;
  *bond = b;
}

/* ======================================================================== */
/* DES: all subdomains' event streams merged in global tick order.          */
/* ======================================================================== */
typedef struct {
  uint64_t j, acc, E, V, lam;
  int64_t anchor, next;
} sub_t;

static int class_of(const lat_t* L, const int8_t* s, int x, int y) {
  int up = 0;
  up += s[(int64_t)y * L->Lx + wrapi(x + 1, L->Lx)] > 0;
  up += s[(int64_t)y * L->Lx + wrapi(x - 1, L->Lx)] > 0;
  up += s[(int64_t)wrapi(y + 1, L->Ly) * L->Lx + x] > 0;
  up += s[(int64_t)wrapi(y - 1, L->Ly) * L->Lx + x] > 0;
  return 5 * (s[(int64_t)y * L->Lx + x] < 0) + up;
}

/* Lambda of subdomain d and its class counts, by a full scan. */
static uint64_t sub_lambda(const lat_t* L, const int8_t* s, int d, int64_t N[NCLS]) {
  int x0 = (d % L->nbx) * L->bx, y0 = (d / L->nbx) * L->by;
  for (int k = 0; k < NCLS; ++k) N[k] = 0;
  for (int ly = 0; ly < L->by; ++ly)
    for (int lx = 0; lx < L->bx; ++lx) N[class_of(L, s, x0 + lx, y0 + ly)]++;
  uint64_t lam = 0;
  for (int k = 0; k < NCLS; ++k) lam += (uint64_t)N[k] * L->rate[k];
  return lam;
}

/* Phases 2 and 3 of Sec. 3 on integers: returns the global site index. */
static int64_t select_site(const lat_t* L, const int8_t* s, int d, uint64_t V) {
  int64_t N[NCLS];
  uint64_t lam = sub_lambda(L, s, d, N);
  uint64_t target = (uint64_t)(((unsigned __int128)V * lam) >> 64);
  uint64_t below = 0;
  int ks = -1;
  for (int k = 0; k < NCLS; ++k) {
    uint64_t w = (uint64_t)N[k] * L->rate[k];
    if (below + w > target) { ks = k; break; }
    below += w;
  }
  if (ks < 0) return -1;
  uint64_t idx = (target - below) / L->rate[ks];
  int x0 = (d % L->nbx) * L->bx, y0 = (d / L->nbx) * L->by;
  uint64_t seen = 0;
  for (int ly = 0; ly < L->by; ++ly)
    for (int lx = 0; lx < L->bx; ++lx)
      if (class_of(L, s, x0 + lx, y0 + ly) == ks) {
        if (seen == idx) return (int64_t)(y0 + ly) * L->Lx + (x0 + lx);
        seen++;
      }
  return -1;
}

int orc_select_site(const orc_params* p, const int8_t* spins, int d, uint64_t V,
                    int64_t* site_out) {
  lat_t L;
  if (lat_init(&L, p) != 0 || d < 0 || d >= L.nsub) return -1;
  int64_t v = select_site(&L, spins, d, V);
  if (v < 0) return -2;
  *site_out = v;
  return 0;
}

int orc_subdomain_lambda(const orc_params* p, const int8_t* spins, int d,
                         uint64_t* lam_out) {
  lat_t L;
  int64_t N[NCLS];
  if (lat_init(&L, p) != 0 || d < 0 || d >= L.nsub) return -1;
  *lam_out = sub_lambda(&L, spins, d, N);
  return 0;
}

/* Segment tree over next ticks: leaf i holds (next_i, i); a node holds the
 * smaller pair. */
typedef struct { int n; int64_t* key; int* idx; } tree_t;

static int tree_init(tree_t* T, int n) {
  int m = 1;
  while (m < n) m <<= 1;
  T->n = m;
  T->key = (int64_t*)malloc(sizeof(int64_t) * 2 * m);
  T->idx = (int*)malloc(sizeof(int) * 2 * m);
  if (!T->key || !T->idx) return -1;
  for (int i = 0; i < 2 * m; ++i) { T->key[i] = TICK_INF; T->idx[i] = -1; }
  for (int i = 0; i < m; ++i) T->idx[m + i] = i;
  return 0;
}
static void tree_set(tree_t* T, int i, int64_t key) {
  int p = T->n + i;
  T->key[p] = key;
  for (p >>= 1; p >= 1; p >>= 1) {
    int a = 2 * p, b = 2 * p + 1;
    int pick = (T->key[b] < T->key[a]) ? b : a;
    T->key[p] = T->key[pick];
    T->idx[p] = T->idx[pick];
  }
}
static void tree_free(tree_t* T) { free(T->key); free(T->idx); }

static int cmp_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

int orc_des_run(const orc_params* p, orc_result* r) {
  lat_t L;
  if (lat_init(&L, p) != 0) return -1;
  int64_t nsite = (int64_t)L.Lx * L.Ly;
  int8_t* s = r->spins; /* caller-owned, Ly*Lx */
  if (!s) return -1;
  if (init_spins(&L, p, s) != 0) return -1;

  sub_t* sub = (sub_t*)calloc((size_t)L.nsub, sizeof(sub_t));
  int* S = (int*)malloc(sizeof(int) * L.nsub);
  int64_t* vsel = (int64_t*)malloc(sizeof(int64_t) * L.nsub);
  int* aff = (int*)malloc(sizeof(int) * 5 * L.nsub);
  char* inS = (char*)calloc((size_t)L.nsub, 1);
  tree_t T;
  if (!sub || !S || !vsel || !aff || !inS || tree_init(&T, L.nsub) != 0) return -2;

  for (int d = 0; d < L.nsub; ++d) {
    int64_t N[NCLS];
    sub[d].j = 0; sub[d].anchor = 0; sub[d].acc = 0;
    draw(&L, d, 0, &sub[d].E, &sub[d].V);
    sub[d].lam = sub_lambda(&L, s, d, N);
    sub[d].next = next_tick(0, sub[d].E, 0, sub[d].lam);
    tree_set(&T, d, sub[d].next);
  }

  int64_t M, bond;
  observe(&L, s, &M, &bond);
  int64_t nwin = p->horizon_ticks == 0 ? 0
               : (p->horizon_ticks + p->window_ticks - 1) / p->window_ticks;
  int64_t snap = 0;           /* next committed-time snapshot index */
  int64_t nev = 0;
  double iM = 0, iM2 = 0, iabsM = 0, ibond = 0, iE2 = 0, iM4 = 0;
  int64_t t_last = p->burn_ticks;  /* integration start */
  double Jd = p->J, hd = p->h;

  for (int d = 0; d < L.nsub; ++d) {
    if (r->sub_flips) r->sub_flips[d] = 0;
    if (r->sub_digest) r->sub_digest[d] = 0;
  }

  int64_t next_wipe = p->window_ticks;   /* next step start (wipe rule) */
  for (;;) {
    int64_t t = T.key[1];
    int64_t stop = p->horizon_ticks;
    /* wipe rule: at each step start t_c in (0, horizon) reached before the
     * next event, every subdomain forgets its pending event and draws its
     * next pair afresh, with the hazard counted from t_c */
    while (p->step_rule == ORC_STEP_WIPE && next_wipe < stop && next_wipe <= t) {
      for (int d = 0; d < L.nsub; ++d) {
        sub[d].j += 1;
        sub[d].anchor = next_wipe;
        sub[d].acc = 0;
        draw(&L, d, sub[d].j, &sub[d].E, &sub[d].V);
        sub[d].next = next_tick(next_wipe, sub[d].E, 0, sub[d].lam);
        tree_set(&T, d, sub[d].next);
      }
      next_wipe += p->window_ticks;
      t = T.key[1];
    }
    int64_t t_eff = t < stop ? t : stop;
    /* committed-time snapshots: state after all flips with tick < k W */
    while (snap <= nwin) {
      int64_t tc = snap * p->window_ticks;
      if (tc > stop) tc = stop;
      if (tc > t_eff) break;
      if (r->snap_M) { int64_t m2, b2; observe(&L, s, &m2, &b2);
                       r->snap_M[snap] = m2; r->snap_bond[snap] = b2; }
      snap++;
    }
    /* time integrals of observables over [burn, horizon) */
    if (t_eff > t_last) {
      double dt = (double)(t_eff - t_last);
      double e = -Jd * (double)bond - hd * (double)M;
      iM += dt * M; iM2 += dt * (double)M * M; iabsM += dt * (M < 0 ? -M : M);
      ibond += dt * bond; iE2 += dt * e * e;
      iM4 += dt * (double)M * M * (double)M * M;
      t_last = t_eff;
    }
    if (t >= stop) break;

    /* S = subdomains with an event at tick t, ascending id */
    int nS = 0;
    while (T.key[1] == t) {                 /* every key equal to t */
      S[nS++] = T.idx[1];
      tree_set(&T, T.idx[1], TICK_INF);     /* restored below: S is affected */
    }
    qsort(S, (size_t)nS, sizeof(int), cmp_int);
    /* all of them choose from the state before tick t */
    for (int a = 0; a < nS; ++a) {
      vsel[a] = select_site(&L, s, S[a], sub[S[a]].V);
      if (vsel[a] < 0) return -3;
    }
    int naff = 0;
    for (int a = 0; a < nS; ++a) {
      int d = S[a];
      int64_t v = vsel[a];
      int x = (int)(v % L.Lx), y = (int)(v / L.Lx);
      int old = s[v];
      s[v] = (int8_t)(-old);
      /* incremental observables (checked against full scans at snapshots) */
      int nn = s[(int64_t)y * L.Lx + wrapi(x + 1, L.Lx)] + s[(int64_t)y * L.Lx + wrapi(x - 1, L.Lx)]
             + s[(int64_t)wrapi(y + 1, L.Ly) * L.Lx + x] + s[(int64_t)wrapi(y - 1, L.Ly) * L.Lx + x];
      M += -2 * old;
      bond += -2 * old * nn;
      if (nev < r->log_cap) {
        r->log_tick[nev] = t; r->log_site[nev] = v; r->log_sub[nev] = d;
      }
      nev++;
      if (r->sub_flips) r->sub_flips[d]++;
      if (r->sub_digest) r->sub_digest[d] += orc_event_digest(t, v);
      aff[naff++] = d;
      aff[naff++] = sub_of_site(&L, wrapi(x + 1, L.Lx), y);
      aff[naff++] = sub_of_site(&L, wrapi(x - 1, L.Lx), y);
      aff[naff++] = sub_of_site(&L, x, wrapi(y + 1, L.Ly));
      aff[naff++] = sub_of_site(&L, x, wrapi(y - 1, L.Ly));
    }
    for (int a = 0; a < nS; ++a) inS[S[a]] = 1;
    qsort(aff, (size_t)naff, sizeof(int), cmp_int);
    for (int a = 0; a < naff; ++a) {
      int e = aff[a];
      if (a > 0 && aff[a - 1] == e) continue;
      int64_t N[NCLS];
      if (inS[e]) {                         /* own event: fresh draw */
        sub[e].j += 1;
        sub[e].anchor = t;
        sub[e].acc = 0;
        draw(&L, e, sub[e].j, &sub[e].E, &sub[e].V);
      } else {                              /* break point: fold hazard */
        sub[e].acc += sub[e].lam * (uint64_t)(t - sub[e].anchor);
        sub[e].anchor = t;
      }
      sub[e].lam = sub_lambda(&L, s, e, N);
      sub[e].next = next_tick(sub[e].anchor, sub[e].E, sub[e].acc, sub[e].lam);
      tree_set(&T, e, sub[e].next);
    }
    for (int a = 0; a < nS; ++a) inS[S[a]] = 0;
  }

  r->n_events = nev;
  r->M = M; r->bond = bond;
  r->int_M = iM; r->int_M2 = iM2; r->int_absM = iabsM; r->int_bond = ibond;
  r->int_E2 = iE2; r->int_M4 = iM4;
  r->int_ticks = (p->horizon_ticks > p->burn_ticks) ? (p->horizon_ticks - p->burn_ticks) : 0;
  if (r->carry) {
    for (int d = 0; d < L.nsub; ++d) {
      r->carry[4 * d + 0] = (int64_t)sub[d].j;
      r->carry[4 * d + 1] = sub[d].anchor;
      r->carry[4 * d + 2] = (int64_t)sub[d].acc;
      r->carry[4 * d + 3] = sub[d].next;
    }
  }
  {
    int64_t m2, b2;
    observe(&L, s, &m2, &b2);
    if (m2 != M || b2 != bond) return -4;   /* incremental bookkeeping broke */
  }
  tree_free(&T);
  free(sub); free(S); free(vsel); free(aff); free(inS);
  (void)nsite;
  return 0;
}

/* ======================================================================== */
/* Literal synchronous relaxation (Sec. 4 box, Sec. 5 details) on the CPU.   */
/* Each subdomain is simulated alone over [t_c, t_end) from the committed    */
/* state, reading neighbour boundary flips of the previous iteration as      */
/* break points.  Boundary history lists per edge: N = top row, S = bottom   */
/* row, W = left column, E = right column; an entry is (tick, position).     */
/* ======================================================================== */
enum { EN = 0, ES = 1, EW = 2, EE = 3 };

typedef struct { int64_t* tick; int32_t* pos; int64_t n, cap; } hlist_t;

static int hl_push(hlist_t* h, int64_t t, int32_t pos) {
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
static int hl_equal(const hlist_t* a, const hlist_t* b) {
  if (a->n != b->n) return 0;
  for (int64_t i = 0; i < a->n; ++i)
    if (a->tick[i] != b->tick[i] || a->pos[i] != b->pos[i]) return 0;
  return 1;
}

/* One subdomain's local view: block spins plus a one-site halo.  A direction
 * whose neighbour is the subdomain itself (the block spans the torus in that
 * direction) wraps inside the block and has no halo. */
typedef struct {
  const lat_t* L;
  int d, x0, y0;
  int wrapx, wrapy;
  int8_t* blk;               /* by*bx */
  int8_t *hN, *hS, *hW, *hE; /* halos: above, below, left, right */
} local_t;

static int l_spin(const local_t* B, int lx, int ly) {
  const lat_t* L = B->L;
  if (lx >= 0 && lx < L->bx && ly >= 0 && ly < L->by) return B->blk[ly * L->bx + lx];
  if (ly < 0) return B->wrapy ? B->blk[(L->by - 1) * L->bx + lx] : B->hN[lx];
  if (ly >= L->by) return B->wrapy ? B->blk[lx] : B->hS[lx];
  if (lx < 0) return B->wrapx ? B->blk[ly * L->bx + L->bx - 1] : B->hW[ly];
  return B->wrapx ? B->blk[ly * L->bx] : B->hE[ly];
}
static int l_class(const local_t* B, int lx, int ly) {
  int up = (l_spin(B, lx + 1, ly) > 0) + (l_spin(B, lx - 1, ly) > 0)
         + (l_spin(B, lx, ly + 1) > 0) + (l_spin(B, lx, ly - 1) > 0);
  return 5 * (l_spin(B, lx, ly) < 0) + up;
}
static uint64_t l_lambda(const local_t* B, int64_t N[NCLS]) {
  const lat_t* L = B->L;
  for (int k = 0; k < NCLS; ++k) N[k] = 0;
  for (int ly = 0; ly < L->by; ++ly)
    for (int lx = 0; lx < L->bx; ++lx) N[l_class(B, lx, ly)]++;
  uint64_t lam = 0;
  for (int k = 0; k < NCLS; ++k) lam += (uint64_t)N[k] * L->rate[k];
  return lam;
}
static int l_select(const local_t* B, uint64_t V) {
  const lat_t* L = B->L;
  int64_t N[NCLS];
  uint64_t lam = l_lambda(B, N);
  uint64_t target = (uint64_t)(((unsigned __int128)V * lam) >> 64);
  uint64_t below = 0;
  int ks = -1;
  for (int k = 0; k < NCLS; ++k) {
    uint64_t w = (uint64_t)N[k] * L->rate[k];
    if (below + w > target) { ks = k; break; }
    below += w;
  }
  if (ks < 0) return -1;
  uint64_t idx = (target - below) / L->rate[ks];
  uint64_t seen = 0;
  for (int ly = 0; ly < L->by; ++ly)
    for (int lx = 0; lx < L->bx; ++lx)
      if (l_class(B, lx, ly) == ks) {
        if (seen == idx) return ly * L->bx + lx;
        seen++;
      }
  return -1;
}

typedef struct { uint64_t j, acc; int64_t anchor; } carry_t;

typedef struct {
  int64_t n;           /* events of this window */
  int64_t* tick; int64_t* site; int64_t cap;
  int64_t nbound;      /* own events on boundary sites (f statistic) */
} evlog_t;

static int ev_push(evlog_t* e, int64_t t, int64_t v) {
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

/* Simulate subdomain d over [t_c, t_end).  in[EN] holds the flips of the
 * halo row above (the north neighbour's bottom row), in[ES] the row below,
 * in[EW] the column to the left, in[EE] the column to the right.  Writes the
 * end-of-window block spins, carry and own boundary lists. */
static int sr_local(const lat_t* L, int d, const int8_t* committed,
                    int64_t t_c, int64_t t_end, carry_t cin,
                    const hlist_t* in[4], int8_t* blk_out, carry_t* cout,
                    hlist_t out[4], evlog_t* ev) {
  local_t B;
  (void)t_c;  /* the committed state already is the state at t_c */
  B.L = L; B.d = d;
  B.x0 = (d % L->nbx) * L->bx; B.y0 = (d / L->nbx) * L->by;
  B.wrapx = (L->nbx == 1); B.wrapy = (L->nby == 1);
  B.blk = blk_out;
  int8_t hN[4096], hS[4096], hW[4096], hE[4096];
  B.hN = hN; B.hS = hS; B.hW = hW; B.hE = hE;
  for (int ly = 0; ly < L->by; ++ly)
    for (int lx = 0; lx < L->bx; ++lx)
      B.blk[ly * L->bx + lx] = committed[(int64_t)(B.y0 + ly) * L->Lx + B.x0 + lx];
  for (int lx = 0; lx < L->bx; ++lx) {
    hN[lx] = committed[(int64_t)wrapi(B.y0 - 1, L->Ly) * L->Lx + B.x0 + lx];
    hS[lx] = committed[(int64_t)wrapi(B.y0 + L->by, L->Ly) * L->Lx + B.x0 + lx];
  }
  for (int ly = 0; ly < L->by; ++ly) {
    hW[ly] = committed[(int64_t)(B.y0 + ly) * L->Lx + wrapi(B.x0 - 1, L->Lx)];
    hE[ly] = committed[(int64_t)(B.y0 + ly) * L->Lx + wrapi(B.x0 + L->bx, L->Lx)];
  }
  for (int e = 0; e < 4; ++e) out[e].n = 0;
  ev->n = 0; ev->nbound = 0;

  uint64_t j = cin.j, acc = cin.acc;
  int64_t anchor = cin.anchor;
  uint64_t E, V;
  draw(L, d, j, &E, &V);
  int64_t N[NCLS];
  uint64_t lam = l_lambda(&B, N);
  int64_t next = next_tick(anchor, E, acc, lam);
  int64_t head[4] = {0, 0, 0, 0};

  for (;;) {
    /* earliest pending break point over the four input lists */
    int64_t tb = TICK_INF;
    for (int e = 0; e < 4; ++e)
      if (in[e] && head[e] < in[e]->n && in[e]->tick[head[e]] < tb) tb = in[e]->tick[head[e]];
    if (next <= tb) {                       /* own event first on a tie */
      if (next >= t_end) break;
      int64_t t = next;
      int lv = l_select(&B, V);
      if (lv < 0) return -3;
      int lx = lv % L->bx, ly = lv / L->bx;
      B.blk[lv] = (int8_t)(-B.blk[lv]);
      int64_t gv = (int64_t)(B.y0 + ly) * L->Lx + B.x0 + lx;
      if (ev_push(ev, t, gv)) return -2;
      int onb = 0;
      if (!B.wrapy && ly == 0)          { if (hl_push(&out[EN], t, lx)) return -2; onb = 1; }
      if (!B.wrapy && ly == L->by - 1)  { if (hl_push(&out[ES], t, lx)) return -2; onb = 1; }
      if (!B.wrapx && lx == 0)          { if (hl_push(&out[EW], t, ly)) return -2; onb = 1; }
      if (!B.wrapx && lx == L->bx - 1)  { if (hl_push(&out[EE], t, ly)) return -2; onb = 1; }
      ev->nbound += onb;
      j += 1; anchor = t; acc = 0;
      draw(L, d, j, &E, &V);
      lam = l_lambda(&B, N);
      next = next_tick(anchor, E, acc, lam);
    } else {                                /* break point before own event */
      if (tb >= t_end) break;
      int64_t t = tb;
      /* apply one neighbour flip at tick t (several at one tick fold with
       * zero elapsed time in between, which changes nothing) */
      for (int e = 0; e < 4; ++e) {
        if (in[e] && head[e] < in[e]->n && in[e]->tick[head[e]] == t) {
          int32_t pos = in[e]->pos[head[e]];
          int8_t* h = (e == EN) ? hN : (e == ES) ? hS : (e == EW) ? hW : hE;
          h[pos] = (int8_t)(-h[pos]);
          head[e]++;
          break;
        }
      }
      acc += lam * (uint64_t)(t - anchor);
      anchor = t;
      lam = l_lambda(&B, N);
      next = next_tick(anchor, E, acc, lam);
    }
  }
  cout->j = j; cout->acc = acc; cout->anchor = anchor;
  return 0;
}

int orc_sr_run(const orc_params* p, orc_result* r, int32_t* g_out, int32_t* f_out,
               int32_t max_iters) {
  lat_t L;
  if (lat_init(&L, p) != 0) return -1;
  if (L.bx > 4096 || L.by > 4096) return -1;
  int8_t* s = r->spins;
  if (init_spins(&L, p, s) != 0) return -1;
  int nsub = L.nsub;
  int64_t nblk = (int64_t)L.bx * L.by;
  carry_t* carry = (carry_t*)calloc((size_t)nsub, sizeof(carry_t));
  carry_t* cwork = (carry_t*)calloc((size_t)nsub, sizeof(carry_t));
  int8_t* blk = (int8_t*)malloc((size_t)(nsub * nblk));
  hlist_t* lists[2];
  lists[0] = (hlist_t*)calloc((size_t)nsub * 4, sizeof(hlist_t));
  lists[1] = (hlist_t*)calloc((size_t)nsub * 4, sizeof(hlist_t));
  evlog_t* ev = (evlog_t*)calloc((size_t)nsub, sizeof(evlog_t));
  hlist_t empty = {0, 0, 0, 0};
  if (!carry || !cwork || !blk || !lists[0] || !lists[1] || !ev) return -2;
  if (max_iters <= 0) max_iters = 10000;

  int64_t nev = 0;
  for (int d = 0; d < nsub; ++d) {
    if (r->sub_flips) r->sub_flips[d] = 0;
    if (r->sub_digest) r->sub_digest[d] = 0;
  }
  int64_t nwin = p->horizon_ticks == 0 ? 0
               : (p->horizon_ticks + p->window_ticks - 1) / p->window_ticks;
  if (r->snap_M) observe(&L, s, &r->snap_M[0], &r->snap_bond[0]);
  for (int64_t w = 0; w < nwin; ++w) {
    int64_t t_c = w * p->window_ticks;
    int64_t t_end = t_c + p->window_ticks;
    if (t_end > p->horizon_ticks) t_end = p->horizon_ticks;
    int it, converged = 0, fmax = 0;
    if (p->step_rule == ORC_STEP_WIPE && t_c > 0) {
      /* wipe the slate: the pending pair of every subdomain is dropped and
       * the next one starts its hazard at t_c */
      for (int d = 0; d < nsub; ++d) {
        carry[d].j += 1;
        carry[d].anchor = t_c;
        carry[d].acc = 0;
      }
    }
    for (it = 0; it < max_iters; ++it) {
      int cur = it & 1, prev = cur ^ 1;
      for (int d = 0; d < nsub; ++d) {
        int cx = d % L.nbx, cy = d / L.nbx;
        int dn = wrapi(cy - 1, L.nby) * L.nbx + cx;
        int ds = wrapi(cy + 1, L.nby) * L.nbx + cx;
        int dw = cy * L.nbx + wrapi(cx - 1, L.nbx);
        int de = cy * L.nbx + wrapi(cx + 1, L.nbx);
        const hlist_t* in[4];
        if (it == 0) {                       /* canonical assumption */
          in[EN] = in[ES] = in[EW] = in[EE] = &empty;
        } else {
          in[EN] = &lists[prev][4 * dn + ES]; /* north neighbour's bottom row */
          in[ES] = &lists[prev][4 * ds + EN];
          in[EW] = &lists[prev][4 * dw + EE];
          in[EE] = &lists[prev][4 * de + EW];
        }
        if (L.nby == 1) in[EN] = in[ES] = NULL;
        if (L.nbx == 1) in[EW] = in[EE] = NULL;
        int rc = sr_local(&L, d, s, t_c, t_end, carry[d], in, blk + d * nblk,
                          &cwork[d], &lists[cur][4 * d], &ev[d]);
        if (rc) return rc;
        if (ev[d].nbound > fmax) fmax = (int)ev[d].nbound;
      }
      int changed = 0;
      for (int q = 0; q < 4 * nsub && !changed; ++q) {
        const hlist_t* old = (it == 0) ? &empty : &lists[prev][q];
        if (!hl_equal(&lists[cur][q], old)) changed = 1;
      }
      if (!changed) { converged = 1; break; }
    }
    if (!converged) return -5;
    if (g_out) g_out[w] = it + 1;
    if (f_out) f_out[w] = fmax;
    /* commit: end-of-window blocks become the committed lattice */
    for (int d = 0; d < nsub; ++d) {
      int x0 = (d % L.nbx) * L.bx, y0 = (d / L.nbx) * L.by;
      for (int ly = 0; ly < L.by; ++ly)
        for (int lx = 0; lx < L.bx; ++lx)
          s[(int64_t)(y0 + ly) * L.Lx + x0 + lx] = blk[d * nblk + ly * L.bx + lx];
      carry[d] = cwork[d];
    }
    /* events of the window, merged into global (tick, subdomain) order */
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
    if (r->snap_M) observe(&L, s, &r->snap_M[w + 1], &r->snap_bond[w + 1]);
  }
  r->n_events = nev;
  observe(&L, s, &r->M, &r->bond);
  if (r->carry) {
    for (int d = 0; d < nsub; ++d) {
      uint64_t E, V;
      draw(&L, d, carry[d].j, &E, &V);
      int64_t N[NCLS];
      uint64_t lam = sub_lambda(&L, s, d, N);
      r->carry[4 * d + 0] = (int64_t)carry[d].j;
      r->carry[4 * d + 1] = carry[d].anchor;
      r->carry[4 * d + 2] = (int64_t)carry[d].acc;
      r->carry[4 * d + 3] = next_tick(carry[d].anchor, E, carry[d].acc, lam);
    }
  }
  for (int q = 0; q < 4 * nsub; ++q) {
    free(lists[0][q].tick); free(lists[0][q].pos);
    free(lists[1][q].tick); free(lists[1][q].pos);
  }
  for (int d = 0; d < nsub; ++d) { free(ev[d].tick); free(ev[d].site); }
  free(lists[0]); free(lists[1]); free(ev); free(carry); free(cwork); free(blk);
  return 0;
}
