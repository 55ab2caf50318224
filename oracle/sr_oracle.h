/*
 * sr_oracle.h -- CPU oracle (test infrastructure only) for synchronous
 * relaxation of the continuous-time n-fold way Ising simulation.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may use it.  Shares nothing with the GPU library.
 */
#ifndef SR_ORACLE_H
#define SR_ORACLE_H
#include <stdint.h>

enum { ORC_METROPOLIS = 0, ORC_GLAUBER = 1 };
enum { ORC_INIT_RANDOM = 0, ORC_INIT_ALL_UP = 1, ORC_INIT_USER = 2 };
/* Sec. 5: subsequent steps continue the pending random pair and its
 * integrated hazard ("Subsequent steps"), or wipe the slate at every step
 * start ("An alternate approach to subsequent steps"). */
enum { ORC_STEP_CONTINUE = 0, ORC_STEP_WIPE = 1 };

typedef struct {
  int32_t Lx, Ly;          /* periodic lattice, Lx, Ly >= 2 */
  int32_t bx, by;          /* subdomain block; Lx % bx == 0, Ly % by == 0 */
  double J, h, T;          /* coupling, field, temperature (k_B = 1) */
  int32_t rule;            /* ORC_METROPOLIS (eq. pMin) or ORC_GLAUBER (eq. pglauber) */
  int32_t tick_bits;       /* one tick = 2^-tick_bits time units */
  int32_t init;            /* ORC_INIT_* */
  int64_t window_ticks;    /* committed-time step (snapshots; SR step size) */
  int64_t horizon_ticks;   /* simulate [0, horizon) */
  int64_t burn_ticks;      /* time integrals start here */
  uint64_t seed;
  const int8_t* init_spins;/* Ly*Lx, for ORC_INIT_USER */
  int32_t step_rule;       /* ORC_STEP_CONTINUE or ORC_STEP_WIPE (Sec. 5) */
} orc_params;

typedef struct {
  int8_t* spins;           /* out, Ly*Lx (required) */
  int64_t* log_tick;       /* out, flat event log in (tick, subdomain) order */
  int64_t* log_site;
  int32_t* log_sub;
  int64_t log_cap;         /* entries available in the log arrays (0: none) */
  int64_t* sub_flips;      /* out, per subdomain committed flips (or NULL) */
  uint64_t* sub_digest;    /* out, per subdomain event digest (or NULL) */
  int64_t* snap_M;         /* out, M at committed times k*W, k = 0..nwin (or NULL) */
  int64_t* snap_bond;      /* out, bond sum at the same times */
  int64_t* carry;          /* out, per subdomain (j, anchor, acc, next) (or NULL) */
  int64_t n_events;
  int64_t M, bond;         /* final */
  double int_M, int_M2, int_absM, int_bond, int_E2, int_M4; /* tick-weighted sums */
  int64_t int_ticks;
} orc_result;

/* 3D simple-cubic lattice (sr_oracle3d.c): 14 classes, six faces. */
typedef struct {
  int32_t Lx, Ly, Lz;      /* periodic lattice, each >= 2 */
  int32_t bx, by, bz;      /* subdomain block, dividing the lattice */
  double J, h, T;
  int32_t rule, tick_bits, init;
  int64_t window_ticks, horizon_ticks, burn_ticks;
  uint64_t seed;
  const int8_t* init_spins;/* Lz*Ly*Lx, for ORC_INIT_USER */
  int32_t step_rule;
} orc3_params;

void orc_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]);
uint64_t orc_expq(uint64_t u, int tick_bits);
int orc_rate_table(double J, double h, double T, int rule, uint32_t out[10]);
uint64_t orc_mix64(uint64_t z);
uint64_t orc_event_digest(int64_t tick, int64_t site);
int orc_select_site(const orc_params* p, const int8_t* spins, int d, uint64_t V, int64_t* site_out);
int orc_subdomain_lambda(const orc_params* p, const int8_t* spins, int d, uint64_t* lam_out);
int orc_des_run(const orc_params* p, orc_result* r);
int orc_sr_run(const orc_params* p, orc_result* r, int32_t* g_out, int32_t* f_out, int32_t max_iters);

int orc3_rate_table(double J, double h, double T, int rule, uint32_t out[14]);
int orc3_select_site(const orc3_params* p, const int8_t* spins, int d, uint64_t V, int64_t* site_out);
int orc3_subdomain_lambda(const orc3_params* p, const int8_t* spins, int d, uint64_t* lam_out);
int orc3_des_run(const orc3_params* p, orc_result* r);
int orc3_sr_run(const orc3_params* p, orc_result* r, int32_t* g_out, int32_t* f_out, int32_t max_iters);

#endif
