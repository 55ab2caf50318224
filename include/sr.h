/*
 * sr.h -- C ABI of the MI355X (gfx950) synchronous-relaxation library for the
 * continuous-time n-fold way Ising simulation (Lubachevsky & Weiss,
 * "Synchronous relaxation for parallel Ising spin simulations").
 *
 * Problem statement (Sec. 2): a rectangular Lx x Ly lattice with periodic
 * boundaries, spins +-1, four nearest neighbours, energy of eq. hamil
 * E = -J sum_<nn bonds> s s' - h sum s (every bond counted once), flip
 * probability p of eq. pMin (Metropolis) or eq. pglauber (Glauber) at
 * temperature T (k_B = 1); every site attempts flips as a Poisson process of
 * rate lambda = 1 (Sec. 3), so time is measured in units of 1/lambda.
 * Method (Secs. 4-5): the lattice is cut into bx x by subdomains (the
 * paper's PEs; one GPU wavefront each); each subdomain runs the rejection-free
 * n-fold way over a window [t_c, t_c + window) reading its neighbours'
 * boundary flip histories of the previous iteration (none in the first
 * iteration: the canonical assumption); iterations repeat until no boundary
 * history changes, then committed time t_c advances by the window (Sec. 4
 * box).  Random numbers are a presimulated list (Philox-4x32-10 keyed by the
 * seed, counter = (event index, subdomain)), reused across iterations and
 * carried across windows (Sec. 5, "Subsequent steps"), so the converged
 * trajectory does not depend on the window length.
 *
 * Integer conventions fixed by the library: ticks of 2^-tick_bits time units
 * (int64); rates as round(2^28 p); -log U as a Q(28 + tick_bits) fixed-point
 * integer; an event falls on the first tick at which the integrated hazard
 * reaches -log U (eq. lambdataua on the tick grid); simultaneous events of
 * different subdomains all choose from the state before their tick.
 *
 * Ownership: the library owns every device buffer of a simulation; callers
 * own every host buffer they pass.  All device work of a simulation is
 * ordered on the HIP stream given at creation (NULL = default stream); every
 * call returns only after that work is complete.  Handles are not
 * thread-safe: one host thread per handle at a time; different handles may
 * be driven from different threads at once (give them different streams so
 * that their device work overlaps).
 *
 * Errors: functions return SR_OK (0) or a negative SR_E* code; the message of
 * the last failure of a handle is sr_last_error(handle) (creation failures:
 * sr_last_error(NULL), kept per calling thread).
 */
#ifndef SR_H
#define SR_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SR_OK = 0,
  SR_EINVAL = -1,    /* invalid argument or parameter combination */
  SR_ENOMEM = -2,    /* device or host allocation failed */
  SR_EOVERFLOW = -3, /* a history buffer could not be grown any further */
  SR_ENOCONV = -4,   /* max_iters reached; the window was NOT committed */
  SR_EDEVICE = -5,   /* a HIP call or kernel failed */
  SR_EDONE = -6      /* committed time already equals the horizon */
};

enum { SR_METROPOLIS = 0, SR_GLAUBER = 1 };                 /* eq. pMin / eq. pglauber */
enum { SR_INIT_RANDOM = 0, SR_INIT_ALL_UP = 1, SR_INIT_USER = 2 };
enum { SR_LOG_DIGEST = 0, SR_LOG_FULL = 1 };
/* How a step (window) starts after the first (Sec. 5).  SR_STEP_CONTINUE:
 * each subdomain's pending random pair, the tick of its last event or break
 * point and the hazard integrated since carry over, so the trajectory does
 * not depend on the window.  SR_STEP_WIPE ("wipe the slate"): at every step
 * start t_c > 0 each subdomain drops its pending event and takes the next
 * pair of its list (one later than any used so far), its hazard counted from
 * t_c; unbiased by Poisson memorylessness, but the trajectory depends on the
 * window, which must then be fixed (window > 0). */
enum { SR_STEP_CONTINUE = 0, SR_STEP_WIPE = 1 };

typedef struct {
  int32_t Lx, Ly;            /* lattice (Sec. 2); 4 <= Lx, Ly; periodic */
  int32_t bx, by;            /* subdomain block (Sec. 5 partition G -> G_i):
                                Lx % bx == 0, Ly % by == 0, 2 <= bx, by <= 64,
                                bx*by <= 1024.
                                bx = by = 0: chosen by the tuner */
  double J, h, T;            /* coupling J > 0 allowed any sign, field, T > 0 */
  int32_t rule;              /* SR_METROPOLIS or SR_GLAUBER */
  double window;             /* T_max of Sec. 4/5 in time units (> 0);
                                0 = chosen by the tuner */
  double horizon;            /* simulate [0, horizon) (>= 0) */
  uint64_t seed;             /* Philox key */
  int32_t init;              /* SR_INIT_* */
  const int8_t* init_spins;  /* host, Ly*Lx row-major (+1/-1), read during
                                sr_create only; SR_INIT_USER only */
  int32_t log_mode;          /* SR_LOG_DIGEST or SR_LOG_FULL (every committed
                                (tick, site) kept on the host) */
  int32_t max_iters;         /* iterations per window before SR_ENOCONV
                                (0 = 10000) */
  int32_t tick_bits;         /* 0 = 28; 4..28 */
  int32_t hist_cap;          /* initial entries per boundary list and window
                                (0 = sized from the window; grown and the
                                window re-run on overflow; at most 1024,
                                SR_EINVAL above) */
  int32_t wlog_cap;          /* initial events per subdomain and window
                                (0 = sized from the window; grown likewise) */
  int32_t step_rule;         /* SR_STEP_CONTINUE (0) or SR_STEP_WIPE: Sec. 5,
                                "Subsequent steps" vs "An alternate approach
                                to subsequent steps" (see below) */
  int32_t Lz, bz;            /* 3D simple-cubic lattice (more dimensions and
                                neighbours, Secs. 3 and 5) when Lz >= 4: six
                                neighbours, 14 classes k = 7*[s = -1] + n_up,
                                blocks bx x by x bz with 2 <= each side and
                                every face (bx*by, by*bz, bx*bz) <= 64 sites,
                                bz = 0: chosen by the tuner (cubic block).
                                Lz = 0 or 1: the 2D square lattice (bz
                                ignored).  Global site (z*Ly + y)*Lx + x;
                                subdomain (cz*nby + cy)*nbx + cx.  3D runs
                                take the plain path (not sr_batch_* or the
                                server) and start every relaxation run at the
                                window start */
} sr_params;

typedef struct {
  int64_t tick;              /* committed time in ticks */
  int64_t M;                 /* sum of spins at committed time */
  int64_t bond_sum;          /* sum over right and down bonds of s s' */
  int64_t flips;             /* committed flips so far */
  int64_t events_processed;  /* flips simulated in all iterations so far */
  int64_t windows;           /* committed windows so far */
  int64_t iterations;        /* relaxation iterations so far */
  int32_t last_g;            /* iterations of the last committed window */
  int32_t last_f;            /* f of Sec. 6 for the last committed window:
                                the most own events on boundary sites of one
                                subdomain in one iteration, the largest over
                                the window's iterations */
  int32_t tick_bits;
  int32_t n_sub;             /* number of subdomains */
  int32_t bx, by;            /* block in use */
  int32_t Lx, Ly;            /* lattice */
  int64_t window_ticks;      /* window in use */
  int64_t horizon_ticks;
  int64_t relax_launches;    /* relaxation-kernel launches so far */
  double relax_ms;           /* their summed device time (HIP events on the
                                simulation's stream), milliseconds */
  int64_t subdomain_runs;    /* subdomain-iterations actually simulated (the
                                others kept their previous outputs) */
  int32_t Lz, bz;            /* 3D lattice and block depth (0, 0 in 2D) */
} sr_obs;

typedef struct sr_sim sr_sim;

/* Create a simulation: validates the parameters, builds the rate table
 * (eqs. pMin / pglauber on the host in IEEE double), allocates the device
 * state and sets the initial spins (Sec. 4 box, first step).
 * `hip_stream` is a hipStream_t (or NULL).  On success *out owns the handle. */
int sr_create(const sr_params* p, void* hip_stream, sr_sim** out);

/* Advance committed time by up to n_windows windows (Sec. 4 box: iterate
 * generate / synchronise / compare / synchronise until no history changes,
 * then increment committed time); n_windows < 0 runs to the horizon.  The last
 * window is truncated at the horizon.  iters_out (may be NULL) receives g of
 * each committed window and must hold n_windows entries; with n_windows < 0
 * it must be NULL (SR_EINVAL otherwise), because a tuned step size makes the
 * number of windows unknown in advance.  *n_done (may be NULL) = windows
 * committed.  On SR_ENOCONV the failing window is left uncommitted and
 * earlier ones stay.  A window that overflows a boundary list or the window
 * log is redone with larger buffers; at their capacity limits (1024 list
 * entries, 448 in 3D; 2^22 log entries) the step size is halved instead and
 * stays so (the continue rule's trajectory does not depend on it, so the
 * committed events are the same, in more windows), while under
 * SR_STEP_WIPE, whose trajectory depends on the step size, the call returns
 * SR_EOVERFLOW with the window uncommitted. */
int sr_run_window(sr_sim* s, int32_t n_windows, int32_t* iters_out, int32_t* n_done);

/* Observables at committed time (eq. hamil parts): M, bond sum, counters. */
int sr_observables(sr_sim* s, sr_obs* out);

/* Return to time 0: initial spins again (random, all up, or the spins given
 * at creation), empty carry, counters cleared, and an adapted step size back
 * to the one chosen at creation (or at load), so that a reset simulation
 * repeats the same windows; keeps every allocation. */
int sr_reset(sr_sim* s);

/* Release everything.  NULL-safe. */
void sr_destroy(sr_sim* s);

/* Committed spins, Ly*Lx int8 row-major (3D: Lz*Ly*Lx), into a
 * caller-owned host buffer. */
int sr_get_spins(sr_sim* s, int8_t* host_out);

/* SR_LOG_FULL only: committed events of subdomain d (row-major block id) in
 * time order: ticks[i], global sites[i] (y*Lx + x).  Copies min(n, cap)
 * entries; *n = total. */
int sr_get_log(sr_sim* s, int32_t d, int64_t* ticks, int64_t* sites, int64_t cap, int64_t* n);

/* Per-subdomain event digests (order-free 64-bit sum over committed events
 * of mix(mix(tick) + global site), mix = SplitMix64 finaliser) and committed
 * flip counts; caller-owned arrays of n_sub entries (either may be NULL). */
int sr_get_digests(sr_sim* s, uint64_t* digests, int64_t* flips);

/* Per-subdomain carry at committed time: (j, anchor, acc) = index of the
 * pending random pair, tick of the last event or break point, integrated
 * hazard since then.  Caller-owned, 3 * n_sub int64. */
int sr_get_carry(sr_sim* s, int64_t* out);

/* The class rates round(2^28 p_k): 10 on the square lattice, class
 * k = 5*[s = -1] + (up neighbours); 14 on the simple-cubic one,
 * k = 7*[s = -1] + (up neighbours).  out must hold 14 entries; the first 10
 * or 14 are written. */
int sr_get_rate_table(sr_sim* s, uint32_t out[14]);

/* The same table computed from parameters alone, as sr_create computes it
 * (eqs. hamil, pMin / pglauber in IEEE double on the host; no device work,
 * so it may be called without a GPU).  Reads J, h, T and rule only.
 * SR_EINVAL for a null argument, T <= 0, non-finite J, h or T, or an unknown
 * rule. */
int sr_rate_table(const sr_params* p, uint32_t out[14]);

/* Checkpoint of the committed state (committed time is a consistent cut,
 * Sec. 4): committed spins, per-subdomain carry, counters, and for an
 * SR_INIT_USER simulation its initial spins (so sr_reset works after a
 * load); a simulation with a tuned step size keeps the step size it had
 * reached.  sr_save with host_blob = NULL reports the size in *n; the caller
 * owns the blob.  sr_load creates a new simulation on `hip_stream` that
 * continues bit for bit where the saved one stood; SR_EINVAL for a blob that
 * is not a checkpoint of this library version or is truncated. */
int sr_save(sr_sim* s, void* host_blob, size_t cap, size_t* n);
int sr_load(const void* host_blob, size_t n, void* hip_stream, sr_sim** out);

/* Message of the last failure (NULL handle: the calling thread's last
 * creation / load failure). */
const char* sr_last_error(const sr_sim* s);

/* ---- batched form: many independent lattices in one persistent launch ----
 * Runs every listed simulation to its horizon with one persistent kernel:
 * resident wavefronts pop (lattice, subdomain) tasks from a device work queue;
 * the last task of a lattice's iteration decides convergence and enqueues the
 * next iteration or the next window.  Results are bit-identical to
 * sr_run_window on each simulation alone.  All simulations must use
 * SR_LOG_DIGEST and the same stream.  A launch whose waves find no work for
 * far longer than any task takes gives up; the lattices it had not finished
 * continue from their last committed window in another launch (the same
 * results), and fail with SR_EDEVICE after 3 such launches in a row. */
int sr_batch_run(sr_sim* const* sims, int32_t n, void* hip_stream);

/* Batched form with a budget: every listed simulation commits at most
 * max_windows windows (all remaining if max_windows <= 0) in one persistent
 * launch, then the call returns; later calls continue where each stopped.
 * This is the scheduling step of continuous batching: between calls,
 * simulations may be added to or removed from the list. */
int sr_batch_step(sr_sim* const* sims, int32_t n, int32_t max_windows, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as sr_batch_step, bit-identical results, but the persistent launch's
 * queue, counters, lattice descriptors and per-lattice records live in one
 * 8 MiB array of device memory per GPU that the library holds for the life
 * of the process; the call allocates and frees no device memory (and, on
 * success, no host memory).  Limits: at most 1024 lattices with unfinished
 * windows per call, and the call's queue must fit the array (about 500 000
 * subdomains in all); SR_EINVAL otherwise, before any device work.  A
 * lattice whose boundary list or window log overflows is not re-run with
 * grown buffers (that would allocate): the call returns SR_EOVERFLOW and the
 * window stays uncommitted (sr_batch_step or sr_run_window can continue it).
 * Every call on one GPU uses that GPU's one array and the next call
 * overwrites it, so calls that overlapped on one GPU would race: the library
 * serialises them within a process (a mutex held for the whole call).  Each
 * process has its own arrays. */
int sr_batch_step_static(sr_sim* const* sims, int32_t n, int32_t max_windows, void* hip_stream);

/* ---- tuner ---- block and first window for a lattice (used when bx = by =
 * 0 or window = 0).  Block: a fixed table over (L, T) -- never load-dependent,
 * because the block partition keys the random streams and so the trajectory.
 * First window: 4 x the step-size rule T_max = log N / (lambda |dG_i|) of
 * Sec. 5, clamped to [1/8, 2].  A 3D lattice (Lz >= 4) gets a cubic block
 * (bz = bx), 8^3 halved until it divides every side.  A simulation created with window = 0 then
 * adapts its step size after every committed window from the measured
 * iterations g (Sec. 4 box: a step size is chosen at each step), aiming at
 * about 12 iterations per window in sr_run_window and 6 in the batched form
 * (whose per-window cost is lower); the trajectory does not depend on it. */
int sr_tune(const sr_params* p, int32_t* bx, int32_t* by, double* window);

/* ---- serving: continuous batching of simulation requests ----
 * Driven by the caller (no threads).  sr_server_submit queues a request (an
 * SR_LOG_DIGEST simulation of a 2D lattice).  The server keeps one persistent
 * batched launch running over every admitted lattice; sr_server_pump never
 * waits for it to finish.  While it runs, a pump that sees a waiting request
 * whose device footprint fits `hbm_budget`, or a lattice that reached its
 * horizon, asks the launch to end (every lattice pauses at its next window
 * boundary, so the launch ends within about one window of work); the pump
 * after it ends retires finished lattices (results to sr_server_poll, memory
 * freed), admits waiting requests in arrival order while their footprint
 * fits, and starts the next launch over all admitted lattices.  A request
 * thus joins the lattices already on the device after the windows in flight,
 * not after a round of fixed length, and its work overlaps theirs.  A
 * request's result equals its simulation run alone (pausing at a window
 * boundary does not change the trajectory).  Not thread-safe: one thread
 * drives a server. */
typedef struct sr_server sr_server;
typedef struct {
  uint64_t req_id;           /* from sr_server_submit */
  uint64_t digest;           /* sum of the per-subdomain event digests */
  int64_t M, bond_sum, flips, events_processed, windows, iterations;
  double t_arrive, t_start, t_done;  /* seconds since server creation:
                                        submitted, admitted, retired */
  int32_t status;            /* SR_OK or an SR_E* code */
  int32_t bx, by;            /* block the request ran with */
} sr_result;
typedef struct {
  int64_t submitted, completed, failed, queued, rounds;
  int64_t bytes_in_use, peak_bytes;
  int32_t peak_active;
  int32_t restarts;          /* lattices continued from their last committed
                              * window after a launch gave up waiting for work */
  double busy_s, uptime_s;   /* time inside batch steps / since creation */
} sr_server_info;

/* hip_stream: stream for all of the server's device work (NULL = default).
 * windows_per_round > 0 additionally ends every launch after that many
 * windows per lattice (a fairness bound); <= 0: launches end only when asked
 * to or when every lattice is done. */
int sr_server_create(size_t hbm_budget, int32_t windows_per_round, void* hip_stream, sr_server** out);
/* Copies the parameters (and SR_INIT_USER spins); the arrival time is now.
 * SR_ENOMEM if the request alone exceeds the budget. */
int sr_server_submit(sr_server* v, const sr_params* p, uint64_t* req_id);
/* One scheduling step (see above); waits at most about a millisecond for a
 * running launch.  *n_open (may be NULL) = requests not yet retired.  When a
 * launch fails, its requests retire with the error code, which is returned,
 * and the reason is sr_last_error(NULL) of the calling thread. */
int sr_server_pump(sr_server* v, int32_t* n_open);
/* Retired requests since the last poll, oldest first; up to cap into the
 * caller's array, *n = how many. */
int sr_server_poll(sr_server* v, sr_result* out, int32_t cap, int32_t* n);
int sr_server_stats(sr_server* v, sr_server_info* out);
/* Frees every simulation still admitted; queued requests are dropped. */
void sr_server_destroy(sr_server* v);

#ifdef __cplusplus
}
#endif
#endif /* SR_H */
