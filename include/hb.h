/*
 * libhb -- MI355X (gfx950) RK4 solver for the Higgs boson equation in de
 * Sitter spacetime (Balogh, Banda, Yagdjian, arXiv:1803.01291).
 *
 * The library advances the first-order system of section 2.1, eq. (rhs),
 *
 *     phi_t = psi
 *     psi_t = -3 psi + inv_L2 exp(-2t) Lap_h phi + mu2 phi - lambda phi^3
 *
 * (eq. (higgs-boson-rescalled) with inv_L2 = 1/L^2; inv_L2 = 1 is eq. (HBE)
 * itself) with the classical explicit fourth-order Runge-Kutta method of
 * section 2.1 and the fourth-order central-difference Laplacian of section 2.1
 * (13-point star), on a uniform 3-D grid with the zero boundary condition of
 * eq. (BC) realised as a 2-cell zero halo.
 *
 * Grid: an axis with n points on [lo, hi] has h = (hi - lo)/n and cell-centred
 * nodes x_i = lo + (i + 1/2) h.  Host/device arrays exchanged through this API
 * hold interior points only, C-ordered [nz][ny][nx] (x fastest), contiguous.
 *
 * Conventions for every call:
 *  - Functions return HB_OK (0) or a negative HB_E_* code; no exception
 *    crosses the ABI.  hb_last_error() gives a message for the calling thread.
 *  - Pointers marked "device" are HIP device pointers on the current device;
 *    "host" pointers are ordinary host memory.  The caller keeps ownership of
 *    every array it passes; the library copies what it needs before returning
 *    (host) or in stream order (device).
 *  - Handles are not thread-safe; distinct handles may be used concurrently.
 *  - All device work of a handle is ordered on its stream (hb_config.stream,
 *    or a stream the library creates when that is NULL).  A library-created
 *    stream is non-blocking: it does not wait for work on other streams, so
 *    device inputs produced elsewhere must be complete before the call, or
 *    the producing stream must be the handle's stream.
 */
#ifndef HB_H
#define HB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HB_OK 0
#define HB_E_ARG (-1)       /* invalid argument                                   */
#define HB_E_CFL (-2)       /* dt beyond the RK4 linear stability limit           */
#define HB_E_NOMEM (-3)     /* device or host allocation failed                   */
#define HB_E_HIP (-4)       /* HIP runtime error                                  */
#define HB_E_STATE (-5)     /* call out of order (e.g. step before initial data)  */
#define HB_E_BUSY (-6)      /* pool: no free slot or HBM budget exhausted         */
#define HB_E_NONFINITE (-7) /* diagnostics found NaN/Inf in the state             */

/* hb_config.precision */
#define HB_F64 0  /* FP64 storage and arithmetic                                */
#define HB_F32C 1 /* FP32 field storage and stencil; the RK4 state update is    */
                  /* carried in FP64 registers and stored as FP32 hi + lo       */

/* memory kind of a user array */
#define HB_HOST 0
#define HB_DEVICE 1

/* element type of a user array */
#define HB_DTYPE_F64 0
#define HB_DTYPE_F32 1

/* hb_config.flags */
#define HB_ALLOW_UNSTABLE 1u /* skip the dt stability check                    */
#define HB_USE_GRAPH 2u      /* replay captured hipGraphs of several steps     */
#define HB_STAGEWISE 4u      /* one launch per RK4 stage (19 field passes per  */
                             /* step); bitwise-equal results                  */
#define HB_PAIRWISE 8u       /* one launch per stage pair (10 passes per step) */
                             /* instead of the default whole-step launch (4   */
                             /* passes); bitwise-equal results                */
#define HB_DEBUG_POISON 32u  /* debug: fill every stored cell outside the     */
                             /* interior and its 2-cell halo (pitch padding,  */
                             /* alignment prefix, tail) with quiet NaNs at    */
                             /* creation, so a kernel reading one would carry */
                             /* NaN into the results; results are unchanged   */
#define HB_BC_PERIODIC 16u   /* periodic boundaries on every axis instead of  */
                             /* the zero 2-cell halo (a test configuration:   */
                             /* e.g. constant data then follows the damped    */
                             /* Duffing ODE); whole-step scheme only          */

typedef struct hb_config {
    int32_t n[3];        /* interior points along x, y, z (each >= 1)              */
    double lo[3], hi[3]; /* box [lo_d, hi_d] per axis, hi_d > lo_d                  */
    double mu2;          /* mu^2 of eq. (HBE) (any finite real)                     */
    double lambda;       /* lambda of eq. (HBE) (any finite real; < 0 allowed)      */
    double inv_L2;       /* 1/L^2 of eq. (higgs-boson-rescalled); 1 for eq. (HBE)   */
    double t0;           /* initial time                                            */
    double dt;           /* RK4 time step (> 0)                                     */
    int32_t precision;   /* HB_F64 or HB_F32C                                       */
    uint32_t flags;      /* HB_ALLOW_UNSTABLE | HB_USE_GRAPH | HB_PAIRWISE |        */
                         /* HB_STAGEWISE | HB_DEBUG_POISON | HB_BC_PERIODIC         */
    void* stream;        /* hipStream_t to order work on, or NULL                   */
} hb_config;

/* FP64 diagnostics of the current state (t = t0 + step dt), cell volume
 * dV = hx hy hz:
 *   integral = dV sum phi, l2_phi = sqrt(dV sum phi^2), l2_psi likewise,
 *   linf_phi = max|phi|, linf_psi = max|psi|,
 *   lap_max  = c(t) max|Lap_h phi|            (the paper's P(t), Example 4)
 *   energy   = dV sum [psi^2/2 + c(t) phi (-Lap_h phi)/2 - mu2 phi^2/2 + lambda phi^4/4]
 *   nonfinite = number of NaN/Inf values of phi and psi,
 *   negative  = number of interior points with phi < 0 (sign changes: the
 *               paper's bubbles, section 1). */
typedef struct hb_diag {
    double t;
    int64_t step;
    double integral, l2_phi, l2_psi, linf_phi, linf_psi, lap_max, energy;
    int64_t nonfinite, negative;
} hb_diag;

typedef struct hb_solver hb_solver;
typedef struct hb_batch hb_batch;
typedef struct hb_pool hb_pool;

/* ---- single solve (section 2.1) ------------------------------------------ */

/* Validate cfg, allocate all device state (library-owned) and zero the halo.
 * The stability check requires dt * sqrt(c0 * sum_d 16/(3 h_d^2)) <= 2 sqrt(2),
 * c0 = inv_L2 exp(-2 t0) (RK4's imaginary-axis limit against the largest
 * eigenvalue of -Lap_h); HB_E_CFL otherwise unless HB_ALLOW_UNSTABLE.
 * Whole-step solves (the default) need an x-y plane of 16-byte cells under
 * 2 GiB (up to 11580^2 points); larger planes are HB_E_ARG.
 * Errors: HB_E_ARG, HB_E_CFL, HB_E_NOMEM, HB_E_HIP.  *out is NULL on error. */
int hb_create(const hb_config* cfg, hb_solver** out);

/* Set phi(., t0) = phi0 and phi_t(., t0) = phi1 (eq. (HBEinit)); resets the
 * step counter to 0.  phi0/phi1: nz*ny*nx values of `dtype` in `mem`
 * (phi1 may be NULL for zero).  For HB_F32C an FP64 input is split into an
 * FP32 high part and an FP32 low part.  Host inputs are copied before the call
 * returns; device inputs are read in stream order. */
int hb_set_initial(hb_solver* s, const void* phi0, const void* phi1, int mem, int dtype);

/* Restore a checkpoint: the state vector v = (phi, phi_t) of eq. (rhs)
 * (section 2.1) at step n, 0 <= n <= 2^40; psi (= phi_t) may be NULL for
 * zero.  The time is not an argument: it is t = t0 + n dt, computed by
 * multiplication as for every step, so a resumed solve sees the stage times
 * it would have seen without stopping and stepping on is bitwise the same as
 * never having stopped.  Arrays as for hb_set_initial. */
int hb_set_state(hb_solver* s, const void* phi, const void* psi, int64_t n, int mem, int dtype);

/* Enqueue nsteps steps of the classical fourth-order Runge-Kutta method of
 * section 2.1 (stages at t_n, t_n + dt/2, t_n + dt/2, t_n + dt, t_n = t0 +
 * n dt) applied to eq. (rhs), on the solver's stream, and return without
 * waiting.
 * Each step is one whole-step kernel (default), 2 stage-pair kernels
 * (HB_PAIRWISE) or 4 per-stage kernels (HB_STAGEWISE); a tiny kernel advances
 * the device step counter after each batch of steps.  HB_E_STATE before
 * initial data.  With HB_TRACE set in the environment (and not "0") every
 * kernel is timed with HIP events and waited for, and each step prints one
 * line with the kernels' times to stderr. */
int hb_step(hb_solver* s, int64_t nsteps);

/* Like hb_step, but waits after every step and returns the summed device time
 * of each kernel of the step in stage_ms[0..3] (HIP events on the solver's
 * stream around each launch): the whole-step kernel in [0], the 2 stage-pair
 * kernels in [0..1] (HB_PAIRWISE) or the 4 per-stage kernels (HB_STAGEWISE);
 * unused entries are 0.  For measurement. */
int hb_step_timed(hb_solver* s, int64_t nsteps, double* stage_ms);

/* Wait for the solver's stream, then copy the interior state vector
 * v = (phi, phi_t) of eq. (rhs) (section 2.1) out: phi into `phi`, phi_t
 * into `phi_t`, each nz*ny*nx values of `dtype` in `mem` (C order, x
 * fastest).  Either output may be NULL.  For HB_F32C the value returned is
 * hi + lo in FP64 (rounded to FP32 for HB_DTYPE_F32). */
int hb_read(hb_solver* s, void* phi, void* phi_t, int mem, int dtype);

/* Current time and step count (host bookkeeping; no wait). */
int hb_time(const hb_solver* s, double* t, int64_t* n);

/* Wait for all work enqueued on the solver's stream. */
int hb_sync(hb_solver* s);

/* FP64 diagnostics (deterministic fixed-order reductions); waits.  Returns
 * HB_E_NONFINITE (with *out filled) when the state holds NaN/Inf. */
int hb_diagnostics(hb_solver* s, hb_diag* out);

/* The paper's bubbles (section 1: maximal connected sets on which the
 * solution has changed sign) in the current state: *negative_sets = the
 * number of maximal face-connected (6-neighbour) sets of interior points
 * with phi < -eps, *positive_sets likewise for phi > eps (periodic solves:
 * neighbours wrap across the faces).  eps >= 0 (0: the sign itself).  FP32c
 * states are classed on hi + lo in FP64.  Keeps a label array of 4 bytes per
 * interior point from the first call (grids of at most 2^32 - 2 points,
 * HB_E_ARG beyond).  Waits.  HB_E_STATE before initial data. */
int hb_bubbles(hb_solver* s, double eps, int64_t* negative_sets, int64_t* positive_sets);

/* Tile shape: zc >= 1 planes per tile (0 = library default: for the
 * whole-step kernel, the length that best fills whole rounds of resident
 * blocks on the device); by in {8, 16}: rows of 64 columns per tile for the
 * stage-pair and per-stage kernels (default 16); for the whole-step kernel
 * by = 8 selects 32 x 24 tiles (1008-thread blocks), by = 16 selects 60 x 12
 * tiles (1024-thread blocks), by = 11 selects 64 x 11 tiles (1020-thread
 * blocks) and by = 20 selects 32 x 16 tiles (720-thread blocks); 11 and 20
 * are whole-step only, else HB_E_ARG.  The whole-step default comes from the
 * library's model of block rounds (e.g. 32 x 16 on a 256^3 grid, 64 x 11 on
 * 512^3, 32 x 24 on 384^3).  Results do not depend on it. */
int hb_set_tiling(hb_solver* s, int by, int zc);

/* The tiling (by, zc as in hb_set_tiling) hb_create would give a single
 * solve of cfg: the region shape and z-march length from the library's model
 * of block rounds on the current device (256 CUs assumed when no device is
 * visible, so it also answers on a host without a GPU; it launches nothing).
 * HB_E_ARG / HB_E_CFL as hb_create for an invalid cfg; by, zc untouched then. */
int hb_default_tiling(const hb_config* cfg, int* by, int* zc);

/* Time every candidate tile shape for `trial_steps` steps on the current
 * state, keep the fastest, and restore the state (bitwise).  The choice is
 * cached per (device, precision, grid) in the text file named by the
 * HB_TUNE_CACHE environment variable, if set (one "key by zc" line each). */
int hb_autotune(hb_solver* s, int trial_steps, int* by, int* zc);

/* Free everything (NULL-safe). */
int hb_destroy(hb_solver* s);

/* Device bytes hb_create would allocate for cfg (0 on invalid cfg): per
 * field, the padded grid; the whole-step scheme keeps a cell's state in one
 * 16-byte slot per step parity, (phi, psi) in FP64 or (phi hi, psi hi, phi
 * lo, psi lo) in FP32c (32 B per padded cell either way); HB_PAIRWISE and
 * HB_STAGEWISE keep separate fields and add G1..G3. */
size_t hb_footprint(const hb_config* cfg);

/* Message of the last failed call on this thread ("" if none). */
const char* hb_last_error(void);

/* Device memory allocator for every later allocation of the library (solve
 * state, coefficient tables, tile tables, staging and diagnostics buffers,
 * batches, pools, radial batches; not the bandwidth probe), so that a
 * framework's caching allocator can own it.  alloc(ctx, bytes, stream)
 * returns device memory on the current device, aligned to at least 256
 * bytes, for work ordered on `stream` (a hipStream_t, NULL for the null
 * stream), or NULL on failure (the call then fails with HB_E_NOMEM);
 * release(ctx, ptr, bytes) takes it back, and is called only after `stream`
 * has finished all work on it.  Every block goes back through the allocator
 * that made it, even after another is installed.  Both NULL restores
 * hipMalloc/hipFree; one NULL is HB_E_ARG.  Process-wide; the functions may
 * be called from any thread that calls the library. */
typedef void* (*hb_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*hb_free_fn)(void* ctx, void* ptr, size_t bytes);
int hb_set_allocator(hb_alloc_fn alloc, hb_free_fn release, void* ctx);

/* ---- batched form: many independent solves in shared launches -------------- */

/* count solves with their own grid, coefficients, dt and precision.  All
 * solves of one precision advance together, one launch per kernel of the
 * scheme (one per step by default) over a device tile table spanning them.
 * Every config must select the same scheme (HB_E_ARG otherwise).  Results are
 * bitwise equal to hb_step on the same solve.  stream: hipStream_t or NULL. */
int hb_batch_create(int count, const hb_config* cfgs, void* stream, hb_batch** out);
int hb_batch_set_initial(hb_batch* b, int i, const void* phi0, const void* phi1, int mem, int dtype);
int hb_batch_step(hb_batch* b, int64_t nsteps);
int hb_batch_read(hb_batch* b, int i, void* phi, void* phi_t, int mem, int dtype);
int hb_batch_sync(hb_batch* b);
int hb_batch_set_tiling(hb_batch* b, int by, int zc);
/* The library's autotuner over a batch: for each precision group (index 0
 * FP64, 1 FP32c) every candidate tile shape and z-march length is timed for
 * trial_steps steps from the current states, the fastest is kept for that
 * group, and every state is restored bitwise.  by[2] and zc[2] (either may
 * be NULL) receive the choices, -1 for an empty group.  With HB_TUNE_CACHE
 * set, choices are cached per device, precision, scheme and mix of member
 * grids (a batch with the same grid sizes hits the entry).  Results do not
 * depend on the tiling.  HB_E_STATE before every solve has initial data. */
int hb_batch_autotune(hb_batch* b, int trial_steps, int* by, int* zc);
int hb_batch_destroy(hb_batch* b);

/* ---- served form: continuous batching of admitted solves ------------------ */

/* A pool with an HBM budget (bytes, > 0) and at most max_slots resident solves
 * (1 <= max_slots <= 2^20; HB_E_ARG otherwise).  stream: hipStream_t or NULL. */
int hb_pool_create(size_t hbm_budget, int max_slots, void* stream, hb_pool** out);

/* Admit one solve of `steps` steps with initial data (as hb_set_initial).
 * Pool solves run the whole-step kernel: a cfg with HB_PAIRWISE or
 * HB_STAGEWISE is rejected (HB_E_ARG).  Returns HB_E_BUSY (nothing allocated,
 * nothing changed) when no slot is free or the solve's device bytes (those of
 * hb_footprint(cfg), with a coefficient table for `steps`) exceed the unused
 * budget.  The solve joins the active set at the next hb_pool_advance. */
int hb_pool_admit(hb_pool* p, const hb_config* cfg, const void* phi0, const void* phi1, int mem,
                  int dtype, int64_t steps, int* slot);

/* Advance every active solve by up to k steps (each stops at its own step
 * count); one whole-step launch per step and precision over all of them. */
int hb_pool_advance(hb_pool* p, int k);

/* Slots that finished since the last poll, written to done[0 .. cap-1] (done
 * may be NULL only when cap <= 0); *ndone is the count.  A finished slot is
 * reported once. */
int hb_pool_poll(hb_pool* p, int* done, int cap, int* ndone);

/* Check every active solve for non-finite values (NaN or Inf in phi or psi;
 * one FP64 diagnostics pass over each, so call it every so many advances):
 * a solve that holds any stops stepping, its slot is written to
 * failed[0 .. cap-1] (*nfailed = the number written) and hb_pool_poll then
 * reports it as finished (its state can still be read); the other solves
 * continue unchanged.  Waits for the pool's stream. */
int hb_pool_check(hb_pool* p, int* failed, int cap, int* nfailed);

/* Number of admitted, unfinished solves and bytes of the budget in use. */
int hb_pool_stats(const hb_pool* p, int* active, size_t* in_use);

int hb_pool_read(hb_pool* p, int slot, void* phi, void* phi_t, int mem, int dtype);
int hb_pool_release(hb_pool* p, int slot);
int hb_pool_destroy(hb_pool* p);

/* ---- batched radial solves (section 2.2, eq. (radial)) ---------------------- */

/* One radial solve: nodes r_i = i dr, i = 0..m-1, with phi = 0 at r = m dr
 * (the outer zero boundary), phi_r(0) = 0 through the symmetric ghost of
 * section 2.2, the operator 2/r phi_r + phi_rr with the fourth-order central
 * first and second differences (3 phi_rr at r = 0 by L'Hospital's rule), and
 * classical RK4 from t0 for `steps` steps of dt. */
typedef struct hb_radial_config {
    int32_t m;        /* 1 <= m <= HB_RADIAL_MAX_NODES                      */
    uint32_t flags;   /* HB_ALLOW_UNSTABLE                                  */
    double dr;        /* node spacing (> 0)                                 */
    double mu2, lambda, inv_L2, t0, dt;
    int64_t steps;    /* >= 0                                               */
} hb_radial_config;

#define HB_RADIAL_MAX_NODES 2700

/* Advance `count` independent radial solves together (one workgroup per
 * solve; each launch runs up to 65536 steps of every solve inside the kernel,
 * so a solve of at most that many steps takes one launch).  phi and psi hold
 * the solves' nodes back to back (solve k starts after the m of solves
 * 0..k-1), FP64, in `mem` (HB_HOST or HB_DEVICE); they are read as the
 * initial state and overwritten with the final state.  Waits for completion.
 * Stability: dt sqrt(c0 16/dr^2) <= 2 sqrt(2), c0 = inv_L2 exp(-2 t0),
 * else HB_E_CFL (unless HB_ALLOW_UNSTABLE).  stream: hipStream_t or NULL. */
int hb_radial_solve(int count, const hb_radial_config* cfgs, double* phi, double* psi, int mem,
                    void* stream);

/* hb_radial_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same solves with bitwise the same results, but phi and
 * psi must be device memory (nodes back to back as for hb_radial_solve,
 * read as the initial state and overwritten with the final one) and the call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * Descriptors and c(t) tables go into a fixed 8 MiB device scratch array
 * that each device holds for the life of the process: a batch whose 80-byte
 * descriptors (count x 80, rounded up to 256 bytes) leave no room for one
 * step's table of 24 bytes per distinct (t0, dt, inv_L2) is rejected with
 * HB_E_ARG before anything runs; launches then cover as many steps as the
 * table room allows.  Every call on a device shares that device's scratch
 * and rewrites it before use, so calls that overlap on one device (from
 * several threads or streams) race and must be serialised.  Validation and
 * stability errors as for hb_radial_solve.  Waits for completion. */
int hb_radial_solve_noalloc(int count, const hb_radial_config* cfgs, double* phi, double* psi,
                            void* stream);

/* ---- measurement ----------------------------------------------------------- */

/* Streamed-bandwidth probe on the current device (the achievable HBM streaming
 * ceiling: one 16-byte element per thread per array).  kind 0: copy (1 read + 1 write
 * array), 1: add (2 reads + 1 write), 2: 5 reads + 2 writes (the FP64 stage-4
 * mix).  Each array holds bytes_per_array bytes (library-allocated, freed
 * before return).  *gbps = bytes moved / time of `iters` launches after one
 * warm-up launch.  Waits; uses the NULL stream. */
int hb_probe_bandwidth(int kind, size_t bytes_per_array, int iters, double* gbps);

#ifdef __cplusplus
}
#endif

#endif /* HB_H */
