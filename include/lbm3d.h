/*
 * lbm3d.h -- C ABI of the MI355X (gfx950) 3D finite-difference lattice
 * Boltzmann solver for compressible Euler flow.
 *
 * The method is that of Chen, Xu, Zhang and Li, "Three-Dimensional Lattice
 * Boltzmann Model for High-Speed Compressible Flows" (arXiv:1010.4135): the
 * 15-velocity Kataoka-Tsutahara model (Sec. 2, Eq. (vv)) with the equilibrium
 * of Eqs. (eq)/(e18), the BGK kinetic equation with the paper's artificial
 * dissipation (Sec. 3, Eq. (lp)), the NND flux-split minmod scheme for the
 * convection term (Sec. 3, Eq. (nnd)) and a forward-Euler time step
 * (Sec. 3, Eq. (fi1)).
 *
 * Conventions for every entry point:
 *   - Return value: int32 status, LBM3D_OK (0) or a negative LBM3D_E_* code.
 *     No entry point aborts, throws or prints; lbm3d_strerror() names a code.
 *   - Host arrays are caller-owned; they are read or written during the call
 *     only (inputs are copied, outputs are filled before return).
 *   - Macroscopic fields are host FP64 arrays of nx*ny*nz values laid out
 *     [nz][ny][nx] (x fastest) over the interior (updated) nodes.
 *   - Gas constant R = 1, so the pressure is p = rho T; b = 2/(gamma-1).
 *   - Device state (two f buffers and small work buffers) is owned by the
 *     library, allocated by lbm3d_create and freed by lbm3d_destroy.
 *   - A solver handle is not thread-safe: serialise calls on one handle.
 *     The server object is thread-safe for submit / poll / wait / cancel.
 *   - All device work of a handle runs on its stream, in call order.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
    LBM3D_OK = 0,
    LBM3D_E_INVAL = -1,     /* bad argument: sizes, constants, boundary pairing, rho<=0 or p<=0 */
    LBM3D_E_UNSTABLE = -2,  /* Courant or diffusion number above its limit */
    LBM3D_E_NOMEM = -3,     /* device or host allocation failed, or over a memory budget */
    LBM3D_E_DEVICE = -4,    /* a HIP runtime call failed */
    LBM3D_E_STATE = -5,     /* call out of order (e.g. step before init) */
    LBM3D_E_NONFINITE = -6, /* the solution holds NaN or Inf */
    LBM3D_E_NOTFOUND = -7,  /* unknown server ticket */
    LBM3D_E_CANCELLED = -8  /* the ticket was cancelled */
};

/* ------------------------------------------------------- enumerations ---- */
/* Storage / arithmetic precision.
 *   FP64      f stored and updated in double.
 *   FP32      f stored and updated in float.
 *   FP32_T64  f stored and updated in float; the moment sums (rho, rho u,
 *             energy) and the temperature T = (E/rho - u^2)/b, which cancels
 *             badly at high Mach number, and the equilibrium coefficients
 *             that depend on T and u^2, are computed in double. */
enum { LBM3D_FP64 = 0, LBM3D_FP32 = 1, LBM3D_FP32_T64 = 2 };

/* Boundary kind per face (Sec. 4 (2) gives the last three for (rho, u, T) on
 * the two boundary-node layers; the distributions there are f^eq of those
 * values).  PERIODIC must be set on both faces of an axis. */
enum {
    LBM3D_PERIODIC = 0, /* wrap around */
    LBM3D_OUTFLOW = 1,  /* linear extrapolation from the two nodes next to the face */
    LBM3D_INFLOW = 2,   /* fixed state params.inflow[face] */
    LBM3D_REFLECT = 3   /* wall layer: last node with zero normal velocity; mirror layer: normal velocity negated */
};

/* params.flags bits */
enum {
    LBM3D_NO_DISSIPATION = 1u, /* drop the artificial dissipation term (lambda_i = 0), the paper's comparison variant */
    LBM3D_UPWIND2 = 2u,        /* convection by the second-order upwind difference of the original scheme
                                  (Sec. 3, opening paragraph; Fig. 6) instead of NND: steps run untiled, and
                                  the batched step and servers refuse such solves */
    LBM3D_CHECK_STABILITY = 4u,/* lbm3d_init refuses (E_UNSTABLE) an initial state lbm3d_admit refuses */
    LBM3D_VELOCITY_MAJOR = 8u  /* store each level velocity by velocity (15 blocks of z planes) even where
                                  it is below 2 GiB; by default such levels are stored plane by plane
                                  (the 15 velocity planes of one z side by side), which the tiled step
                                  streams faster.  Results are bitwise the same either way. */
};

/* health bits reported by lbm3d_status (sticky since init) */
enum {
    LBM3D_HEALTH_NONFINITE = 1u, /* some f became NaN or Inf */
    LBM3D_HEALTH_RHO_NONPOS = 2u,/* some node had rho <= 0 */
    LBM3D_HEALTH_T_NONPOS = 4u   /* some node had T <= 0 (can occur transiently at sharp interfaces) */
};

/* --------------------------------------------------------- parameters ---- */
typedef struct {
    int32_t nx, ny, nz;   /* interior nodes per axis (>= 1; >= 2 on an axis with a non-periodic face) */
    double c1, c2, eta0;  /* velocity-model constants of Eq. (vv): nonzero, c1 != c2 */
    double gamma;         /* adiabatic index (> 1); b = 2/(gamma-1) */
    double tau;           /* relaxation time (> 0) */
    double dt;            /* time step (> 0) */
    double dx;            /* grid spacing, the same on all axes (> 0) */
    int32_t bc[6];        /* faces -x, +x, -y, +y, -z, +z: LBM3D_PERIODIC .. LBM3D_REFLECT */
    double inflow[6][5];  /* (rho, ux, uy, uz, p) per LBM3D_INFLOW face; ignored elsewhere */
    int32_t precision;    /* LBM3D_FP64, LBM3D_FP32 or LBM3D_FP32_T64 */
    uint32_t flags;       /* LBM3D_NO_DISSIPATION | LBM3D_UPWIND2 | LBM3D_CHECK_STABILITY | LBM3D_VELOCITY_MAJOR */
} lbm3d_params;

typedef struct lbm3d_solver* lbm3d_t;

/* Library version string (static storage). */
const char* lbm3d_version(void);

/* Name of a status code (static storage; never NULL). */
const char* lbm3d_strerror(int32_t code);

/* Number of visible HIP devices in *count (0 when no GPU). */
int32_t lbm3d_device_count(int32_t* count);

/* Device bytes a solve with these parameters holds (both f buffers with
 * their boundary layers plus work buffers).  Validates like lbm3d_create. */
int32_t lbm3d_footprint(const lbm3d_params* p, size_t* bytes);

/* Validate parameters (E_INVAL / E_UNSTABLE as below), allocate the device
 * state on the current device and return a handle in *out.  The explicit
 * step is admitted only if the Courant number dt/dx * sum_a |v_ia| of the
 * fastest (diagonal) velocity, sqrt(3) c2 dt/dx, is <= 1 and the diffusion
 * number 6 lambda_1 dt/dx^2 = 6 c1 dt/dx is <= 1 (lambda_i of Eq. (lp)). */
int32_t lbm3d_create(const lbm3d_params* p, lbm3d_t* out);

/* Release a handle and its device memory.  NULL is accepted. */
int32_t lbm3d_destroy(lbm3d_t h);

/* Run the handle's device work on an existing hipStream_t (NULL restores the
 * library's own stream).  The caller keeps the stream alive while in use. */
int32_t lbm3d_set_stream(lbm3d_t h, void* hip_stream);

/* Initial state: f_i = f_i^eq(rho, u, T = p/rho) on every interior node
 * (the paper states initial macroscopic fields only), then the boundary
 * layers.  E_INVAL if any rho <= 0 or p <= 0 or a value is not finite.
 * With LBM3D_CHECK_STABILITY in params.flags, E_UNSTABLE (and nothing
 * changed) if lbm3d_admit refuses the state.  Resets the step counter and
 * the health word.  Blocking. */
int32_t lbm3d_init(lbm3d_t h, const double* rho, const double* ux, const double* uy,
                   const double* uz, const double* p);

/* Enqueue nsteps explicit time steps (asynchronous on the handle's stream;
 * runs of steps are replayed from a captured HIP graph).  One step is
 * Sec. 3, Eq. (fi1) applied to Eq. (lp): at every interior node
 *   f_i <- f_i - dt/dx sum_a (h_{I+1/2} - h_{I-1/2})_ia - dt/tau (f_i - f_i^eq)
 *          + lambda_i dt/dx^2 sum_a (f_{I+1} - 2 f_I + f_{I-1})_a,
 * the convection by the NND fluxes of Eq. (nnd) (or the second-order upwind
 * difference with LBM3D_UPWIND2), f^eq of Eqs. (eq)/(e18) from the moments
 * of Eqs. (e1)-(e3), every term at the old level; then the boundary layers
 * of Sec. 4 (2) are refreshed for the new level.  E_STATE before init;
 * E_INVAL for nsteps < 0. */
int32_t lbm3d_step(lbm3d_t h, int64_t nsteps);

/* As lbm3d_step, then wait; *ms receives the device time of the steps
 * measured with HIP events on the handle's stream (ms may be NULL). */
int32_t lbm3d_step_timed(lbm3d_t h, int64_t nsteps, double* ms);

/* Measurement run: enqueue nsteps steps one launch at a time (no graph),
 * each launch of the fused step kernel recording HIP events at its own
 * start and end (hipExtLaunchKernel: the dispatch records them, so no
 * separate markers surround the kernel), then wait.  *total_ms receives
 * the device time of all nsteps steps, *step_kernel_ms the mean duration
 * of one fused-step launch (either pointer may be NULL).  The state
 * advances exactly as lbm3d_step. */
int32_t lbm3d_step_profiled(lbm3d_t h, int64_t nsteps, double* total_ms, double* step_kernel_ms);

/* Launch shape of the fused step kernel: a tile is 64 x `by` nodes in x-y
 * and `tz` nodes deep in z (by = 2, 4 or 8 -- 8 in the FP32 modes only --
 * or 0 for the untiled one-node-per-thread kernel; tz >= 1).  Results are
 * bitwise independent of the shape.  E_INVAL for an unsupported shape.
 * The store kind (below) is kept. */
int32_t lbm3d_set_tile(lbm3d_t h, int32_t by, int32_t tz);
int32_t lbm3d_get_tile(lbm3d_t h, int32_t* by, int32_t* tz);

/* Store kind of the tiled kernels' new level: 1 = non-temporal (streaming
 * past the caches), 0 = plain.  A solve starts with plain stores when its
 * two distribution levels fit in 320 MiB (the next step then reads much of
 * its input from the 256 MB memory-side cache), else with non-temporal
 * ones; the autotuner picks it with the shape.  Results are bitwise
 * independent of it; the untiled kernel always stores plainly and the
 * batched step non-temporally.  E_INVAL for a value other than 0 or 1. */
int32_t lbm3d_set_streaming(lbm3d_t h, int32_t streaming);
int32_t lbm3d_get_streaming(lbm3d_t h, int32_t* streaming);

/* Autotuner of the launch shape.  Times every supported tile shape with
 * both store kinds (and the untiled kernel) over `launches` steps each (<= 0: 10), in three
 * interleaved rounds, with HIP events on the solver's stream.  The trials
 * are real steps (alternating buffers, boundary layers included); the
 * current level and the health word are copied to temporary device memory
 * (one distribution buffer) first and restored afterwards, so the solve's
 * state and step count are unchanged (without memory for the copy, each
 * trial recomputes the current level instead).  Keeps the shape with the
 * fastest round (as lbm3d_set_tile) and remembers it for the
 * process: later lbm3d_create calls for the same precision, grid and
 * boundary kinds start with it.  Blocking.  by / tz (may be NULL) receive
 * the shape.  E_STATE before lbm3d_init. */
int32_t lbm3d_tune(lbm3d_t h, int32_t launches, int32_t* by, int32_t* tz);

/* On-disk cache of the autotuner's results (the tile shape and store kind
 * per precision, grid and boundary kinds, and the batch tile depth per
 * precision), so that a later process starts with the tuned shapes without
 * tuning again.  The file is text: a header "lbm3d-tune 2 <arch>" naming the
 * GPU architecture (gcnArchName, "none" without a device) the shapes were
 * timed on, then lines
 * "tile <precision> <nx> <ny> <nz> <six boundary kinds> <by> <tz> <streaming>"
 * and "batch <precision> <tz>".
 * lbm3d_tune_save writes every result of this process (atomically: a
 * temporary file renamed over `path`); E_INVAL if it cannot be written.
 * lbm3d_tune_load merges a file's results into this process's: E_NOTFOUND
 * if it cannot be opened, E_INVAL (and nothing merged) if it is not such a
 * file, was written for another architecture, or holds a bad line.
 * With the environment variable LBM3D_TUNE_CACHE set to a path, that file is
 * loaded (errors ignored) before the first lookup of the process, and saved
 * after every lbm3d_tune and lbm3d_batch_tune. */
int32_t lbm3d_tune_save(const char* path);
int32_t lbm3d_tune_load(const char* path);

/* Wait for all work enqueued on the handle's stream. */
int32_t lbm3d_sync(lbm3d_t h);

/* Von Neumann stability analysis of the scheme (Sec. 3, the amplification
 * matrix G_ij of a Fourier mode about a uniform equilibrium): the largest
 * eigenvalue modulus max|omega| of G over nk wave numbers k dx spaced evenly
 * in [kdx_lo, kdx_hi] (nk = 1: kdx_lo only).  q = (rho, ux, uy, uz, T) is
 * the uniform state (rho, T > 0).  axis 0, 1, 2 puts the wave vector along
 * x, y or z; 3 gives every axis the same k dx.  alpha_t is the limiter's
 * linearisation parameter of the NND symbol (|alpha_t| < 1/2; 0 for the
 * paper's figures).  Uses c1, c2, eta0, gamma, tau, dt, dx and the
 * no-dissipation and second-order-upwind flags of p (with LBM3D_UPWIND2 the
 * convection symbol is (3 - 4 e^{-ik dx} + e^{-2ik dx}) / 2, mirrored for
 * v < 0; grid sizes and boundaries must be valid but do not enter);
 * parameters the step would reject as E_UNSTABLE are analysed
 * too.  *max_omega receives the maximum and *kdx_at_max (may be NULL) the
 * k dx where it occurs.  Host computation only, no device work; the
 * eigenvalue modulus is taken from the growth of G^(2^20), accurate to
 * about 1e-5.  E_INVAL for bad arguments. */
int32_t lbm3d_stability(const lbm3d_params* p, const double* q, int32_t axis, double kdx_lo,
                        double kdx_hi, int32_t nk, double alpha_t, double* max_omega,
                        double* kdx_at_max);

/* Stability admission of an initial state (the von Neumann analysis of
 * Sec. 3 with the paper's rule of thumb turned into a check): the largest
 * max |omega| of lbm3d_stability over k dx in [0, pi] (33 points, alpha_t =
 * 0) along x, y, z and the diagonal, at the fastest node (largest |u|), the
 * coldest and the hottest node of the initial fields (host FP64, nx*ny*nz
 * each, as lbm3d_init) and at every fixed inflow state.  Returns LBM3D_OK
 * if it is at most 1 + 1e-3 (the paper calls its Fig. 3 setting, 1.0009 in
 * this analysis, stable), else E_UNSTABLE; *max_omega (may be NULL)
 * receives it.  Host only.  E_INVAL / E_UNSTABLE from parameter validation
 * as lbm3d_create; E_INVAL for rho <= 0 or p <= 0. */
int32_t lbm3d_admit(const lbm3d_params* p, const double* rho, const double* ux, const double* uy,
                    const double* uz, const double* pr, double* max_omega);

/* Diagnostic, not part of the scheme: the device's practical streaming
 * rate for a kernel like the time step.  Copies `bytes` (rounded down to
 * 16) back and forth between two device buffers it allocates and frees,
 * one float4 per thread with non-temporal stores, `launches` round trips
 * after two warm-up ones, timed with HIP events.  *gbs receives the bytes
 * read plus written per second in GB/s.  Blocking.  E_INVAL for bytes <
 * 4096, launches < 1 or gbs NULL; E_NOMEM if the buffers do not fit. */
int32_t lbm3d_stream_copy_rate(int64_t bytes, int32_t launches, double* gbs);

/* (rho, u, p = rho T) on the interior nodes into caller arrays of nx*ny*nz
 * doubles each (any pointer may be NULL to skip that field): the moments of
 * Sec. 2, Eqs. (e1)-(e3), applied to f (rho = sum f, rho u = sum f v,
 * rho (b T + u^2) = sum f (v^2 + eta^2)), in FP64 in the FP64 and FP32_T64
 * modes.  Blocking.  Returns E_NONFINITE (after filling the arrays) if the
 * health word has the NONFINITE bit; E_STATE before init. */
int32_t lbm3d_moments(lbm3d_t h, double* rho, double* ux, double* uy, double* uz, double* p);

/* Domain totals over the interior nodes of the densities the scheme
 * conserves (Sec. 2, Eqs. (e1)-(e3): the collision invariants 1, v and
 * (v^2 + eta^2)/2 summed against f), accumulated in FP64 with a fixed
 * reduction order (bitwise reproducible): out[0] mass sum rho, out[1..3]
 * momentum sum rho u, out[4] energy sum rho (b T + u^2)/2.  On periodic
 * boxes they are conserved to rounding.  Blocking; E_STATE before init. */
int32_t lbm3d_conserved(lbm3d_t h, double out[5]);

/* Health bits (LBM3D_HEALTH_*) accumulated since init, and steps done. */
int32_t lbm3d_status(lbm3d_t h, uint32_t* health, int64_t* steps_done);

/* Debug aid: fill the buffer the next step writes (interior, boundary
 * layers and padding) with NaN, then restore its fixed-state layers (which
 * the steps never rewrite).  A correct step reads nothing it has not
 * written, so the results stay bitwise the same; a stale read shows up as
 * NaN.  Blocking.  E_STATE before lbm3d_init. */
int32_t lbm3d_poison_next(lbm3d_t h);

/* Checkpoint: the interior distributions as [15][nz][ny][nx] in storage
 * precision (double for FP64, float otherwise); bytes must equal
 * 15*nx*ny*nz*elem.  Velocity order: rest; c1 (+x, -x, +y, -y, +z, -z);
 * then (c2/sqrt3)(sx, sy, sz) with bit a of the index-7 giving the sign of
 * axis a (clear = +).  Blocking. */
int32_t lbm3d_get_f(lbm3d_t h, void* host, size_t bytes);

/* Restore distributions written by lbm3d_get_f (same layout and size) and
 * refresh the boundary layers; the step counter is left unchanged. */
int32_t lbm3d_set_f(lbm3d_t h, const void* host, size_t bytes);

/* Advance `count` independent solves (any mix of sizes, all of the same
 * precision) by nsteps[k] steps each: the time step of Sec. 3, Eqs. (nnd),
 * (lp), (fi1), applied to every member.  The group runs max(nsteps) steps,
 * each one launch of a persistent kernel whose workgroups take 64 x BY x TZ
 * tiles from per-XCD work lists (see lbm3d_batch_plan); a member takes part
 * while it has steps to do (a device-side count per member, advanced by a
 * small launch after each step), and runs of 16 steps are replayed from a
 * captured HIP graph.  Results are bitwise identical to stepping each solve
 * alone.  Blocking.  E_INVAL for mixed precisions, duplicate or NULL
 * handles, count < 1, a negative step count, a solve with the
 * second-order upwind flag, or one beyond the tiled kernels' 32-bit
 * offsets (a velocity-major level whose velocity block reaches 2 GiB).
 * E_STATE if a member is not initialised. */
int32_t lbm3d_batch_step(lbm3d_t* hs, int32_t count, const int64_t* nsteps);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same
 * step as lbm3d_batch_step, with the same arguments, errors and results
 * (bitwise), that allocates nothing.  Its work tables (the solve table,
 * tile lists, counters, boundary-layer jobs, step counts and health words) go into a
 * static device array of 4 MiB per device, held until the process ends,
 * instead of a hipMalloc'd buffer; they are copied there from host memory
 * with hipMemcpyAsync on the first member's stream, and every step is
 * launched directly (no graph is instantiated).  4 MiB holds the tables of
 * up to about 200,000 tiles (20 B each, plus about 0.5 KB per solve); the
 * benchmark's mix of 64 uneven solves needs about 0.1 MB at the default tile depth.
 * E_NOMEM, before any device work, for a batch whose tables exceed it.
 * All calls on one device share the array: calls that overlap on one device
 * (from several threads or streams) race and must be serialised.  Like
 * lbm3d_batch_step it waits for the first member's stream before returning,
 * so it cannot itself be recorded into a stream capture. */
int32_t lbm3d_batch_step_noalloc(lbm3d_t* hs, int32_t count, const int64_t* nsteps);

/* Work plan of the batched step, computed on the host (no device work): the
 * tiles of solves with parameters ps[0..count-1] (validated as lbm3d_create,
 * all of one precision) at tile depth tz (0: the tuned depth of the
 * precision, else a launch model's for these solves; < 0: the model's; a
 * depth at or beyond a solve's nz gives whole columns), for a device of
 * `cus` compute units.  Tiles are 64 x BY nodes in x-y (BY = 4 in FP64, 8
 * otherwise).  Each solve's tiles are cut into contiguous row slabs, the
 * slabs are dealt to up to 8 lists (one per XCD) largest first onto the
 * least-loaded list, and each list runs its deepest tiles first.
 * *ntiles, *nlists and *nblocks (persistent workgroups, a multiple of the
 * list count) may be NULL.  If `tiles` is not NULL it receives, list by
 * list, 7 int32 per tile: solve index, x0, x1, y0, y1, z0, z1 (node ranges
 * [x0, x1) etc.); `cap` is its room in tiles (E_NOMEM if too small).
 * list_first (9 int32, may be NULL) receives the list boundaries in tiles.
 * E_INVAL / E_UNSTABLE as lbm3d_create, E_INVAL for mixed precisions. */
int32_t lbm3d_batch_plan(const lbm3d_params* ps, int32_t count, int32_t tz, int32_t cus, int32_t* ntiles,
                         int32_t* nlists, int32_t* nblocks, int32_t* tiles, int64_t cap, int32_t* list_first);

/* Autotuner of the batched step: times the persistent launch over the given
 * solves (same rules as lbm3d_batch_step) for tile depths 16, 32, 64 and 128
 * (a depth at or beyond a solve's nz gives whole columns), over `launches`
 * steps each (<= 0: 5) in three interleaved rounds, as real steps over
 * alternating buffers with the solves' current levels and health words
 * saved to temporary device memory and restored afterwards (states
 * unchanged; without memory for the copies each trial recomputes the
 * current levels), and keeps the depth with the fastest round for every later batched
 * step (lbm3d_batch_step) of that precision in this process.  Servers do
 * not use it: their membership changes from tick to tick, and each of
 * their plans takes the launch model's depth for its members (the
 * persistent workgroups share the tiles' planes, and no launch ends before
 * its longest tile).
 * Blocking.  *tz (may be NULL) receives the depth. */
int32_t lbm3d_batch_tune(lbm3d_t* hs, int32_t count, int32_t launches, int32_t* tz);

/* Tile depth of later batched steps (lbm3d_batch_step) of one precision
 * in this process, as the autotuner would set it; 0 restores the default
 * (the launch model's depth for each batch).  Results do not depend on it.
 * E_INVAL for a bad precision or tz outside [0, 65535]. */
int32_t lbm3d_batch_set_depth(int32_t precision, int32_t tz);

/* ------------------------------------------------------------- serving --- */
typedef struct lbm3d_server* lbm3d_server_t;

typedef struct {
    double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
    int64_t steps;                    /* steps done */
    uint32_t health;                  /* LBM3D_HEALTH_* of the solve */
} lbm3d_timing;

/* A server owns a worker thread that admits submitted solves while their
 * device footprint fits in hbm_budget_bytes and fewer than max_active are
 * running, keeps their state resident on the device, advances all active
 * solves together in batched ticks (continuous batching: solves admitted
 * between ticks join the next one; within a tick each solve takes only the
 * steps it still needs), and completes a ticket when its solve has done its
 * steps, or early, with E_NONFINITE, after the first tick that leaves it
 * non-finite.  A second thread creates and initialises admitted solves and
 * reads back finished ones while the ticks run.  Solves of any precision
 * may be mixed; each tick groups them by precision. */
int32_t lbm3d_server_create(size_t hbm_budget_bytes, int32_t max_active, lbm3d_server_t* out);

/* Steps per batched tick (default 32): solves submitted during a tick join
 * at the next one, so a shorter tick admits sooner and a longer one
 * amortises more launches. */
int32_t lbm3d_server_set_tick(lbm3d_server_t s, int64_t steps);

/* Queue a solve.  Parameters and the five initial fields are copied; returns
 * immediately with a ticket.  E_NOMEM if the solve alone exceeds the budget;
 * E_INVAL / E_UNSTABLE as lbm3d_create, E_INVAL also for a solve the
 * batched kernel cannot take (see lbm3d_batch_step). */
int32_t lbm3d_server_submit(lbm3d_server_t s, const lbm3d_params* p, const double* rho,
                            const double* ux, const double* uy, const double* uz,
                            const double* pr, int64_t nsteps, uint64_t* ticket);

/* *done = 1 once the ticket's result is ready (or it failed / was cancelled). */
int32_t lbm3d_server_poll(lbm3d_server_t s, uint64_t ticket, int32_t* done);

/* Block until the ticket completes, copy its (rho, u, p) into caller arrays
 * (any may be NULL) and its timing into *t (may be NULL), then forget the
 * ticket.  Returns the solve's own status (E_NONFINITE, E_CANCELLED, ...).
 * One thread may wait on a ticket: a second concurrent waiter gets E_STATE,
 * and a wait after the ticket was collected gets E_NOTFOUND. */
int32_t lbm3d_server_wait(lbm3d_server_t s, uint64_t ticket, double* rho, double* ux,
                          double* uy, double* uz, double* p, lbm3d_timing* t);

/* Counters of a server since its creation (a snapshot). */
typedef struct {
    int64_t ticks;      /* batched ticks run */
    int64_t rebuilds;   /* work plans rebuilt for a changed membership */
    int64_t admitted;   /* solves admitted */
    int64_t completed;  /* solves finished (done, failed or evicted) */
    int64_t evicted;    /* solves stopped before their last step because they went non-finite */
    double wall_s;      /* seconds since the server was created */
    double busy_s;      /* device time of the ticks' launches (HIP events around each tick) */
    double admit_s;     /* host time creating and initialising admitted solves */
    double plan_s;      /* host time rebuilding work plans (planning and table upload) */
    double finish_s;    /* host time reading back and freeing finished solves */
} lbm3d_server_counters;

int32_t lbm3d_server_stats(lbm3d_server_t s, lbm3d_server_counters* out);

/* Cancel a queued or running ticket; a later wait returns E_CANCELLED. */
int32_t lbm3d_server_cancel(lbm3d_server_t s, uint64_t ticket);

/* Stop the worker (running solves are cancelled) and free everything. */
int32_t lbm3d_server_destroy(lbm3d_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
