/*
 * hosc.h -- C ABI of libhosc, an MI355X (gfx950) implementation of the hot path of
 * the higher-order super-compact (HOSC) finite-difference scheme for natural
 * convection of a power-law fluid in a differentially heated cubic cavity
 * (Punia & Ray, arXiv 2411.06563).
 *
 * Problem (Sec. 2.1): unit cube, x = 0 hot wall (theta = theta_hot), x = 1 cold
 * wall (theta = theta_cold), the other four walls adiabatic; no-slip on every wall;
 * zero wall-normal pressure derivative; gravity along -y (buoyancy in the v
 * equation); power-law viscosity eta = I2^((n-1)/2) (Eqs. 6-8); dimensionless
 * groups Ra and Pr.  Each time step (Sec. 2.2) assembles the compact (19,7) stencil
 * of the generic transport PDE (Eq. 1) for u, v, w and theta from level-n fields,
 * solves the four 7-point implicit systems at level n+1, and applies the modified
 * artificial-compressibility pressure correction; diagnostics give the Nusselt
 * numbers (Sec. 4.2), entropy generation and Bejan number (Sec. 4.3).
 *
 * Conventions for every function:
 *   - The return value is an hosc_status; HOSC_OK (0) is success.  No C++
 *     exception crosses the ABI.  hosc_last_error() gives a message for the last
 *     failing call on a handle (valid until the next call on that handle).
 *   - Fields are N^3 arrays of double holding every node of the cube including the
 *     walls, x fastest: node (i, j, k) at index i + N*(j + N*k), x_i = i/(N-1).
 *   - Host arrays are copied synchronously on the solver's stream; the call returns
 *     after the copy.  The library never frees caller memory.
 *   - Device memory: the caller supplies one workspace buffer of at least
 *     hosc_workspace_bytes() bytes (e.g. a torch tensor); the library only carves it
 *     and never allocates device memory for a solver.  The workspace must stay
 *     valid and untouched by the caller until hosc_destroy().
 *   - A handle may be used by one host thread at a time.  All device work of a
 *     handle is ordered on the stream given at creation.
 *   - Errors HOSC_E_NONFINITE and HOSC_E_NOCONV are sticky: the handle refuses to
 *     step until hosc_set_state() or hosc_init_fields() resets it.
 */
#ifndef HOSC_H
#define HOSC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HOSC_OK = 0,
    HOSC_E_ARG = -1,        /* invalid argument or parameter */
    HOSC_E_NOMEM = -2,      /* workspace too small */
    HOSC_E_DEVICE = -3,     /* a HIP call failed */
    HOSC_E_NOCONV = -4,     /* an implicit solve hit solve_maxit sweeps or iterations, or BiCGSTAB's
                               residual did not halve within 400 iterations */
    HOSC_E_NONFINITE = -5,  /* a residual or divergence became NaN/Inf */
    HOSC_E_STATE = -6,      /* handle in a sticky error state / no state set */
    HOSC_E_BUDGET = -7      /* (server) one request exceeds the whole budget */
} hosc_status;

typedef enum {
    HOSC_FP64 = 0,          /* every stage in FP64 */
    HOSC_FP32_REFINED = 1   /* FP32 implicit matrix and inner sweeps, FP64 residual refinement */
} hosc_precision;

/* Solver of the 7-point implicit systems (Sec. 2.2 uses BiCGSTAB without
 * preconditioning because SOR fails where the rows lose diagonal dominance). */
typedef enum {
    HOSC_SOLVER_AUTO = 0,       /* red-black SOR; a system whose SOR residual stalls or grows is
                                   re-solved with BiCGSTAB (kept for the next 50 steps) */
    HOSC_SOLVER_SOR = 1,        /* red-black SOR only (fails with HOSC_E_NOCONV / NONFINITE) */
    HOSC_SOLVER_BICGSTAB = 2    /* BiCGSTAB on the diagonally scaled rows only */
} hosc_solver_kind;

/* Parameters of one cavity (Sec. 2.1 problem statement, Sec. 2.2 scheme). */
typedef struct hosc_params {
    int32_t N;              /* nodes per side including walls, 5 <= N <= 1025; h = 1/(N-1) */
    int32_t precision;      /* hosc_precision */
    double Ra;              /* Rayleigh number, >= 0 */
    double Pr;              /* Prandtl number, > 0 */
    double n_pl;            /* power-law index n, 0 < n <= 2 (1 = Newtonian) */
    double dt;              /* time step, > 0 */
    double theta_hot;       /* theta on x = 0 (default 1) */
    double theta_cold;      /* theta on x = 1 (default 0) */
    double theta_ref;       /* buoyancy reference: Ra Pr (theta - theta_ref) (default 0.5) */
    double lambda;          /* artificial-compressibility relaxation; 0 -> h^2/(3 dt) */
    double div_tol;         /* correct p when max|div v| > div_tol (default 0: every step) */
    double solve_rtol;      /* stop a solve when ||r|| <= solve_rtol ||b|| (diagonally scaled 2-norms), default 1e-10 */
    int32_t solve_maxit;    /* cap on red-black sweeps (or BiCGSTAB iterations) per solve (default 4000) */
    int32_t check_every;    /* sweeps between convergence checks; 0 -> adaptive */
    int32_t solver;         /* hosc_solver_kind (default HOSC_SOLVER_AUTO) */
    int32_t p_iters;        /* pressure iterations (Sec. 2.2): momentum solves per step at most.
                               After a momentum solve whose trial velocity has max|div v| > div_tol
                               the pressure is corrected (p <- p - lambda div v) and, while fewer
                               than p_iters solves were made, the momentum sources are re-formed
                               from level n with the corrected pressure and the momentum increments
                               solved again.  0 or 1: one solve and at most one correction per step
                               (default 1); at most 64.  In batches and the server the re-solves of a
                               cavity run as single-cavity launches after the fused solve. */
    double omega;           /* SOR relaxation of the red-black sweeps: 0 = adaptive per system (default),
                               else fixed in (0, 2) */
    double i2_floor;        /* eta = max(I2, i2_floor)^((n-1)/2), default 1e-8 */
    double phi;             /* irreversibility ratio of the fluid-friction entropy, default 1e-4 */
    double eta_relax;       /* viscosity relaxation for steady-state marching (an addition to the
                               paper's scheme): the viscosity of level n is r eta(v^n) + (1 - r) times
                               that of level n-1, r = eta_relax in (0, 1].  1 (default) is the stated
                               scheme; r < 1 damps the period-2 oscillation the lagged viscosity can
                               sustain and leaves every steady state unchanged (a fixed point of
                               both).  The first step after a state is set uses eta(v^n). */
} hosc_params;

/* Per-step report. */
typedef struct hosc_step_info {
    double res[4];          /* steady residual ||chi^{n+1}-chi^n||_2/||chi^{n+1}||_2 of u, v, w, theta */
    double relres[4];       /* last measured relative residual of each implicit solve */
    double maxdiv;          /* max |div v^{n+1}| over interior nodes of the accepted velocity, before
                               its correction */
    int64_t step;           /* steps taken since the state was set */
    int32_t sweeps[2];      /* red-black sweeps of the momentum and the energy solve (last step) */
    int32_t bicg_iters[2];  /* BiCGSTAB iterations of the momentum and the energy solve (last step) */
    double omega[2];        /* SOR relaxation of the momentum and the energy sweeps after the last step */
    double dominance[2];    /* max over rows of (sum |off-diagonal|) / |centre| of the momentum and energy
                               matrices (> 1: a row is not diagonally dominant); 0 if not measured */
    int32_t corrected;      /* pressure corrections applied in the step (0 .. p_iters; 0 or 1 with one
                               pressure iteration) */
    int32_t status;         /* hosc_status of the step */
} hosc_step_info;

/* Scalar diagnostics (Secs. 4.2, 4.3). */
typedef struct hosc_diag {
    double nu_mean_hot;     /* int int Nu dy dz on x = 0, Nu = -d theta/dx */
    double nu_mean_cold;    /* same on x = 1 */
    double nu_max_hot;      /* max_z Nu_avg(z) on x = 0 (the quantity of Table 2) */
    double nu_max_cold;
    double e_total;         /* int E_local dV */
    double e_ht;            /* int E_HT dV, E_HT = |grad theta|^2 */
    double e_ff;            /* int E_FF dV, E_FF = phi eta I2 */
    double be_global;       /* int E_HT / int E_local */
    double be_mean;         /* int (E_HT / E_local) dV */
    double nu_local_max_hot;/* max over the hot wall of Nu_local */
} hosc_diag;

/* Kernel timing of the implicit solves (HIP events around every sweep launch) and
 * their algorithmic HBM bytes: per launch, each updated node reads its stored row
 * (momentum s, a_x, a_y, a_z, b_u, b_v, b_w; energy a_x, a_y, a_z, b), reads and
 * writes its own increments, and each node of the other colour is read once. */
typedef struct hosc_perf {
    int64_t sweep_launches;     /* half-sweep kernel launches timed */
    double sweep_ms;            /* summed kernel time of those launches */
    double sweep_bytes;         /* summed algorithmic bytes of those launches */
    int64_t assemble_launches;
    double assemble_ms;
    double assemble_bytes;
    int64_t bicg_launches;      /* BiCGSTAB vector-phase launches (matrix-vector products and updates) */
    double bicg_ms;
    double bicg_bytes;          /* per launch: rows of the active systems once, each vector read or written once */
    int64_t refine_launches;    /* precision mode: FP64 refinement passes (one launch over both colours each) */
    double refine_ms;
    double refine_bytes;
} hosc_perf;

typedef struct hosc_solver hosc_solver;

/* Fill p with the defaults (N = 17, Ra = 1e3, Pr = 1, n = 1, dt = 1e-4, ...). */
hosc_status hosc_params_default(hosc_params *p);

/* Device bytes a solver with these parameters needs (for admission by budget).
 * Fails with HOSC_E_ARG on invalid parameters. */
hosc_status hosc_workspace_bytes(const hosc_params *p, size_t *bytes);

/* Create a solver on the current HIP device.  d_ws: device buffer of ws_bytes >=
 * hosc_workspace_bytes(p), 256-byte aligned; stream: where all work is ordered
 * (0 = null stream).  The state is unset until hosc_init_fields / hosc_set_state.
 * Allocates only pinned host memory: a staging buffer and a mapped, coherent copy
 * of the reduction results, which the kernels write and the convergence checks read
 * (HOSC_E_DEVICE if that allocation fails). */
hosc_status hosc_create(const hosc_params *p, void *d_ws, size_t ws_bytes, hipStream_t stream, hosc_solver **out);

/* Release the handle (not the workspace).  Accepts NULL. */
hosc_status hosc_destroy(hosc_solver *s);

/* Initial condition of the cavity runs: u = v = w = p = 0; theta = theta_hot +
 * (theta_cold - theta_hot) x + noise_amp (2U - 1) at interior nodes, U uniform in
 * [0,1) from SplitMix64 seeded with seed, one draw per interior node in storage
 * order; then the boundary conditions.  Resets the step counter (level n-1 is
 * taken equal to level n at the next step). */
hosc_status hosc_init_fields(hosc_solver *s, uint64_t seed, double noise_amp);

/* Set level n from host arrays (any pointer may be NULL: that field becomes 0).
 * apply_bc != 0 imposes the boundary conditions (no-slip, wall temperatures, zero
 * normal derivative of theta on the y/z walls and of p everywhere by the closure
 * f_0 = (4 f_1 - f_2)/3).  Resets the step counter and clears sticky errors. */
hosc_status hosc_set_state(hosc_solver *s, const double *u, const double *v, const double *w, const double *theta,
                           const double *p, int32_t apply_bc);

/* Copy level n to host arrays (any pointer may be NULL). */
hosc_status hosc_get_state(hosc_solver *s, double *u, double *v, double *w, double *theta, double *p);

/* Advance nsteps time steps (Sec. 2.2).  Each step ends with the Nusselt, entropy
 * and Bejan reductions of the new level (hosc_diagnostics then returns them
 * without recomputing).  info (may be NULL) reports the last step.  nsteps = 0
 * takes no step; HOSC_E_ARG for nsteps < 0, HOSC_E_STATE before a state was set or
 * after a step failed with HOSC_E_NOCONV or HOSC_E_NONFINITE (sticky until
 * hosc_set_state or hosc_init_fields). */
hosc_status hosc_step(hosc_solver *s, int32_t nsteps, hosc_step_info *info);

/* Step until max_f res[f] < res_tol or max_steps steps were taken (max_steps = 0:
 * no step, info untouched).  HOSC_E_ARG for res_tol <= 0 or max_steps < 0,
 * HOSC_E_STATE before a state was set or in a sticky error state; a failing step's
 * status otherwise. */
hosc_status hosc_run_to_steady(hosc_solver *s, double res_tol, int64_t max_steps, hosc_step_info *info);

/* Nusselt, entropy and Bejan diagnostics of level n (those of the step that produced
 * it, or computed now after a state was set).  Optional host outputs (may
 * be NULL): nuavg_hot[N], nuavg_cold[N] (Nu_avg(z_k)); nu_hot[N*N], nu_cold[N*N]
 * (Nu_local at node (j, k) stored at j + N*k). */
hosc_status hosc_diagnostics(hosc_solver *s, hosc_diag *d, double *nuavg_hot, double *nuavg_cold, double *nu_hot,
                             double *nu_cold);

/* Local entropy generation E_local and local Bejan number at every node (host N^3
 * arrays; either may be NULL). */
hosc_status hosc_entropy_fields(hosc_solver *s, double *e_local, double *be_local);

/* Monitoring points (the probes of the grid-independence study, Sec. 3.1, Table 1):
 * u, v, w, theta and p of level n at n points of the closed unit cube, each by
 * trilinear interpolation of the eight surrounding nodes (a point on a node returns
 * that node's values).  xyz: host, n x 3 (x, y, z of each point, every coordinate
 * in [0, 1]); out: host, n x 5 (u, v, w, theta, p of each point).  1 <= n <=
 * min(4096, N^3/8).  Fails with HOSC_E_ARG on a bad count or coordinate and
 * HOSC_E_STATE before a state was set.  Synchronous on the solver's stream. */
hosc_status hosc_probe(hosc_solver *s, const double *xyz, int32_t n, double *out);

/* Parity hook: assemble the step from the current state without advancing it.
 * Outputs (host, any may be NULL): eta[N^3], estar[3 N^3] (E*_u, E*_v, E*_w),
 * b[4 N^3] right-hand sides of the u, v, w, theta increment systems (walls 0),
 * Bmom[7 N^3], Btheta[7 N^3]: the 7-point weights of the implicit operators in the
 * order centre, x+, x-, y+, y-, z+, z- (walls 0; theta rows before the wall closure).
 * When the step counter is 0, level n-1 is taken equal to level n. */
hosc_status hosc_debug_assemble(hosc_solver *s, double *eta, double *estar, double *b, double *Bmom,
                                double *Btheta);

/* One HOSC step of the generic transport PDE (Sec. 2.2, Eq. 1 with K* = 0):
 *     L chi_t + G* chi_x + H* chi_y + I* chi_z - lap chi = E*
 * with coefficient fields given by the caller instead of formed from the cavity's
 * state (the hook the momentum and energy equations are instances of; it serves
 * convergence tests against manufactured solutions).  Host N^3 arrays, x fastest:
 * L, G, H, I, E at level n and Lp, Gp, Hp, Ip, Ep at level n-1 (only their values at
 * the interior nodes enter, through the time differences; pass level n again at a
 * first step); E and Ep may both be NULL (zero source).  chi: level n, every node.
 * chi_new: on entry its wall nodes hold the Dirichlet values of level n+1 (its
 * interior is ignored); on return its interior holds level n+1.  The implicit
 * system is solved as the momentum systems are (solver, solve_rtol, solve_maxit and
 * precision of the solver's parameters; N and dt from them too; Ra, Pr, n and the
 * other physical parameters are not used).  info (may be NULL): relres[0],
 * sweeps[0], bicg_iters[0], omega[0], dominance[0] of the solve and res[0] =
 * ||chi_new - chi||_2 / ||chi_new||_2 over all nodes; other entries 0.
 * The call uses the solver's workspace for the coefficients: afterwards the solver
 * has no state (hosc_step and hosc_get_state fail with HOSC_E_STATE until
 * hosc_set_state or hosc_init_fields).  HOSC_E_ARG for a missing array or only one
 * of E, Ep; HOSC_E_NOCONV / HOSC_E_NONFINITE from the solve.  Synchronous. */
hosc_status hosc_transport_step(hosc_solver *s, const double *L, const double *G, const double *H, const double *I,
                                const double *E, const double *Lp, const double *Gp, const double *Hp,
                                const double *Ip, const double *Ep, const double *chi, double *chi_new,
                                hosc_step_info *info);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the diagnostics of
 * hosc_diagnostics (same kernels, same values) computed from the caller's device
 * fields, with every intermediate (Simpson weights, local and z-averaged Nusselt
 * numbers, partial sums) in one fixed device array of the library of 2.7 MB, held
 * on each device the library is used on until the process ends.  Allocates
 * nothing, never synchronises: launches only, on `stream` (a stream of the
 * current device; the first call on a device looks up the array's address there).
 * p: the cavity's parameters, validated as by hosc_create; N <= 257 (HOSC_E_ARG
 * above: that is the array's limit); n_pl, i2_floor and phi are used.
 * d_u, d_v, d_w, d_theta: device N^3 fields of one state (x fastest), not modified.
 * d_out: device, 10 doubles: the hosc_diag fields in declaration order.
 * d_nuavg_hot, d_nuavg_cold: device N doubles each (Nu_avg(z_k)), or NULL.
 * Every call on a device shares its array, whose contents are the last call's and
 * are fully rewritten by the next: calls that overlap on one device (different
 * streams, or host threads) race; order them on one stream.  Errors (HOSC_E_ARG,
 * HOSC_E_DEVICE) are reported through hosc_last_error(NULL). */
hosc_status hosc_diagnostics_noalloc(const hosc_params *p, const double *d_u, const double *d_v, const double *d_w,
                                     const double *d_theta, double *d_out, double *d_nuavg_hot, double *d_nuavg_cold,
                                     hipStream_t stream);

/* Switch kernel timing on (on != 0, counters cleared) or off.  Timing adds two
 * event records per timed launch on the solver's stream. */
hosc_status hosc_perf_enable(hosc_solver *s, int32_t on);

/* Counters accumulated since the last hosc_perf_enable(s, 1). */
hosc_status hosc_perf_get(hosc_solver *s, hosc_perf *out);

/* Achievable-bandwidth probe (measurement aid, not part of the method): copies
 * `bytes` (multiple of 16, both device buffers 16-byte aligned, not overlapping)
 * from d_src to d_dst `reps` times on `stream` with a plain 16-byte-per-lane copy
 * kernel and returns the mean kernel time per copy (HIP events).  Each copy moves
 * 2 * bytes through HBM (read + write). */
hosc_status hosc_copy_bandwidth(const void *d_src, void *d_dst, size_t bytes, int32_t reps, hipStream_t stream,
                                double *ms_per_copy);

/* Streaming probe with the access mix of a red-black half-sweep (measurement aid,
 * not part of the method).  A half-sweep reads 19 and writes 4 elements per
 * updated node (rows, right-hand sides, own and neighbouring increments; the own
 * increments rewritten in place); the probe streams 15 read-only arrays, carved
 * one after another from d_read (15 * bytes), and 4 arrays that it reads and
 * rewrites in place, from d_inplace (4 * bytes): `bytes` per array, a multiple of
 * 16, both buffers 16-byte aligned and not overlapping; one 16-byte element of
 * every array per thread.  One warm-up launch, then `reps` launches on `stream`;
 * returns the mean kernel time per launch (HIP events).  A launch moves
 * 23 * bytes through HBM; d_inplace's contents change (each element becomes half
 * itself plus the sum of the read elements), d_read is only read.  HOSC_E_ARG for
 * null or misaligned buffers, overlap, bytes = 0 or reps < 1. */
hosc_status hosc_stream_mix_bandwidth(const void *d_read, void *d_inplace, size_t bytes, int32_t reps,
                                      hipStream_t stream, double *ms_per_launch);

/* Message of the last failing call on the handle ("" if none; NULL handle: last
 * failing create). */
const char *hosc_last_error(const hosc_solver *s);

/* Name of a status code. */
const char *hosc_status_string(hosc_status st);

/* ------------------------------------------------------------------------------
 * Batches: many cavities (any mix of N, Ra, Pr, n, dt; one precision) advanced
 * together on one stream.  Each cavity is an hosc_solver carved from the batch
 * workspace; the implicit solves of all cavities run as fused launches (one
 * persistent launch per red-black half-sweep and per refinement pass (both
 * colours) over every cavity still iterating, one launch for all reductions and one host
 * copy per convergence check), while each cavity keeps exactly the arithmetic and
 * solver decisions of its single-cavity run, so a cavity's results do not depend
 * on the batch it is in.
 * ------------------------------------------------------------------------------ */
typedef struct hosc_batch hosc_batch;

/* Device bytes for a batch of `count` cavities with parameters p[0..count). */
hosc_status hosc_batch_workspace_bytes(const hosc_params *p, int32_t count, size_t *bytes);

/* Create a batch on the current device in d_ws (>= hosc_batch_workspace_bytes,
 * 256-byte aligned, owned by the caller, untouched until hosc_batch_destroy).
 * All p[i].precision must be equal (HOSC_E_ARG otherwise).  Allocates only pinned
 * host staging memory. */
hosc_status hosc_batch_create(const hosc_params *p, int32_t count, void *d_ws, size_t ws_bytes, hipStream_t stream,
                              hosc_batch **out);

/* Release the batch and its cavity handles (not the workspace).  Accepts NULL. */
hosc_status hosc_batch_destroy(hosc_batch *b);

/* Borrow the solver of cavity idx (owned by the batch, valid until
 * hosc_batch_destroy) for the single-cavity calls: hosc_init_fields,
 * hosc_set_state, hosc_get_state, hosc_diagnostics, hosc_entropy_fields. */
hosc_status hosc_batch_cavity(hosc_batch *b, int32_t idx, hosc_solver **out);

/* hosc_init_fields on every cavity, cavity i with seeds[i]. */
hosc_status hosc_batch_init_fields(hosc_batch *b, const uint64_t *seeds, double noise_amp);

/* Advance every cavity nsteps steps.  info (may be NULL): count entries, the last
 * step of each cavity.  A cavity that fails is reported by status and message
 * ("cavity i: ..."); the step of the other cavities completes. */
hosc_status hosc_batch_step(hosc_batch *b, int32_t nsteps, hosc_step_info *info);

/* Step the cavities until each reaches max_f res[f] < res_tol or has taken
 * max_steps steps in this call (the batched form of hosc_run_to_steady).  Every
 * fused step advances only the cavities still marching, so each cavity takes the
 * steps, and reaches the state, of its own hosc_run_to_steady.  info (may be NULL):
 * count entries, the last step each cavity took.  A cavity whose step fails stops
 * (its status in its info entry) while the others go on; the call then returns the
 * first failure, with "cavity i: ..." as the message.  HOSC_E_ARG for res_tol <= 0
 * or max_steps < 0; HOSC_E_STATE if a cavity has no state or is in an error state. */
hosc_status hosc_batch_run_to_steady(hosc_batch *b, double res_tol, int64_t max_steps, hosc_step_info *info);

/* Autotuner: time the fused half-sweep at each candidate schedule (persistent
 * workgroup counts 256 ... 4096, or one workgroup per tile) on this batch and keep
 * the fastest (returned in *grid, 0 = one per tile).  Needs every cavity on a
 * freshly set state (step counter 0); leaves the states unchanged. */
hosc_status hosc_batch_tune(hosc_batch *b, int32_t *grid);

/* Set the schedule by hand (persistent workgroups, 0 = one per tile). */
hosc_status hosc_batch_set_grid(hosc_batch *b, int32_t grid);

/* Timing of the fused solver launches: sweep_* and refine_* counters, one event
 * pair around each batch of fused launches (the other counters stay 0; the phases
 * around the solves keep running as captured graphs). */
hosc_status hosc_batch_perf_enable(hosc_batch *b, int32_t on);
hosc_status hosc_batch_perf_get(hosc_batch *b, hosc_perf *out);

/* Launches of captured graphs so far.  On a stream other than the null stream,
 * the per-cavity phases around the solves (viscosity, sources, assembly and their
 * reductions before; update, walls, divergence, pressure correction and the
 * gather of the step report after) are captured once per level parity and
 * replayed as one graph launch each. */
hosc_status hosc_batch_graph_launches(const hosc_batch *b, int64_t *count);

/* Message of the last failing call on the batch (NULL: last failing create). */
const char *hosc_batch_last_error(const hosc_batch *b);

/* ------------------------------------------------------------------------------
 * Server: cavity solves submitted as they arrive, admitted first-come first-served
 * while their workspace fits an HBM budget (and a resident-count limit), kept
 * resident on the device, and advanced together by fused steps (continuous
 * batching: every hosc_server_step admits what fits, advances each resident cavity
 * one time step, and retires the cavities that reached res_tol or max_steps).  A
 * request's arithmetic is that of its single-cavity run, whatever else is resident.
 * The caller provides the device memory: one workspace holding the arena of the
 * budget and small fused-launch tables.
 * ------------------------------------------------------------------------------ */
typedef struct hosc_server hosc_server;

typedef struct hosc_request {
    hosc_params params;
    uint64_t seed;          /* hosc_init_fields seed and noise amplitude */
    double noise_amp;
    double res_tol;         /* done when max_f res[f] < res_tol ... */
    int64_t max_steps;      /* ... or after max_steps steps */
    double t_arrival;       /* server clock (hosc_server_now), seconds; < 0: now */
} hosc_request;

typedef struct hosc_result {
    uint64_t id;
    int32_t status;         /* HOSC_OK, or the error the request ended with */
    int32_t steady;         /* 1 if res_tol was reached */
    int64_t steps;
    double res;             /* max_f res[f] of the last step */
    double t_arrival, t_admit, t_done;   /* server clock, seconds */
    hosc_diag diag;         /* diagnostics of the final state (zeros on error) */
} hosc_result;

typedef struct hosc_server_stats {
    int64_t queued, resident, completed;
    int64_t server_steps;   /* hosc_server_step calls that advanced cavities */
    int64_t cavity_steps;   /* cavity time steps taken */
    size_t budget, in_use, peak;   /* arena bytes */
    double busy_s;          /* time spent inside hosc_server_step */
} hosc_server_stats;

/* Device bytes of a server workspace: an arena of hbm_budget_bytes (rounded down
 * to 256 bytes) for the resident cavities plus the fused-launch tables of
 * max_resident cavities (1..1024).  HOSC_E_ARG for a budget under 256 bytes. */
hosc_status hosc_server_workspace_bytes(size_t hbm_budget_bytes, int32_t max_resident, size_t *bytes);

/* Create a server on the current device in the caller's workspace d_ws (device,
 * 256-byte aligned, >= hosc_server_workspace_bytes(hbm_budget_bytes, max_resident),
 * owned by the caller and untouched until hosc_server_destroy): cavities are
 * admitted while their workspaces fit the arena of hbm_budget_bytes.  Allocates
 * only pinned host staging memory and its side streams. */
hosc_status hosc_server_create(void *d_ws, size_t ws_bytes, size_t hbm_budget_bytes, int32_t max_resident,
                               hipStream_t stream, hosc_server **out);

/* Finish nothing further and release every resident cavity (not the workspace);
 * waits only for the server's own streams. */
hosc_status hosc_server_destroy(hosc_server *srv);

/* Seconds since the server was created (steady clock). */
hosc_status hosc_server_now(const hosc_server *srv, double *t);

/* Queue a request (copied).  HOSC_E_ARG for invalid parameters; HOSC_E_BUDGET if
 * its workspace exceeds the whole budget. */
hosc_status hosc_server_submit(hosc_server *srv, const hosc_request *rq, uint64_t *id);

/* Admit, advance every resident cavity one step, retire finished ones.  *resident
 * (may be NULL): cavities resident after the call.  A failing request is retired
 * with its status; the return value reports failures of the server itself. */
hosc_status hosc_server_step(hosc_server *srv, int32_t *resident);

/* Move up to max completed results (completion order) into out. */
hosc_status hosc_server_poll(hosc_server *srv, hosc_result *out, int32_t max, int32_t *n_out);

hosc_status hosc_server_stats_get(const hosc_server *srv, hosc_server_stats *st);

/* Message of the last failing call on the server (NULL: last failing create). */
const char *hosc_server_last_error(const hosc_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HOSC_H */
