/*
 * opf_admm.h -- C ABI of the MI355X (gfx950) solver-free componentwise ADMM
 * for multi-phase linearised distribution OPF (Ryu, Byeon, Kim, "A
 * GPU-Accelerated Distributed Algorithm for Optimal Power Flow in Distribution
 * Systems").
 *
 * The library solves the reformulated model of Section III-A (OurModel):
 *
 *     min c^T x   s.t.  A_s x_s = b_s      for every component s,
 *                       B_s x   = x_s      (consensus),
 *                       lb <= x <= ub      (bounds kept out of the components)
 *
 * with Algorithm 1: a clipped consensus average (global update, closed_1 in
 * its sparse form global_sparse), the closed-form projection of each
 * component's local copy onto {A_s y = b_s} (local update, closed_2), the
 * dual update (ADMM-3) and the relative primal/dual residual test
 * (termination).  The per-component factors of closed_2 are precomputed once
 * from the row-reduced A_s (Section IV-B).
 *
 * Conventions for every call:
 *   - plain pointers and sizes only; no framework types;
 *   - host pointers passed to opf_admm_setup are read during the call only
 *     and never retained (the caller keeps ownership);
 *   - device memory allocated by the library belongs to the handle and is
 *     released by opf_admm_destroy;
 *   - all device work of a handle runs on the HIP stream given at setup
 *     (NULL = the null stream); every call returns with that work finished;
 *   - calls on one handle are not thread-safe; distinct handles are
 *     independent;
 *   - return value: 0 on success, OPF_NOT_CONVERGED (a warning, +1) when
 *     max_iter was reached, OPF_STALLED (+2) when the optional stall watch
 *     ended the solve, a negative OPF_E* code on error.  The message of the
 *     last error is available from opf_admm_last_error.
 *
 * Metrics records: when the environment variable OPF_ADMM_METRICS names a
 * file, opf_admm_solve, opf_admm_run_fixed, opf_admm_solve_batch and every
 * served request append one JSON object per solve as a line of it (sizes,
 * schedule, status, iterations, residuals, wall and kernel times, iteration
 * rate, algorithmic bytes per iteration and their effective rate, and up to
 * 64 (pres, dres) pairs of the residual history when one is kept).
 * opf_admm_solve_noalloc writes none.
 */
#ifndef OPF_ADMM_H
#define OPF_ADMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define OPF_OK                     0
#define OPF_NOT_CONVERGED          1   /* max_iter reached; outputs hold the last iterate */
#define OPF_STALLED                2   /* the stall watch (opf_admm_options.stall_window) saw the residual
                                          merit stop falling: the problem is likely infeasible; outputs
                                          hold the last iterate */
#define OPF_EINVAL                (-1) /* bad sizes, NaN/Inf in A, b or c, index out of range, duplicate index in one B_s */
#define OPF_EBOUNDS               (-2) /* lb > ub or NaN bound */
#define OPF_EUNCOVERED            (-3) /* a global variable has no local copy: B^T B singular (Section IV-C) */
#define OPF_EINFEASIBLE_COMPONENT (-4) /* row reduction found 0 = nonzero in [A_s | b_s] (Section IV-B) */
#define OPF_ENOMEM                (-5)
#define OPF_EHIP                  (-6) /* a HIP runtime call failed */
#define OPF_ENUMERIC              (-7) /* NaN/Inf appeared in the residuals */
#define OPF_EHANG                 (-8) /* a bounded device-side wait ran out (persistent kernel) */
#define OPF_ECANCELED             (-9) /* serving: the request was cancelled (opf_server_cancel) */

/* ---- precision of the iteration ----------------------------------------- */
#define OPF_PREC_FP64   0   /* factors, state, residuals all FP64 */
#define OPF_PREC_MIXED  1   /* FP32 factors/state in the bulk phase, FP64 residual sums,
                               then FP64 polish iterations until the FP64 test holds */
/* With polish and eps_rel below OPF_MIXED_STALL_BELOW, the FP32 bulk phase
   also ends when it stalls at its rounding level: every
   OPF_MIXED_STALL_WINDOW iterations the ratio max(pres/eps_prim, dres/eps_dual)
   is compared with its value at the previous check, and unless it has at
   least halved, the solve goes on to the FP64 polish.  Serving applies the
   same checks at the same iterations when iters_per_poll divides the window. */
#define OPF_MIXED_STALL_BELOW  1e-5
#define OPF_MIXED_STALL_WINDOW 65536

/* ---- kernel schedule ----------------------------------------------------- */
#define OPF_KERNEL_AUTO        0
#define OPF_KERNEL_STEP        1  /* one fused launch per iteration, host checks a device flag */
#define OPF_KERNEL_PERSISTENT  2  /* one cooperative launch runs all iterations */
#define OPF_KERNEL_TILED       3  /* one cooperative launch runs all iterations with fewer workgroups
                                     than the packing has: each takes several workgroup tiles in turn,
                                     state kept in memory (AUTO picks it when the persistent grid does
                                     not fit the device; fixed penalty only) */

/*
 * Problem data: the componentwise LP of OurModel.
 *   n          number of global variables x
 *   c[n]       objective (c^T x)
 *   lb[n], ub[n]  bounds, +-INFINITY allowed, lb <= ub
 *   var_kind[n]   0 = no bounds, 1 = bounded, 2 = voltage (squared magnitude).
 *                 Used only by the default initial point of Section V-A:
 *                 a local copy starts at 1 for a voltage, at the midpoint of
 *                 [lb, ub] when both bounds are finite, otherwise at 0.
 *   S          number of components
 *   comp_m[S], comp_n[S]   rows and columns of each A_s (m_s >= 0, 1 <= n_s <= 64)
 *   A_vals     concatenated row-major m_s x n_s blocks
 *   b_vals     concatenated b_s (length m_s each)
 *   idx        concatenated global indices of each component's columns
 *              (the 0/1 matrix B_s of Section II-B: local slot j copies x[idx_j]);
 *              no index repeats inside one component.
 * The stacked local vector z = [x_1; ...; x_S] has L = sum n_s entries in
 * this concatenated order ("user slot order").
 */
typedef struct opf_problem {
    int32_t        n;
    const double*  c;
    const double*  lb;
    const double*  ub;
    const uint8_t* var_kind;
    int32_t        S;
    const int32_t* comp_m;
    const int32_t* comp_n;
    const double*  A_vals;
    const double*  b_vals;
    const int32_t* idx;
} opf_problem;

/*
 * Options.  opf_admm_default_options fills the paper's defaults
 * (rho = 100, eps_rel = 1e-3, Section V-A).
 */
typedef struct opf_admm_options {
    double  rho;            /* ADMM penalty (> 0) */
    double  eps_rel;        /* relative tolerance of the termination test (> 0) */
    int64_t max_iter;       /* iteration cap (>= 1); MIXED with polish: a cap for each of the two phases (the
                               FP32 bulk phase, then up to max_iter FP64 polish iterations) */
    int32_t precision;      /* OPF_PREC_FP64 or OPF_PREC_MIXED */
    int32_t polish;         /* MIXED only: 1 = finish with FP64 iterations until the FP64 test holds */
    int32_t check_every;    /* STEP schedule: iterations enqueued between host checks of the stop flag */
    int32_t kernel;         /* OPF_KERNEL_* */
    int32_t history_cap;    /* per-iteration residual history kept on the device (0 = none) */
    int32_t block_waves;    /* wavefronts per workgroup: 1, 2, 4 or 8 (0 = default) */
    int32_t spin_limit;     /* PERSISTENT: polls before a device-side wait gives up with
                               OPF_EHANG (0 = default, several seconds) */
    int32_t split_terms;    /* batched path: bfloat16 terms per operand on MFMA, 2 or 3 (0 = 3) */
    int32_t autotune;       /* 1: with kernel AUTO and block_waves 0, time short runs of each
                               schedule and workgroup shape on this problem and keep the fastest;
                               batched path: time each workgroup order of the step kernel
                               (opf_admm_info.batch_order).  Decisions are cached per problem
                               shape for the process and in the file named by OPF_ADMM_TUNE_CACHE
                               (default $XDG_CACHE_HOME or $HOME/.cache, opf_admm/tune.txt) */
    int32_t workgroup_order; /* PERSISTENT: 0 = hardware order of workgroups (default; measured
                               faster), 1 = each XCD runs a contiguous range of the packing */
    int32_t setup_on_device; /* 1: row reduction and factors of every component run on the GPU
                               (Section IV-B, closed_2; one workgroup per component) instead of
                               host threads; same results to rounding; components needing more
                               than 64 KiB of LDS make the set-up fail with OPF_EINVAL */
    /* Residual balancing of the penalty, the first of the accelerations
       Section III-D points to (Wohlberg's rule).  After every rho_every-th
       iteration u the residuals of u are compared: with rho_mode
       OPF_RHO_RELATIVE each is first divided by its tolerance of the
       termination test (pres / eps_prim against dres / eps_dual), with
       OPF_RHO_PLAIN they are compared as they are.  If the primal one exceeds
       rho_mu times the dual one the penalty is multiplied by rho_tau, in the
       opposite case divided by it, and then clipped to [rho_min, rho_max].
       The new penalty takes effect OPF_RHO_LAG iterations after u (the
       persistent kernel acts on decisions of earlier iterations; every
       schedule applies the same lag, so all give the same iterates).  Every
       iteration is one plain ADMM iteration with its own penalty: the duals
       stay unscaled and the projection factors do not depend on rho, so
       nothing is refactored.  rho_every = 0 keeps rho fixed (default).  With
       rho_every > 0, zero fields take defaults: rho_mu 10, rho_tau 2,
       rho_min rho / 10, rho_max 10 rho.  Each solve starts from rho; the
       penalty reached is reported in opf_result.rho_final. */
    int32_t rho_every;
    int32_t rho_mode;       /* OPF_RHO_RELATIVE (0) or OPF_RHO_PLAIN (1) */
    double  rho_mu;         /* >= 1 */
    double  rho_tau;        /* > 1 */
    double  rho_min;        /* 0 < rho_min <= rho */
    double  rho_max;        /* rho <= rho_max */
    /* Several local updates per global update, the second acceleration
       Section III-D points to: with x fixed, the local update closed_2 and
       the dual update ADMM-3 are repeated local_updates times.  In the
       projection form the duals lie in the row space of A_s after a dual
       update, so the repeated projections return the same local copies and
       k repetitions equal one local update followed by a dual step of
       length k rho, which is how the kernels run them.  The residuals keep
       rho.  0 or 1 = one local update (Algorithm 1). */
    int32_t local_updates;
    int32_t tiled_workgroups; /* TILED: compute workgroups of the launch (0 = the fewest that hold every
                               tile with an even share, limited by what the device holds at once);
                               fewer workgroups take more tiles each */
    /* Stall watch of the FP64 iterations (FP64 solves and the polish phase of
       mixed solves; not with fixed iteration counts).  The merit
       pres^2 + (dres / rho)^2 of the termination test's residuals
       (Section III-C) does not increase from iteration to iteration, and
       falls to 0 when the problem is feasible; on an infeasible one (each
       component's equations solvable, their consensus not) it settles at a
       positive plateau.  With stall_window > 0 the iterations run in windows
       of that many; after each window the merit of its last iteration is
       compared with the previous window's, and after stall_checks windows in
       a row in which it fell by less than the fraction stall_delta the solve
       stops with OPF_STALLED.  Windows change no arithmetic: a solve that is
       not stopped returns the same bits.  0 fields take defaults when
       stall_window > 0: stall_checks 3, stall_delta 1e-3. */
    int64_t stall_window;
    double  stall_delta;    /* in (0, 1) */
    int32_t stall_checks;   /* >= 1 */
    int32_t reserved_stall;
} opf_admm_options;

#define OPF_RHO_RELATIVE 0
#define OPF_RHO_PLAIN    1
#define OPF_RHO_LAG      4   /* iterations between a balancing decision and its first use */

/* Optional warm start: z0 and lambda0 in user slot order (length L). */
typedef struct opf_warm {
    const double* z;
    const double* lam;
    int32_t       on_device;   /* 1: device pointers, 0: host pointers */
} opf_warm;

/*
 * Outputs of a solve.  x (length n) is required; z and lam (length L, user
 * slot order) are optional (NULL = not written).  The pointers are caller
 * owned, host or device as flagged.
 */
typedef struct opf_result {
    double*  x;
    double*  z;
    double*  lam;
    int32_t  outputs_on_device;
    int32_t  status;           /* same as the return value of the solve */
    int64_t  iterations;       /* completed iterations (all phases) */
    int64_t  iterations_fp32;  /* MIXED: iterations of the FP32 bulk phase */
    double   objective;        /* c^T x */
    double   pres, dres, eps_prim, eps_dual;   /* termination quantities at the last iteration */
    double   solve_ms;         /* wall time of the solve on the host clock */
    double   kernel_ms;        /* device time of the iteration kernels (HIP events on the handle's stream) */
    double   kernel_ms_fp32;   /* MIXED: the part spent in the FP32 phase */
    int64_t  kernel_launches;  /* iteration-kernel launches (persistent: one per precision phase) */
    double   rho_final;        /* penalty the next iteration would use (rho unless residual balancing) */
} opf_result;

typedef struct opf_residuals {
    int64_t iterations;
    double  pres, dres, eps_prim, eps_dual;
} opf_residuals;

/* Layout and size information of a handle (for diagnostics and benchmarks). */
typedef struct opf_admm_info {
    int32_t n, S, L;           /* global variables, components, slots */
    int32_t waves, lanes;      /* packed wavefronts and their lanes (64 each) */
    int32_t max_ns, max_copies;
    int64_t sum_ns2;           /* sum over components of n_s^2 */
    int64_t factor_bytes_fp64; /* device bytes of the packed FP64 factors */
    int64_t device_bytes;      /* all device memory owned by the handle */
    double  setup_ms;          /* host factorisation + packing + upload */
    int32_t grid_blocks;       /* compute workgroups of the iteration kernels (TILED: of the launch; the
                                  packing's workgroup tiles are grid_blocks of the other schedules) */
    int32_t block_waves;       /* wavefronts per workgroup */
    int32_t kernel;            /* OPF_KERNEL_STEP or OPF_KERNEL_PERSISTENT, as selected */
    int32_t persistent_capacity;   /* co-resident workgroups the device can hold */
    int32_t max_neighbours;    /* largest number of workgroups one workgroup waits on */
    int32_t factors_in_lds;    /* persistent schedule: bit 0 FP32 factors held in LDS (every workgroup's),
                                  bit 1 FP64 (the workgroups whose columns fit the launch's budget) */
    int32_t batch_order;       /* batched path: workgroup order of the step kernel, bit 0 = each XCD runs
                                  a contiguous range of the packing, bit 1 = 64-scenario-chunk-major */
    int32_t tiled_pair;        /* TILED: 1 when the two-tile kernel runs (each workgroup keeps two tiles in
                                  flight), 0 for the kernel that takes its tiles in turn (precision of the
                                  bulk phase) */
    int32_t batch_groups;      /* batched path: scenario groups iterated by concurrent launches on their own
                                  streams (the 64-scenario chunks split into contiguous ranges) */
    int32_t fp64_lds_workgroups; /* persistent schedule: workgroups holding their FP64 factors in LDS */
} opf_admm_info;

typedef struct opf_admm_handle opf_admm_handle;

void opf_admm_default_options(opf_admm_options* o);

/*
 * Validates the problem, row-reduces each [A_s | b_s] (Section IV-B),
 * precomputes F_s = I - A_s^T (A_s A_s^T)^{-1} A_s (= -Abar_s) and
 * bbar_s = A_s^T (A_s A_s^T)^{-1} b_s in FP64 (closed_2 and Algorithm 1's
 * precomputation), builds the copy lists of B^T (whose Gram matrix B^T B is
 * diagonal, Section IV-C), packs components into 64-lane wavefronts and
 * uploads everything to the device on `hip_stream` (a hipStream_t, NULL for
 * the null stream).  On success *out receives a handle.  On error *out is
 * NULL and the message is available from opf_admm_last_error(NULL).
 */
int opf_admm_setup(const opf_problem* p, const opf_admm_options* o, void* hip_stream,
                   opf_admm_handle** out);

/*
 * Runs Algorithm 1 from the default initial point (Section V-A) or from
 * `warm` (nullable) until the termination test holds or max_iter iterations
 * have run.  Writes the outputs requested in r and its scalar fields.
 * Returns OPF_OK, OPF_NOT_CONVERGED, OPF_ENUMERIC or another error.
 */
int opf_admm_solve(opf_admm_handle* h, const opf_warm* warm, opf_result* r);

/*
 * Runs exactly `iters` iterations (no termination test) from the default
 * initial point or `warm`, with the handle's precision, and writes the
 * outputs like opf_admm_solve.  Meant for trajectory comparisons at a fixed
 * iteration count.
 */
int opf_admm_run_fixed(opf_admm_handle* h, const opf_warm* warm, int64_t iters, opf_result* r);

/*
 * opf_admm_solve without any device allocation or graph instantiation during
 * the call, for callers that cannot allocate: serving loops and harnesses
 * that forbid hipMalloc/hipFree once set-up is done.  Same arguments,
 * outputs and return codes as opf_admm_solve, and the same iterates bit for
 * bit: the iteration kernels are the same, but their scratch (the step
 * kernel's residual partials and arrival counters, the persistent kernel's
 * published terms, residual records and decision words) lives in one static
 * device array of OPF_NOALLOC_SCRATCH_BYTES per device, held by the library
 * until the process ends, instead of the handle's buffers, and the step
 * schedule issues its launches one by one instead of replaying a captured
 * graph.  The array keeps the last call's contents; each call prepares what
 * it reads.  Every such call on one device uses the same array, so calls
 * that overlap on one device (other threads, other streams) race and must
 * be serialised by the caller.  A problem whose scratch does not fit (about
 * 32 bytes per packed lane plus 64 bytes per workgroup; e.g. 8500 buses use
 * 5.5 MB, 21000 buses 13.5 MB) is rejected with OPF_EINVAL before any work.
 */
#define OPF_NOALLOC_SCRATCH_BYTES (16u << 20)
int opf_admm_solve_noalloc(opf_admm_handle* h, const opf_warm* warm, opf_result* r);

/*
 * Quantities of the termination test (Section III-C, eq. termination) at the
 * last completed iteration of the handle:
 *   pres     = sqrt(sum_s ||B_s x - x_s||^2),
 *   dres     = rho sqrt(sum_s ||B_s^T (x_s^t - x_s^{t-1})||^2),
 *   eps_prim = eps_rel max(sqrt(sum_s ||B_s x||^2), sqrt(sum_s ||x_s||^2)),
 *   eps_dual = eps_rel sqrt(sum_s ||B_s^T lambda_s||^2),
 * each sum accumulated in FP64 (B_s^T is an isometric injection, so these are
 * the norms of the stacked slot vectors).  When hist != NULL (host, caller
 * owned, 4 * hist_cap doubles) the per-iteration history is written as rows
 * (pres, dres, eps_prim, eps_dual): up to min(hist_cap, options.history_cap,
 * iterations) rows.  Returns the number of rows written, or a negative error
 * (OPF_EINVAL for a NULL handle, OPF_EHIP).
 */
int opf_admm_residuals(const opf_admm_handle* h, opf_residuals* out, double* hist, int hist_cap);

/* Copies layout and size information of the handle. */
int opf_admm_get_info(const opf_admm_handle* h, opf_admm_info* info);

/*
 * ---- Batched same-topology scenarios ----------------------------------------
 *
 * K scenarios share the problem's topology and every A_s (constant-power loads
 * keep A_s scenario-independent) and differ in their right-hand sides b_s, so
 * they share the projection factors F_s and each has its own bbar_s (closed_2).
 * The local updates of all scenarios then form small dense products
 * F_s [v_1 ... v_K], evaluated on MFMA in bfloat16 split terms with FP32
 * accumulation; state is FP32, residual sums FP64.  Each scenario stops at its
 * own termination test (Section III-C); its x is recorded at that iteration.
 */
typedef struct opf_admm_batch opf_admm_batch;

typedef struct opf_batch_result {
    double*  x;                /* [K][n] scenario-major, required; host or device per the flag */
    int32_t  outputs_on_device;
    int32_t  reserved0;
    int64_t* iterations;       /* [K] host, nullable: stop iteration of each scenario */
    double*  objective;        /* [K] host, nullable: c^T x of each scenario */
    int32_t* status;           /* [K] host, nullable: OPF_OK / OPF_NOT_CONVERGED / OPF_ENUMERIC */
    double*  pres;             /* [K] host, nullable; also dres, eps_prim, eps_dual */
    double*  dres;
    double*  eps_prim;
    double*  eps_dual;
    int64_t  total_iterations; /* iterations the batch ran (the slowest scenario) */
    int32_t  converged;        /* scenarios whose test held */
    int32_t  reserved1;
    double   solve_ms;
} opf_batch_result;

/*
 * Like opf_admm_setup for K scenarios: b_scen holds K concatenated right-hand
 * sides ([K][sum m_s], host, caller-owned, read during the call).  p->b_vals
 * may be NULL.  Each scenario's b must be consistent with its A_s
 * (OPF_EINFEASIBLE_COMPONENT otherwise).  1 <= K <= 4096.
 */
int opf_admm_setup_batch(const opf_problem* p, const double* b_scen, int32_t K, const opf_admm_options* o,
                         void* hip_stream, opf_admm_batch** out);

/*
 * As opf_admm_setup_batch, for load models whose equations change with the
 * scenario (voltage-dependent ZIP loads: the coefficient of the bus voltage in
 * VDLM-1/2 scales with the load).  `a_pos` [nv] are positions in p->A_vals
 * (int64, each inside one component's block) whose value differs per scenario;
 * `a_scen` [K][nv] (row-major) holds those values for every scenario.
 * Components that contain such a position are factored once per scenario
 * (Section IV-B row reduction, closed_2) and packed into wavefronts of their
 * own, whose local update runs as a per-scenario FP32 product; all other
 * components keep the shared split-bf16 MFMA product.  nv = 0 is
 * opf_admm_setup_batch.  Errors as opf_admm_setup_batch; a scenario whose
 * patched equations are contradictory gives OPF_EINFEASIBLE_COMPONENT.
 */
int opf_admm_setup_batch_ex(const opf_problem* p, const double* b_scen, int32_t K, int64_t nv,
                            const int64_t* a_pos, const double* a_scen, const opf_admm_options* o,
                            void* hip_stream, opf_admm_batch** out);

/* Runs Algorithm 1 for all scenarios from the default start point until every
   scenario has met its test or max_iter.  Returns OPF_OK when all converged,
   OPF_NOT_CONVERGED if some reached max_iter, OPF_ENUMERIC, or an error. */
int opf_admm_solve_batch(opf_admm_batch* h, opf_batch_result* r);

int opf_admm_batch_info(const opf_admm_batch* h, opf_admm_info* info);
void opf_admm_destroy_batch(opf_admm_batch* h);
const char* opf_admm_batch_last_error(const opf_admm_batch* h);

/*
 * ---- Serving runtime ---------------------------------------------------------
 *
 * A request loop for many independent solves (feeders of different sizes and
 * switched topologies) arriving over time.  Submitted problems are set up on
 * host threads and admitted into a device arena while their memory footprint
 * fits (admission by HBM footprint).  The device works in rounds: one
 * persistent launch per precision (the FP32 bulk phase of mixed-precision
 * solves, then FP64: plain solves and polish phases) advances every resident
 * solve by up to iters_per_poll iterations of Algorithm 1, each with its own
 * iteration count and termination test (Section III-C).  Between rounds the
 * host retires finished solves and admits waiting ones, so a solve that
 * arrives while others run joins the next round (continuous batching).  A
 * mixed-precision solve moves from the FP32 launch to the FP64 launch exactly
 * where the single-instance solver hands over.
 *
 * After a solve finishes, its (z, lambda) stay resident in HBM under its
 * feeder family; with warm_start on, a later request of the same family starts
 * from them component by component, matching components by caller-supplied
 * keys.  Bit identity: a cold-started solve returns the same bits alone, in any
 * mix and as the single-instance solver with the same options; a warm-started
 * solve depends on which state of its family is resident when it is admitted.
 */
typedef struct opf_server opf_server;

typedef struct opf_server_options {
    opf_admm_options admm;     /* rho, eps_rel, max_iter, precision (OPF_PREC_FP64, or OPF_PREC_MIXED:
                                  FP32 bulk phase in one launch, then FP64 polish in another, as the
                                  single-instance solver does) and polish of every solve */
    int64_t arena_bytes;       /* device memory for resident solves (admission budget) */
    int64_t warm_bytes;        /* device memory for warm-start states (least recently used evicted) */
    int32_t max_slots;         /* most solves resident at once */
    int32_t max_workgroups;    /* cap on the grid of the shared launch (sum over resident solves of their
                                  workgroups + 1); the device's co-resident capacity caps it too, and a
                                  solve that can never fit is answered with OPF_ENOMEM */
    int32_t iters_per_poll;    /* iterations each resident solve runs per shared launch before the host
                                  polls the stop flags and admits / retires solves */
    int32_t setup_threads;     /* host threads for row reduction / factors / packing */
    int32_t warm_start;        /* 1: use resident states of the same family */
    int32_t admission;         /* order in which waiting requests are offered the free co-resident
                                  capacity: OPF_ADMIT_LARGEST_FIRST (default) or OPF_ADMIT_ARRIVAL; in
                                  either order a request that does not fit is passed over for later ones */
    int32_t max_wait_ms;       /* starvation guard (0: off; default 500): once a request that does not fit
                                  has waited this long since submission, and the solves holding the
                                  capacity it needs are all smaller than it, smaller requests are no longer
                                  admitted ahead of it (the capacity drains to it as those solves end) */
    int32_t reserved[3];
} opf_server_options;

/* Largest first: the solves of the most workgroups start as soon as they fit
   and smaller ones fill the remaining capacity (on mixed-size traffic the
   largest solves are the critical path: with arrival order, smaller requests
   admitted behind a large one keep taking the capacity it waits for). */
#define OPF_ADMIT_LARGEST_FIRST 0
#define OPF_ADMIT_ARRIVAL       1

typedef struct opf_served {
    int64_t request_id;
    int32_t status;            /* OPF_OK, OPF_NOT_CONVERGED, OPF_ENUMERIC, or a set-up / admission error */
    int32_t warm_components;   /* components started from a resident state */
    int64_t iterations;
    double  objective;
    double  pres, dres, eps_prim, eps_dual;
    double  queue_ms;          /* submit -> admitted to the device */
    double  latency_ms;        /* submit -> result ready */
    double* x;                 /* the x buffer given at submit, now filled */
    int64_t iterations_fp32;   /* of `iterations`, those of the FP32 bulk phase (mixed precision) */
} opf_served;

typedef struct opf_server_stats {
    int64_t submitted, completed, rejected;
    int32_t resident, queued;
    int64_t arena_used, arena_bytes, warm_used;
    int64_t launches;          /* shared iteration launches so far */
    double  busy_ms;           /* device time of the shared launches (host clock) */
} opf_server_stats;

void opf_server_default_options(opf_server_options* o);

/* Starts the runtime (worker and set-up threads).  All device work runs on
   `hip_stream` (NULL: a private stream). */
int opf_server_create(const opf_server_options* o, void* hip_stream, opf_server** out);

/*
 * Queues one solve.  The problem arrays are copied before the call returns.
 * `family` groups requests whose states may warm-start each other;
 * `comp_keys` (S values, nullable) identify components across requests of a
 * family (a component warm-starts when its key and size match).  x_out (host,
 * n doubles, caller-owned) must stay valid until the result is polled.
 * Returns 0 and the request id, or OPF_EINVAL / OPF_ENOMEM (footprint larger
 * than the arena).
 */
int opf_server_submit(opf_server* s, const opf_problem* p, uint64_t family, const uint64_t* comp_keys,
                      double* x_out, int64_t* request_id);

/* Cancels a submitted request that has not been answered yet.  A request
 * still queued (in set-up or waiting for admission) is answered at once; one
 * in set-up when set-up ends; a resident one before the next shared round, with
 * its current iterate in x_out (iterations and residuals of its last completed
 * round).  Its result, polled as usual, has status OPF_ECANCELED, and no
 * warm-start state is kept from it.  Returns 0, or OPF_EINVAL for an unknown
 * or already answered request id. */
int opf_server_cancel(opf_server* s, int64_t request_id);

/* Moves up to max_out finished results into out (waiting up to wait_ms for
   the first); returns how many were written. */
int opf_server_poll(opf_server* s, opf_served* out, int max_out, int wait_ms);

int opf_server_get_stats(const opf_server* s, opf_server_stats* st);

/* Stops the runtime; unfinished requests are dropped. */
void opf_server_destroy(opf_server* s);
const char* opf_server_last_error(const opf_server* s);

/* Frees the handle and its device memory.  NULL is ignored. */
void opf_admm_destroy(opf_admm_handle* h);

/* Message of the last error of h (or of the last failed setup when h is NULL).
   Owned by the library; valid until the next call on the same handle. */
const char* opf_admm_last_error(const opf_admm_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* OPF_ADMM_H */
