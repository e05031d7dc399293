/*
 * irk.h -- C ABI of the MI355X (gfx950) fully implicit Runge-Kutta stage
 * solver.
 *
 * The library advances a method-of-lines system  M u' = N(u, t)  (paper,
 * Section 1.1, equation (problem)) by one step of an s-stage Gauss or
 * Radau IIA method: it solves the nonlinear stage equations (equation
 * (stages); for the index-1 DAE, equation (dae_stage) of Section 6) and
 * applies the update (equation (update)).  Each nonlinear iteration is the
 * Newton-like iteration of Section 3.2 (Algorithm 1 of Section 5) written in
 * the real eigenbasis of A0^{-1}: one preconditioned FGMRES solve per real
 * eigenvalue and per conjugate pair, the pair blocks preconditioned with the
 * block lower-triangular preconditioner of equation (Lprec) with the Schur
 * complement approximation gamma_* of equation (gamma*), whose diagonal
 * inverses are one geometric-multigrid V-cycle each.
 *
 * Conventions for every entry point:
 *   - Nothing throws across the ABI; every call returns an irk_status
 *     (irk_destroy returns nothing and accepts NULL).
 *   - "device" pointers are HIP device addresses on the device that is
 *     current when irk_create is called; "host" pointers are ordinary host
 *     memory.  All device pointers must be 8-byte aligned; the workspace
 *     256-byte aligned.
 *   - The caller owns every buffer it passes; the library owns only the
 *     context: host memory, a small pinned host staging buffer (fine-
 *     grained and mapped: the reduction kernels write the scalars the host
 *     reads there), the streams and events of its eigen-blocks and, with
 *     the option lane_threads, one host thread per eigen-block.
 *   - All device work is ordered with the HIP stream given to irk_create:
 *     the eigen-blocks run on the context's own streams, which wait for
 *     and are joined back into that stream through events.  Calls on one
 *     context must not overlap; distinct contexts may run concurrently on
 *     distinct streams.
 *
 * Field layout: a scalar field is row-major [ny][nx] float64, x fastest
 * (1-D problems have ny = 1).  The vorticity-streamfunction state is
 * [2][ny][nx]: omega then psi.
 *
 * Mapping onto the proposed boundary (irk_create / irk_step / irk_destroy
 * plus a serving interface): the stages are always transformed into the
 * real eigenbasis of A0^{-1} by default (its blocks are independent, so
 * they run concurrently; irk_options.transform selects the paper's real
 * Schur basis, solved by back-substitution between blocks); serving polls with
 * irk_server_progress (one pass for all requests) and reads a request's
 * state with irk_server_info, its result landing in the request's own
 * output buffer, instead of a per-request poll and result call.
 */
#ifndef IRK_H
#define IRK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IRK_MAX_STAGES 5
#define IRK_MAX_RESTART 64

typedef enum irk_status {
    IRK_OK = 0,
    IRK_E_ARG = -1,         /* invalid argument (sizes, pointers, options)   */
    IRK_E_NOMEM = -2,       /* workspace too small / budget exceeded         */
    IRK_E_NOCONV = -3,      /* Newton-like iteration did not converge        */
    IRK_E_NONFINITE = -4,   /* NaN or Inf in the input or in a residual      */
    IRK_E_DEVICE = -5,      /* a HIP runtime call failed                     */
    IRK_E_UNSUPPORTED = -6, /* option combination not implemented            */
    IRK_E_BUSY = -7         /* serving: request not finished yet             */
} irk_status;

typedef enum irk_family {
    IRK_GAUSS = 0,          /* s-stage Gauss, order 2s                       */
    IRK_RADAU_IIA = 1,      /* s-stage Radau IIA, order 2s-1                 */
    IRK_LOBATTO_IIIC = 2,   /* s-stage Lobatto IIIC, order 2s-2, s >= 2      */
    IRK_SDIRK = 3           /* published L-stable SDIRK methods (comparison
                               class): s = 1 backward Euler, 2 Alexander
                               order 2, 3 Alexander order 3, 5 Hairer-Wanner
                               order 4; the stages are solved one after
                               another, each as a single real block with the
                               same preconditioner (eta = 1/gamma)          */
} irk_family;

typedef enum irk_op_kind {
    /* u_t + (u^2/2)_x = nu u_xx: N_i = -(u_{i+1}^2-u_{i-1}^2)/(4h)
       + nu (u_{i+1}-2u_i+u_{i-1})/h^2, periodic, M = I                       */
    IRK_OP_BURGERS_1D = 0,
    /* u_t = div((1+u^2) grad u) + f: 5-point flux form with face
       coefficient (kappa(u_c)+kappa(u_nb))/2, periodic, M = I               */
    IRK_OP_NLDIFF_2D = 1,
    /* omega_t = J_A(psi, omega) + nu Lap omega (Arakawa Jacobian),
       0 = Lap psi + omega - mean(omega) - mean(psi) (index-1 constraint
       with the gauge mean(psi) = 0), periodic, M = diag(I, 0)               */
    IRK_OP_VSF_2D = 2
} irk_op_kind;

typedef enum irk_forcing {
    IRK_FORCING_NONE = 0,
    /* f = u*_t - div((1+u*^2) grad u*), u* = sin(2 pi x) sin(2 pi y) cos t  */
    IRK_FORCING_MMS = 1,
    /* f = u*_t - N_h(u*): u* solves the semi-discrete system exactly        */
    IRK_FORCING_MMS_DISCRETE = 2
} irk_forcing;

/* Spatial operator on the periodic domain [0, length)^d, nodes x_i = i h,
 * h = length / nx (nx = ny required in 2-D).                               */
typedef struct irk_operator {
    int kind;               /* irk_op_kind                                    */
    int nx, ny;             /* grid; 1-D: ny = 1                              */
    double length;          /* domain side                                    */
    double nu;              /* viscosity (Burgers, VSF); unused for NLDIFF    */
    int forcing;            /* irk_forcing (NLDIFF only)                      */
} irk_operator;

typedef struct irk_options {
    double newton_rtol;     /* stop when ||F(K)|| <= rtol ||F(K0)|| + atol    */
    double newton_atol;
    double krylov_rtol;     /* relative FGMRES tolerance per block solve      */
    int restart;            /* FGMRES restart length (1..IRK_MAX_RESTART)     */
    int max_krylov;         /* FGMRES iteration cap per block solve           */
    int max_newton;         /* Newton-like iteration cap                      */
    int newton_like;        /* Section 3.2 in the eigenbasis, d_rq,k =
                               (T^{-1})_rk T_kq:
                               0: simplified Newton (last-stage Jacobian),
                               1: lump each row to its argmax |d_rr,k| stage
                                  (among weights within a relative 1e-12
                                  of the largest, the lowest stage index),
                               2: each row its weighted sum_k d_rr,k L(U_k),
                               3: as 2 plus the coupling sum_k d_rq,k L(U_k)
                                  between the two rows of a pair (the
                                  truncation to the blocks of Lambda; exact
                                  Newton for 2-stage methods).  (2), (3):
                               each row's V-cycle is built at
                               sum_k d_rr,k U_k; (3) is never batched       */
    int gamma_mode;         /* 0: gamma_* = eta + beta^2/eta, 1: gamma = eta  */
    int prec_fp32;          /* 1: V-cycles in float32, 0: float64            */
    int cheb_degree;        /* Chebyshev pre- and post-smoothing degree       */
    int mg_coarsest;        /* coarsening stops before a side below this (the
                               coarsest level, at most 1024 points, is
                               solved by Chebyshev iteration); vorticity
                               V-cycles stop earlier, at the first level
                               whose operator is diagonally dominant
                               (Gershgorin ratio <= 1/4: D Jacobi sweeps
                               there), and streamfunction (Poisson) cycles at
                               the first level of side <= 32 (solved
                               exactly, by fast diagonalization)          */
    int coarse_iters;       /* Chebyshev iterations on the coarsest level     */
    int batch_mg;           /* 1: V-cycles of blocks (and, in a server, of
                               requests) waiting at the same time run in
                               shared launches; 0: one launch sequence per
                               V-cycle on its block's stream                 */
    int start_extrapolate;  /* 1: when a step continues the context's
                               previous one (u_n is that step's output
                               buffer and t_n its end time), the previous
                               stage vectors extrapolated along their
                               interpolating polynomial are a third starting
                               candidate; 0: zero and explicit only         */
    int krylov_adaptive;    /* 1: the block solves of a Newton iteration stop
                               at max(krylov_rtol, 0.1 target / ||F||), at
                               most 0.1, target = the acceptance threshold
                               (never solving further than the outer test
                               can use); 0: krylov_rtol always             */
    int dae_reorder;        /* IRK_OP_VSF_2D only.  0: Krylov on each block's
                               whole system (vorticity and streamfunction
                               rows, eq (vsf-system-1)) preconditioned by
                               L_P then one Poisson V-cycle per
                               streamfunction row; 1: the reordered
                               block-triangular system (eq (vsf-system-2)):
                               forward substitution, a Krylov solve of the
                               vorticity rows (preconditioned by L_P), then
                               one of the streamfunction rows (a Poisson
                               V-cycle per row as preconditioner)          */
    int transform;          /* 0: the real eigenbasis of A0^{-1} (blocks
                               independent, solved concurrently); 1: the
                               real Schur basis (Section 3.1, irk_schur_
                               blocks): the blocks are solved last to first
                               by back-substitution (Section 5, equation
                               (D+U)), each block's right-hand side losing
                               R0_ij M y_j for every solved block j (and,
                               under Newton-like (3), the stage-weighted
                               Jacobian terms -dt sum_k d_rq,k L(U_k) y_j
                               of the truncation to R0's block-upper
                               pattern).  Burgers and nonlinear diffusion
                               only (IRK_E_UNSUPPORTED otherwise)          */
    int psi_solve;          /* IRK_OP_VSF_2D only: how the streamfunction rows'
                               Poisson block -dt Lap_h is applied in the
                               preconditioner.  0: exactly, by a spectral
                               solve on the finest grid (its discrete
                               Fourier modes diagonalize the periodic
                               5-point Laplacian), in the V-cycle precision,
                               when the side is a power of two from 16 up
                               to 2048 (float32) or 1024 (float64), else
                               as 1; 1: one Poisson V-cycle.  In float32
                               the solve is exact only to about the
                               Laplacian's condition number times float32
                               rounding (1e-2 at 1024^2)                  */
    int lane_threads;       /* 1: a context made by irk_create with two or
                               more independent eigen-blocks (eigenbasis,
                               no batch_mg) drives each block's solve from
                               a host thread of its own, so that the
                               blocks' kernel launches are issued in
                               parallel; the threads live as long as the
                               context and sleep between steps.  Off while
                               irk_profile_enable is on.  0: the calling
                               thread drives every block.  The device work
                               and its results are the same either way    */
} irk_options;

/* Per-step counters.  "Preconditioner applications" follow the paper's
 * accounting (Section 7.1): one per Krylov iteration on a 1x1 block, two per
 * Krylov iteration on a 2x2 block.                                          */
typedef struct irk_stats {
    int newton_its;
    int krylov_its;             /* all blocks, all Newton iterations          */
    int krylov_its_block[IRK_MAX_STAGES];
    int vcycles;                /* diagonal-block solves of the preconditioner:
                                   V-cycles, and the spectral Poisson solves
                                   of psi_solve = 0                         */
    int prec_applications;
    double res0;                /* ||F(K0)||_2                                */
    double final_res;           /* ||F(K)||_2 at acceptance                   */
    int start;                  /* starting stage vectors Newton began from:
                                   0 zero, 1 explicit, 2 extrapolated       */
    int acceptance;             /* how the iteration was accepted: 0 the
                                   threshold (rtol ||F(K0)|| + atol, or the
                                   rounding level of the residual evaluation),
                                   1 stagnation within 16x that rounding
                                   level, 2 stagnation (three iterations each
                                   reducing ||F|| by less than 10 %) below
                                   1e-8 ||F(K0)||: the rounding level was
                                   underestimated -- the step is returned
                                   with IRK_OK but final_res may exceed the
                                   threshold.  SDIRK: the largest over the
                                   stages.                                   */
    int krylov_its_psi;         /* reordered DAE system (dae_reorder = 1):
                                   the iterations of the streamfunction
                                   solves, included in krylov_its (one per
                                   block and Newton iteration when the
                                   Poisson block is solved exactly)          */
} irk_stats;

/* ---------------- host-only entry points (no GPU needed) ---------------- */

const char *irk_status_str(irk_status st);

/* Starting stage vectors K0 (Algorithm 1 leaves them open): the candidates
 * K = 0 (every stage value at u_n), the explicit k_i = N(u_n, t_n) on
 * differential rows (0 on algebraic rows) and, with start_extrapolate on a
 * continued step, k_i = sum_j l_j(1 + c_i dt / dt_prev) k_j^prev (l_j the
 * Lagrange basis on the nodes c) are evaluated in that order; Newton starts
 * from the one with the smallest stage residual, the earlier one on ties.
 * Defaults: newton_rtol 1e-12, newton_atol 0 (then 1e-14 ||F(K0)||),
 * krylov_rtol 1e-5 (the paper's GMRES tolerance, Section 7.1), restart 30,
 * max_krylov 200, max_newton 30, newton_like 1, gamma_mode 0, prec_fp32 1,
 * cheb_degree 3, mg_coarsest 16, coarse_iters 24, batch_mg 0 (shared
 * launches couple the blocks' progress and were measured slower on the
 * bench workloads; see the option), start_extrapolate 1, krylov_adaptive 1,
 * dae_reorder 0, transform 0.                                              */
void irk_default_options(irk_options *opt);

/* Butcher tableau of the s-stage method (Section 1.1): A row-major s x s,
 * b and c of length s, written to host arrays.  Nodes are the roots of
 * P_s(2x-1) (Gauss) or P_s(2x-1) - P_{s-1}(2x-1) (Radau IIA), A and b the
 * collocation integrals; computed in long double.  1 <= s <= 5.            */
irk_status irk_tableau(irk_family family, int s, double *A, double *b, double *c);

/* Real eigenbasis of A0^{-1} (Sections 3.1 and 5): A0^{-1} = T Lambda T^{-1},
 * Lambda block diagonal with a 1x1 block eta per real eigenvalue and a 2x2
 * block [[eta, beta], [-beta, eta]] per pair eta +- i beta (beta > 0; this is
 * the form [[eta, phi], [-beta^2/phi, eta]] of Section 3.1 with phi = beta).
 * Blocks are ordered real first, then pairs by decreasing beta.  Host
 * outputs: T, Tinv (s x s row-major), nblocks, and per block its width
 * (1 or 2), eta, beta, gamma_* = eta + beta^2/eta (equation (gamma*)) and the
 * first transformed row it covers.  Arrays sized IRK_MAX_STAGES suffice.
 * IRK_E_ARG for IRK_SDIRK (its stages are solved one after another).     */
irk_status irk_eigen_blocks(irk_family family, int s, double *T, double *Tinv,
                            int *nblocks, int *width, double *eta, double *beta,
                            double *gamma_star, int *first_row);

/* Real Schur basis of A0^{-1} (Section 3.1): A0^{-1} = Q0 R0 Q0^T with Q0
 * orthogonal and R0 block upper triangular, its diagonal blocks those of
 * irk_eigen_blocks in the same order (eta, or [[eta, phi], [-beta^2/phi,
 * eta]] with |phi| <= beta: the standardized form), the blocks above the
 * diagonal coupling them.  Built from the real eigenbasis by Gram-Schmidt
 * (long double); each column's largest entry positive.  Host outputs Q0, R0
 * (s x s row-major).  IRK_E_ARG for IRK_SDIRK or bad s.  The option
 * `transform` = 1 runs the Newton-like iteration in this basis.          */
irk_status irk_schur_blocks(irk_family family, int s, double *Q0, double *R0);

/* Bytes of device workspace irk_create needs for this problem (0 on bad
 * arguments).                                                               */
size_t irk_workspace_bytes(irk_family family, int s, const irk_operator *op,
                           const irk_options *opt);

/* ---------------------------- device entry points ------------------------ */

typedef struct irk_ctx irk_ctx;   /* opaque, library-owned */

/* Build the tableau, its eigenbasis and the solver state for one problem.
 * device_workspace: caller-owned device buffer of at least
 * irk_workspace_bytes(...) bytes, 256-byte aligned, kept alive and unused by
 * the caller until irk_destroy.  hip_stream: a hipStream_t (NULL = default
 * stream).  opt may be NULL (defaults).  On success *out receives the
 * context.  Errors: IRK_E_ARG (bad sizes: s outside 1..5, grid not divisible
 * by 2 down to mg_coarsest, nx != ny in 2-D), IRK_E_NOMEM (workspace too
 * small), IRK_E_DEVICE.                                                     */
irk_status irk_create(irk_family family, int s, const irk_operator *op,
                      const irk_options *opt, void *device_workspace,
                      size_t workspace_bytes, void *hip_stream, irk_ctx **out);

/* One step from (u_n, t_n) with step dt (Algorithm 1): device input u_n,
 * device output u_np1 (may alias u_n), both in the field layout above.
 * tol > 0 overrides options.newton_rtol for this step.  stats (host) may be
 * NULL.  The call returns after the step has completed on the stream.
 * Errors: IRK_E_NONFINITE (NaN/Inf in u_n or a residual), IRK_E_NOCONV
 * (max_newton reached or the residual grows by 1e8), IRK_E_DEVICE.  On any
 * error u_np1 is not written.                                               */
irk_status irk_step(irk_ctx *ctx, const double *u_n, double t_n, double dt,
                    double tol, double *u_np1, irk_stats *stats);

/* Stage residual F_i(K) = M k_i - N(u_n + dt sum_j a_ij k_j, t_n + c_i dt)
 * (equation (stages) / (dae_stage)) for caller stage vectors K (device,
 * [s][field]) into F (device, [s][field]).  Evaluates exactly the residual
 * the Newton loop of irk_step uses.  IRK_E_UNSUPPORTED for IRK_SDIRK.    */
irk_status irk_eval_residual(irk_ctx *ctx, const double *u_n, double t_n,
                             double dt, const double *K, double *F);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * irk_eval_residual without a context or a caller workspace.  F_i =
 * M k_i - N(u_n + dt sum_j a_ij k_j, t_n + c_i dt) for the s-stage method of
 * `family` on operator *op, with the same kernels and the same arithmetic
 * as irk_eval_residual.  u_n (field layout above), K and F ([s][field]) are
 * device pointers on the current device; the work is enqueued on hip_stream
 * (NULL = the null stream) and F is complete when that stream's work is: the
 * call itself neither waits nor allocates (no hipMalloc, hipFree, memset or
 * host-staged copy; its host-side tableau arithmetic uses stack memory only),
 * so it can be captured into a HIP graph.  Its scratch (the stage values,
 * reduction partials, forcing tables) is one fixed device array of
 * IRK_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends and shared
 * by every call on that GPU: calls that overlap on one GPU race.  Errors:
 * IRK_E_NOMEM when s * field * 8 bytes plus about 140 KiB exceed that size
 * (e.g. a 1024^2 vorticity-streamfunction field with s = 4), IRK_E_ARG,
 * IRK_E_UNSUPPORTED for IRK_SDIRK, IRK_E_DEVICE (a launch failed).        */
#define IRK_NOALLOC_SCRATCH_BYTES (64u << 20)
irk_status irk_eval_residual_noalloc(irk_family family, int s, const irk_operator *op, const double *u_n,
                                     double t_n, double dt, const double *K, double *F, void *hip_stream);

/* y = D_b x: the Krylov operator of eigen-block `block` (0 <= block <
 * nblocks of irk_eigen_blocks; equation (diag_blocks) under the context's
 * Newton-like truncation, Section 3.2) at the stage values of the last
 * irk_eval_residual call or successful irk_step.  x, y: device
 * [width][field] (the block's transformed components, one after the
 * other), not aliased.  Errors: IRK_E_ARG (no stage values yet, bad block),
 * IRK_E_UNSUPPORTED for IRK_SDIRK, IRK_E_DEVICE.                           */
irk_status irk_apply_block(irk_ctx *ctx, int block, const double *x, double *y);

/* Copy the stage vectors K of the last successful irk_step (device, [s][field])
 * into the caller's device buffer (for IRK_SDIRK the s stage derivatives). */
irk_status irk_get_stages(irk_ctx *ctx, double *K);

/* ------------------------------ measurement ------------------------------ */

/* Per-kernel timing for roofline measurement (not part of the method).
 * enable != 0 starts (and resets) recording: every kernel launch of later
 * irk_step calls is bracketed by HIP events on the context's stream and
 * attributed its algorithmic bytes (compulsory field traffic of that launch).
 * Results are grouped by kernel symbol (template instance); irk_profile_count
 * gives the number of groups, irk_profile_entry group idx: its name (written
 * to name, at most name_len bytes including the terminator), launches, summed
 * event time in milliseconds and summed algorithmic bytes.  Recording adds
 * event overhead; do not time throughput with it enabled.                  */
irk_status irk_profile_enable(irk_ctx *ctx, int enable);
int irk_profile_count(irk_ctx *ctx);
irk_status irk_profile_entry(irk_ctx *ctx, int idx, char *name, int name_len, long *launches,
                             double *total_ms, double *total_bytes);

/* Back-to-back timing of one kernel group: while recording, the context
 * keeps the most recent launches of every group (at most 32, all on one
 * stream, with their arguments).  This re-issues them reps times in a row on
 * that stream between two HIP events and returns the average duration of one
 * launch in milliseconds (and the average algorithmic bytes of one launch),
 * free of the per-launch event overhead of irk_profile_entry.  The replays
 * overwrite the context's internal buffers: call it only between steps.
 * IRK_E_ARG if nothing of that name was recorded.                          */
irk_status irk_profile_replay(irk_ctx *ctx, const char *name, int reps, double *avg_ms, double *avg_bytes);

/* Release the context (not the caller's workspace).  NULL is accepted.     */
void irk_destroy(irk_ctx *ctx);

/* -------------------------------- serving -------------------------------- */
/* Continuous batching of step-solve requests on one GPU (not in the paper).
 * Requests are admitted first-in first-out as soon as a slot is free and
 * their resident state fits in the caller's device arena: the solver
 * workspace of irk_workspace_bytes plus two state fields.  Admitted requests
 * stay resident until their last step; running requests progress
 * concurrently, each on its own HIP streams.  A request's result is the same
 * as irk_step's on the same problem, whatever else runs.                   */

typedef struct irk_server irk_server;

typedef enum irk_request_state {
    IRK_REQ_QUEUED = 0, IRK_REQ_RUNNING = 1, IRK_REQ_DONE = 2, IRK_REQ_FAILED = 3
} irk_request_state;

typedef struct irk_request {
    int family;             /* irk_family                                     */
    int s;                  /* stages, 1..5                                   */
    irk_operator op;
    irk_options opt;        /* used when use_options != 0, else defaults      */
    int use_options;
    double t0, dt;          /* start time, step                               */
    int nsteps;             /* steps to take (>= 1)                           */
    double tol;             /* Newton tolerance (<= 0: options)               */
    const double *u0;       /* device, initial field; read at admission; the
                               caller keeps it valid until the request ends   */
    double *out;            /* device, final field written at completion      */
    void *stream;           /* hipStream_t on which u0 is produced (NULL: the
                               null stream): irk_server_submit records an
                               event on it, and the admission copy of u0
                               waits for that event, so u0 may still be in
                               flight on that stream when it is submitted    */
} irk_request;

typedef struct irk_request_info {
    int state;              /* irk_request_state                              */
    irk_status status;      /* IRK_OK, or why the request failed              */
    int steps_done;
    int newton_its, krylov_its;        /* summed over the steps               */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock       */
} irk_request_info;

/* arena: caller-owned device memory (256-byte aligned) the server carves
 * request state from; arena_bytes is the HBM admission budget; max_slots
 * bounds the number of requests resident at once.  Every slot's HIP
 * streams, events and pinned host staging are made here (grids of side up
 * to 16384), so that admitting a request allocates nothing and waits for
 * nothing.  IRK_E_DEVICE if they cannot be made (no GPU).                  */
irk_status irk_server_create(void *arena, size_t arena_bytes, int max_slots, irk_server **out);
/* Queue a request (nothing runs until irk_server_progress).  IRK_E_ARG for
 * invalid requests (also grids of side above 16384), IRK_E_DEVICE if the
 * ordering event on req->stream cannot be recorded; a request larger than
 * the whole arena is failed with IRK_E_NOMEM when it reaches the head of
 * the queue.  The result is in req->out once irk_server_info reports
 * IRK_REQ_DONE (an event behind the copy has completed by then).          */
irk_status irk_server_submit(irk_server *srv, const irk_request *req, long *id);
/* One non-blocking scheduling pass: retire finished requests whose last
 * work has completed, admit what fits (enqueueing only), advance every
 * running request; returns the number of requests queued, running or
 * finishing (-1 on NULL).                                                  */
int irk_server_progress(irk_server *srv);
irk_status irk_server_info(irk_server *srv, long id, irk_request_info *info);
/* Latencies (milliseconds, host clock) of every completed step so far (up to
 * cap written), the peak number of resident requests and arena bytes.      */
irk_status irk_server_stats(irk_server *srv, double *step_ms, int cap, int *nsteps, int *peak_running,
                            size_t *peak_bytes);
/* Finish or abandon everything and release the server (not the arena).     */
void irk_server_destroy(irk_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* IRK_H */
