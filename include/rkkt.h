/*
 * rkkt -- reduced-KKT (Schur complement) hot path of a block-structured
 * interior-point method, for AMD MI355X (gfx950), FP64.
 *
 * Method: Pacaud, Schanen, Shin, Maldonado, Anitescu, "Parallel interior-point
 * solver for block-structured nonlinear programs on SIMD/GPU architectures"
 * (arXiv 2301.04869).  The problem is the two-stage program of its problem
 * statement (eq. "originalproblem", slack form "slackedproblem"): N scenario
 * blocks with states x_i, one shared control u, state equations
 * g_i(x_i, u) = 0 and operational constraints h_i(x_i, u) + s_i = 0.  The
 * instance is the block (stochastic) AC optimal power flow of its case study.
 *
 * Variable split (the paper's Table 1 dimensions follow from it):
 *   x_i = [voltage angle of every non-reference bus (bus order);
 *          voltage magnitude of every bus without a generator (bus order)]
 *         n_x = 2 n_bus - n_gen - 1
 *   u   = [voltage magnitude of every generator bus (generator order);
 *          active output of every non-reference generator (generator order)]
 *         n_u = 2 n_gen - 1
 *   g_i = [P balance of every non-reference bus; Q balance of every bus
 *          without a generator]  (row r pairs with x entry r)
 *   h_i = [reference active output; reactive output of every generator;
 *          |S_from|^2 of every line; |S_to|^2 of every line]
 *         m = 2 n_line + n_gen + 1
 *   f_i = obj_weight * sum_k (c2_k (100 Pg_k)^2 + c1_k (100 Pg_k) + c0_k)
 * The reference bus is the bus of the reference generator (ref_bus); its
 * generator's output is per scenario (it balances each scenario).
 *
 * Layout.  All arrays are FP64 unless stated.  Per-scenario arrays are
 * scenario-major: a [N][n] array holds scenario i's n-vector contiguously at
 * offset i*n (the paper stacks one column per scenario, X_M = (x_1 .. x_M)).
 * Dense n_u x n_u matrices are row-major.  Pointers named *_dev or passed to
 * evaluate/condense/factor/step are device pointers; rkkt_network arrays and
 * the loads given to rkkt_create are host pointers.
 *
 * Ownership.  The caller owns every buffer it passes and keeps it alive until
 * the stream has finished the call.  The handle owns its sparsity patterns,
 * level schedules, cached Jacobian/Hessian/condensed/LU values and workspace,
 * all allocated by rkkt_create and freed by rkkt_destroy.  evaluate, condense,
 * factor and step allocate nothing and never synchronise the host with the
 * device; they enqueue work on the given stream and return.
 *
 * Errors.  Every call returns RKKT_OK (0) or a negative RKKT_ERR_* code and
 * then rkkt_last_error() describes it.  Argument errors are detected on the
 * host before anything is enqueued.  Numerical conditions found on the device
 * (a G_x pivot failing the health test, a non-finite value) are recorded in a
 * device status word that rkkt_status() reads (it synchronises the stream).
 * The library never aborts or exits.  A handle is not thread-safe; calls that
 * share a handle must be ordered on one stream.
 */
#ifndef RKKT_H
#define RKKT_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RKKT_OK = 0,
  RKKT_ERR_ARG = -1,          /* bad argument (null pointer, size, index)       */
  RKKT_ERR_HIP = -2,          /* a HIP runtime call failed                      */
  RKKT_ERR_SINGULAR_GX = -3,  /* a G_x pivot failed |u_ii| >= 1e-10 max|row i| */
  RKKT_ERR_NOT_PD = -4,       /* reduced matrix not positive definite           */
  RKKT_ERR_NONFINITE = -5,    /* non-finite value found on the device           */
  RKKT_ERR_NOMEM = -6         /* device allocation failed                       */
};

typedef struct rkkt_problem rkkt_problem;

/* Host-side description of one grid (per unit on 100 MVA). */
typedef struct {
  int n_bus, n_line, n_gen, n_load;
  int ref_bus;                       /* bus of the reference generator          */
  const int *line_from, *line_to;    /* [n_line] bus indices, pi-model lines    */
  const double *r, *x, *b;           /* [n_line] series r, x; total charging b  */
  const double *rate;                /* [n_line] apparent-power limit           */
  const int *gen_bus;                /* [n_gen] distinct buses                  */
  const double *pmin, *pmax, *qmin, *qmax;   /* [n_gen]                         */
  const double *c2, *c1, *c0;        /* [n_gen] $/MW^2h, $/MWh, $/h             */
  const double *vmin, *vmax;         /* [n_bus]                                 */
  const int *load_bus;               /* [n_load] distinct buses                 */
} rkkt_network;

typedef struct {
  int col_tile;   /* right-hand-side columns per workgroup in the reduction,
                     1..64; 0 picks one from the sizes                        */
  int device;     /* HIP device ordinal                                        */
  int variant;    /* how the reduction is closed (both give the same khat in
                     exact arithmetic):
                     1 adjoint: khat_i V = L_u - G_u^T G_x^-T L_x, two more
                       sparse triangular solves per column (the paper's form);
                     2 stacked product: khat = sum_i Z_i^T (K_i Z_i) as one
                       dense FP64 matrix-core product over the stacked rows of
                       all scenarios;
                     0 picks 2 when the reduction's data fits on chip, else 1 */
  int scen_per_group;  /* level-schedule grouping of the refactorisation and
                          step kernels: at most this many scenarios (1, 2 or
                          4, one wavefront each) per workgroup; 0 the most
                          that fit in LDS                                      */
  int chain_rows;      /* longest run of single-row levels at the end of the
                          elimination order solved sequentially in registers
                          instead of one barrier-separated phase per row:
                          0 the length with the fewest phases (at most 32),
                          -1 none, 1..32 at most that many                    */
  int sweep_form;      /* schedule of the reduction's triangular solves:
                          1 push: in the phase of each level, every row that
                            depends on that level's rows subtracts their terms
                            (a row is updated once per level it depends on);
                          2 pull: every row subtracts all its terms once, in
                            the phase of its own level, which needs its sources
                            only (forces the reduction's panels into device
                            memory, where it writes each row once per solve);
                          0 push when the reduction runs in LDS, else pull   */
} rkkt_options;

typedef struct {
  int n_x, n_u, m, n_scen, n_bus, n_line, n_gen;
  long long nnz_gx, nnz_gu, nnz_h, nnz_k, nnz_lu;   /* per scenario            */
  long long lu_update_flops;        /* multiply-adds of one G_x refactorisation */
  long long nnz_kx;                 /* entries of K in x columns (K_xx and K_ux) */
  long long n_ev;                   /* evaluation outputs per scenario          */
  long long n_trip;                 /* H^T Sigma_s H product terms per scenario  */
  int levels_up, levels_down;       /* level-schedule depths of the LU solves   */
  int col_tile;                     /* chosen column tile                       */
  long long workspace_bytes;        /* device bytes owned by the handle         */
  int variant;                      /* chosen reduction variant (1 or 2)         */
  int lds_reduce;                   /* reduction panels and factors in LDS       */
  int lds_group;                    /* refactorisation data in LDS               */
  int scen_per_group;               /* scenarios per workgroup of that kernel    */
  int lds_step;                     /* step data in LDS                          */
  int chain_rows;                   /* rows at the top of the elimination order,
                                       each alone in its level, that the solves
                                       and the refactorisation take sequentially */
  long long nnz_kxx, nnz_kxu, nnz_kuu; /* blocks of K (K_ux has nnz_kxu entries) */
  long long idx_bytes;              /* device bytes of the shared index arrays
                                       (patterns, schedules, gather lists); 0
                                       from rkkt_analyze                        */
  int n_load;                       /* load buses                               */
  int sweep_form;                   /* reduction solve schedules: 1 push, 2 pull */
} rkkt_dims;

/*
 * Symbolic analysis and allocation (problem statement; condensation and
 * reduction propositions fix which matrices exist).  Builds the fixed
 * sparsity patterns of G_x, G_u, H, W and K = W + H^T Sigma_s H, a
 * fill-reducing symmetric ordering of G_x (minimum degree), its filled LU
 * pattern with static diagonal pivots, level schedules and gather maps, and
 * copies them and the network to device `opt->device`.
 *   pd, qd : host [N][n_load] active / reactive load of every scenario.
 * Returns RKKT_ERR_ARG for inconsistent networks (bad bus index, duplicate
 * generator bus, ref_bus without generator, disconnected G_x).
 */
int rkkt_create(const rkkt_network* net, int n_scen, const double* pd, const double* qd,
                const rkkt_options* opt, rkkt_problem** out);

/* Host-only analysis: the sizes rkkt_create would produce, no device use. */
int rkkt_analyze(const rkkt_network* net, int n_scen, const rkkt_options* opt, rkkt_dims* out);

/*
 * Host-only: the fill-reducing order and the filled LU pattern rkkt_create
 * would use.  perm [n_x]: perm[i] is the external x index of internal row i;
 * f_ptr [n_x+1], f_col [nnz_lu]: CSR of the filled pattern of P G_x P^T
 * (sorted columns); sizes from rkkt_analyze.  The caller owns the buffers.
 */
int rkkt_analyze_lu(const rkkt_network* net, int n_scen, const rkkt_options* opt, int* perm,
                    int* f_ptr, int* f_col);

/*
 * Host-only: one of the level-sliced schedules rkkt_create would build, for
 * testing and inspection.  which: 0 reduction up (L and U^T solves), 1
 * reduction down (U and L^T solves), 2 step up, 3 step down, 4
 * refactorisation.  First call with ptr, ent, chain_pos NULL to get the
 * sizes: *nphase phases, *slots slots, *n_ent entries, *chain_rows rows in
 * the chain (the last chain_rows rows of the internal order, solved
 * sequentially after the up phases and before the down phases).  Second call
 * fills ptr [nphase * slots + 1] (entries of phase q, slot s:
 * [ptr[q slots + s], ptr[q slots + s + 1])), ent [4 n_ent] (solves: dest row,
 * source row, position of (dest, source) and of (source, dest) in f_col of
 * rkkt_analyze_lu; refactorisation: position of l_ik, position of u_kk,
 * length of the U part of row k, first index into the update targets) and
 * chain_pos [chain_rows^2] (position of (c0 + a, c0 + b), -1 if absent).
 * For the refactorisation *n_upd gets the number of update targets and upd
 * [n_upd] the targets (position of (i, j) for each U column j of row k, per
 * entry); n_upd and upd may be NULL for the other schedules.
 */
int rkkt_analyze_schedule(const rkkt_network* net, int n_scen, const rkkt_options* opt, int which,
                          int* nphase, int* slots, int* n_ent, int* chain_rows, int* ptr, int* ent,
                          int* chain_pos, int* n_upd, int* upd);

/* Replace the scenario loads with device arrays [N][n_load]. */
int rkkt_set_loads(rkkt_problem* p, const double* pd_dev, const double* qd_dev, hipStream_t stream);

/*
 * Line status per scenario (contingencies; the paper's scenarios may carry
 * them next to the loads, case-study section): status_dev [N][n_line] device
 * array, copied into the handle; 1 = in service, 0 = tripped (any factor
 * scales the line's series and charging admittance).  A tripped line keeps
 * its place in the shared patterns with zero admittance, so its flows and
 * every derivative of them are zero and the reduction is the one of the grid
 * without the line.  The caller keeps the grid connected (a tripped bridge
 * makes G_x singular: RKKT_ERR_SINGULAR_GX from the next condense).  All ones
 * after rkkt_create.  Stream-ordered; allocates nothing.
 */
int rkkt_set_line_status(rkkt_problem* p, const double* status_dev, hipStream_t stream);

int rkkt_dims_get(const rkkt_problem* p, rkkt_dims* out);

/*
 * Batched evaluation of every scenario block (paper: block evaluation through
 * a nonlinear basis, eq. "eval:block"; first- and second-order derivatives).
 *   x [N][n_x], u [n_u], y [N][n_x] (multipliers of g), z [N][m] (of h + s)
 * Outputs (device, caller-owned):
 *   f [N], grad_x [N][n_x], grad_u [N][n_u] (gradient of f_i w.r.t. u),
 *   g [N][n_x], h [N][m].
 * Also computes and caches on the handle the values of G_x, G_u, H and of the
 * Hessian of the Lagrangian W_i = Hess(f_i + y_i^T g_i + z_i^T h_i), used by
 * the next condense and step calls.
 */
int rkkt_evaluate(rkkt_problem* p, const double* x, const double* u, const double* y,
                  const double* z, double obj_weight, double* f, double* grad_x,
                  double* grad_u, double* g, double* h, hipStream_t stream);

/*
 * Condensation and reduction (propositions "Condensed KKT system" and
 * "Reduction"; the local reduction and global sum of the parallel KKT solver):
 *   K_i    = W_i + H_i^T Sigma_s,i H_i, with diag(sigma_x,i) + delta_w on K_xixi
 *   G_x,i  = L_i U_i (refactorised on the fixed pattern, every scenario)
 *   khat   = sum_i Z_i^T K_i Z_i + diag(sigma_u) + delta_w I,
 *            Z_i = [-(G_x,i)^-1 G_u,i ; I]
 * using the Jacobians and Hessian of the last rkkt_evaluate.
 *   sigma_x [N][n_x], sigma_u [n_u], sigma_s [N][m] : IPM diagonals (>= 0)
 *   khat    [n_u][n_u] row-major output
 * The K and LU values are kept on the handle for rkkt_step.  A pivot that
 * fails the health test sets RKKT_ERR_SINGULAR_GX in the device status word.
 */
int rkkt_condense(rkkt_problem* p, const double* sigma_x, const double* sigma_u,
                  const double* sigma_s, double delta_w, double* khat, hipStream_t stream);

/*
 * Dense Cholesky khat = L L^T in place (lower triangle, row-major; the input's
 * strict upper triangle is not referenced).  The reduced matrix is factorised
 * densely in the paper ("Lapack on the GPU").  info_dev (device int) gets 0
 * on success or the 1-based column of the first non-positive pivot, which
 * signals wrong inertia of the condensed KKT system.  For n_u <= 128, on
 * success, the strict upper triangle of each 16 x 16 diagonal block (rows and
 * columns 16 b .. 16 b + 15) receives the transpose of the strict lower
 * triangle of that block's inverse (khat[j][i] = (L_bb^-1)[i][j], i > j),
 * which rkkt_step applies as small dense products; the rest of the strict
 * upper triangle is left as it was.  When info_dev is not 0 the contents of
 * khat are unspecified.
 */
int rkkt_factor(rkkt_problem* p, double* khat, int* info_dev, hipStream_t stream);

/*
 * Newton step from the factorised reduced matrix: reduced right-hand side
 * (eq. "kkt:reduced"), p_u, then per-scenario recovery of p_x, p_y
 * (proposition "Reduction") and p_s, p_z (proposition "Condensed KKT system";
 * p_s is taken from the fourth block row of the augmented system,
 * p_s = -(r4 + H p_d)).  The step solves the augmented system of the paper
 * (eq. "kkt:augmented") with right-hand side -r:
 *   r1x [N][n_x], r1u [n_u], r2 [N][m], r3 [N][n_x], r4 [N][m]   (inputs)
 *   sigma_s [N][m]   the diagonal given to the last rkkt_condense
 *   chol [n_u][n_u]  the factor written by rkkt_factor
 *   px [N][n_x], pu [n_u], ps [N][m], py [N][n_x], pz [N][m]     (outputs)
 * Uses the K and LU values of the last rkkt_condense.
 */
int rkkt_step(rkkt_problem* p, const double* r1x, const double* r1u, const double* r2,
              const double* r3, const double* r4, const double* sigma_s, const double* chol,
              double* px, double* pu, double* ps, double* py, double* pz, hipStream_t stream);

/*
 * Interior-point solve on the device around evaluate / condense / factor /
 * step.  The paper runs its KKT solver inside an IPOPT-style primal-dual
 * method it does not spell out; this driver follows the published filter
 * line-search rules (start point pushed into the boxes; monotone barrier
 * update mu <- max(tol/10, min(0.2 mu, mu^1.5)) while E_mu <= 10 mu; fraction
 * to boundary max(0.99, 1 - mu); inertia correction on the reduced matrix;
 * switching / Armijo / filter acceptance with halving; no second-order
 * correction, no restoration phase).  Objective scaled by
 * min(1, 100 / max|grad f(x0)|) / N.  Per iteration the host reads a few
 * scalars (this call synchronises; its workspace is allocated on first use).
 * Outputs (device, caller-owned, may be NULL): the final x [N][n_x], u [n_u],
 * y [N][n_x], z [N][m], s [N][m].  res->status: 0 converged (scaled KKT
 * error <= tol), 1 iteration limit, 2 line search failed, 3 inertia
 * correction failed, 4 device error.
 */
typedef struct {
  double tol;      /* scaled KKT tolerance; <= 0 means 1e-8 */
  int max_iter;    /* < 0 means 200 */
  double mu0;      /* initial barrier parameter; <= 0 means 0.1 */
  int verbose;     /* one line per iteration on stdout */
  int warm_duals;  /* warm starts: bound multipliers 0 = implied by stationarity at the
                      start point plus complementarity at mu0, 1 = complementarity only */
} rkkt_ipm_options;

typedef struct {
  int status, iters;
  double obj;          /* average scenario cost (unscaled) */
  double kkt_error;    /* scaled KKT error at the last iterate */
  double mu;           /* final barrier parameter */
  double obj_weight;   /* objective weight used by evaluate */
  int factorizations;  /* Cholesky factorisations, inertia corrections included */
} rkkt_ipm_result;

int rkkt_solve(rkkt_problem* p, const rkkt_ipm_options* opt, double* x, double* u, double* y,
               double* z, double* s, rkkt_ipm_result* res, hipStream_t stream);

/*
 * The same solve from a given start point (a learned warm start): x0
 * [N][n_x], u0 [n_u] are pushed into their boxes by 1e-6 (relative), the
 * slacks follow from h as in the cold start, y0 [N][n_x], z0 [N][m] are the
 * multipliers for the objective weighted 1/N (the solver rescales them to its
 * own objective scaling; a cold solve's multipliers convert with the factor
 * 1 / (N res.obj_weight)), and every bound multiplier is set from
 * complementarity at opt->mu0, which is also the starting barrier parameter,
 * plus (opt->warm_duals = 0) the part of the stationarity condition of its
 * variable that it must carry: with v the derivative of the Lagrangian
 * without bound terms at the start point (grad f + G^T y + H^T z for x and
 * u, z for s), the lower-bound multiplier gets max(v, 0) and the upper-bound
 * multiplier max(-v, 0), so that the start is dual feasible where the
 * multipliers are right (the slack form's dual condition z = z_L - z_U for
 * s, and its counterparts for x and u).
 * Device arrays; RKKT_ERR_ARG if any start array is null.
 */
int rkkt_solve_warm(rkkt_problem* p, const rkkt_ipm_options* opt, const double* x0, const double* u0,
                    const double* y0, const double* z0, double* x, double* u, double* y, double* z,
                    double* s, rkkt_ipm_result* res, hipStream_t stream);

/*
 * Stage timing with HIP events recorded on the caller's stream around every
 * internal launch group (for benchmarks).  rkkt_profile_begin creates up to
 * max_records event pairs (this call allocates) and starts recording;
 * rkkt_profile_end synchronises `stream`, writes the summed milliseconds and
 * the number of records of every stage into ms[RKKT_NSTAGES] and
 * count[RKKT_NSTAGES], stops recording and releases the events.  Records past
 * max_records are dropped (count stops growing).
 */
enum {
  RKKT_STAGE_EVALUATE = 0,        /* line kernel, gathers, line Hessians, W     */
  RKKT_STAGE_CONDENSE_VALUES,     /* K = W + H^T Sigma_s H + diagonals          */
  RKKT_STAGE_REFACTOR,            /* batched LU of G_x                          */
  RKKT_STAGE_REDUCE,              /* local reduction, all scenarios and tiles   */
  RKKT_STAGE_SCENARIO_SUM,        /* sum over scenarios + Sigma_u + delta_w     */
  RKKT_STAGE_FACTOR,              /* dense Cholesky                             */
  RKKT_STAGE_STEP_RHS,            /* reduced right-hand side contributions      */
  RKKT_STAGE_REDUCED_SOLVE,       /* p_u                                        */
  RKKT_STAGE_STEP_RECOVER,        /* p_x, p_y, p_s, p_z                         */
  RKKT_STAGE_STACKED_PRODUCT,     /* Z^T (K Z) over all scenarios (variant 2)   */
  RKKT_NSTAGES
};
int rkkt_profile_begin(rkkt_problem* p, int max_records);
int rkkt_profile_end(rkkt_problem* p, hipStream_t stream, double* ms, int* count);

/*
 * Machine-balance probes for roofline reports (measurement only; no stage of
 * the hot path uses them).  On `device` it times, best of five launches after
 * one untimed launch each, on a stream of its own:
 *   hbm_gbs       a device-to-device copy of 1 GiB in 16-byte units
 *                 (GB/s = 2 GiB moved / time);
 *   fp64_vec_tfs  eight independent FP64 multiply-add chains per thread over
 *                 8 workgroups of 256 threads per compute unit (TFLOP/s);
 *   fp64_mfma_tfs four independent v_mfma_f64_16x16x4f64 accumulations per
 *                 wavefront over the same grid (TFLOP/s, 2048 flops each).
 * Allocates and frees 2 GiB plus a small output buffer and synchronises the
 * device.  RKKT_ERR_ARG for a null output, RKKT_ERR_NOMEM when the buffers do
 * not fit, RKKT_ERR_HIP for any other failed HIP call (outputs then unset).
 */
int rkkt_probe_peaks(int device, double* hbm_gbs, double* fp64_vec_tfs, double* fp64_mfma_tfs);

/*
 * One hot-path pass with fixed buffers: evaluate, condense, factor, step (the
 * calls above, each argument as documented there), with the same results as
 * those calls in that order, except that the factor of khat is written to
 * chol (its lower triangle; khat is left as it is and the strict upper
 * triangle of chol is not written).  The step's right-hand-side solves run on
 * a second stream of the handle, concurrently with the reduction and the
 * factorisation; the pass is ordered after earlier work on `stream`, and later
 * work on `stream` is ordered after all of it.
 */
typedef struct {
  const double *x, *u, *y, *z;
  double obj_weight;
  double *f, *grad_x, *grad_u, *g, *h;
  const double *sigma_x, *sigma_u, *sigma_s;
  double delta_w;
  double *khat, *chol;
  int* info;
  const double *r1x, *r1u, *r2, *r3, *r4;
  double *px, *pu, *ps, *py, *pz;
} rkkt_iteration;

int rkkt_iterate(rkkt_problem* p, const rkkt_iteration* it, hipStream_t stream);

/*
 * The same pass captured once into a HIP graph owned by the handle
 * (rkkt_graph_capture records it from a capture stream of the handle; no
 * device work runs) and replayed on `stream` by rkkt_graph_launch: one launch
 * per iteration instead of one per kernel.  The graph keeps the pointers and
 * scalars of `it`; capture again after changing any of them (e.g. delta_w).
 */
int rkkt_graph_capture(rkkt_problem* p, const rkkt_iteration* it);
int rkkt_graph_launch(rkkt_problem* p, hipStream_t stream);

/*
 * Graph batch of independent instances (rkkt_batch_create / launch /
 * destroy): switched off.  A capture of several instances whose passes forked
 * to side streams ended in a host segmentation fault inside this call and
 * the cause was not shown, so rkkt_batch_create returns RKKT_ERR_ARG with
 * that message and creates nothing; rkkt_batch_launch and
 * rkkt_batch_destroy accept only what it would return.  Independent
 * instances in one launch per stage: rkkt_multi_* below.
 */
/*
 * Independent instances of uneven sizes in one launch per kernel
 * configuration (the paper batches the independent scenario blocks of one
 * problem on a device, parallel KKT solver section; here whole independent
 * problems of different sizes, each with its own scenarios and reduced
 * matrix, no sum across instances).  rkkt_multi_create takes n distinct
 * handles (each created by rkkt_create with its own, possibly autotuned,
 * launch shape) and one rkkt_iteration per handle (device buffers that must
 * outlive the multi handle; their addresses are copied to the device here).
 * rkkt_multi_iterate runs, for every instance, the pass of rkkt_iterate
 * (evaluate, condense, factor, step) on one stream, with every kernel of the
 * pass launched once for all instances that use the same kernel variant and
 * block size: a table maps each block to (instance, block of that instance's
 * own grid), the dynamic LDS is the group's largest; the outputs equal
 * rkkt_iterate's bit for bit.  rkkt_multi_launches gives the number of
 * launches of one pass.  rkkt_multi_capture records that pass as one HIP
 * graph (one stream, no forks) and rkkt_multi_launch replays it.  The handles
 * are not owned and must outlive the multi handle; rkkt_status on each handle
 * reports its own device status.  Errors: RKKT_ERR_ARG (null or repeated
 * handle, null array, non-finite scalar, instances on different devices),
 * RKKT_ERR_HIP, RKKT_ERR_NOMEM; message in rkkt_multi_last_error.
 */
typedef struct rkkt_multi rkkt_multi;
int rkkt_multi_create(rkkt_problem* const* problems, const rkkt_iteration* its, int n, rkkt_multi** out);
int rkkt_multi_iterate(rkkt_multi* m, hipStream_t stream);
int rkkt_multi_capture(rkkt_multi* m);
int rkkt_multi_launch(rkkt_multi* m, hipStream_t stream);
int rkkt_multi_launches(const rkkt_multi* m);
int rkkt_multi_destroy(rkkt_multi* m);
const char* rkkt_multi_last_error(const rkkt_multi* m);

typedef struct rkkt_batch rkkt_batch;

/*
 * Autotuner of the launch shape (a project addition: the paper fixes its
 * batch width by hand).  Builds one handle per candidate, evaluates it at a
 * fixed interior point (angles 0, magnitudes 1, outputs mid-range,
 * multipliers 0, all IPM diagonals and residuals 1, delta_w = 1) and times
 * `reps` calls with HIP events, in two stages: (1) every reduction variant
 * (1 and 2; 2 only while its stacked panels stay under 4 GiB) with the
 * automatic column tile and with 8, 16, 32, 64 up to n_u, each with the
 * automatic, push and pull forms of the reduction's solve schedules (and the
 * LDS or device-memory layout each implies), timed on condense; (2) the
 * level-schedule grouping for the winner of (1): scen_per_group 0, 1, 2, 4 x
 * chain_rows 0, -1, timed on whole rkkt_iterate passes.  Writes the fastest
 * options (device copied from opt; col_tile, variant and sweep_form as
 * resolved, scen_per_group and chain_rows as requested) into *best and its mean pass time in ms into
 * *best_ms; allocates and frees device memory and synchronises.
 */
int rkkt_autotune(const rkkt_network* net, int n_scen, const double* pd, const double* qd,
                  const rkkt_options* opt, int reps, rkkt_options* best, double* best_ms);
int rkkt_batch_create(rkkt_problem* const* problems, const rkkt_iteration* its, int n,
                      rkkt_batch** out);
int rkkt_batch_launch(rkkt_batch* b, hipStream_t stream);
int rkkt_batch_destroy(rkkt_batch* b);

/*
 * Synchronise `stream`, read and clear the device status word:
 * *code = RKKT_OK, RKKT_ERR_SINGULAR_GX or RKKT_ERR_NONFINITE;
 * *scenario = first scenario that raised it (or -1).
 */
int rkkt_status(rkkt_problem* p, hipStream_t stream, int* code, int* scenario);

int rkkt_destroy(rkkt_problem* p);

/* Message of the last error on this handle (or of the last failed
 * rkkt_create / rkkt_analyze when p is NULL).  Never NULL. */
const char* rkkt_last_error(const rkkt_problem* p);

#ifdef __cplusplus
}
#endif

#endif /* RKKT_H */
