/*
 * pasm.h -- C ABI of the MI355X (gfx950) parallel augmented subspace eigensolver.
 *
 * The library computes the k smallest eigenpairs of the P1 finite element
 * discretisation of
 *
 *     -div(kappa grad u) + V u = lambda u   in (0,1)^d,   u = 0 on the boundary,
 *
 * (the model problem of Section 2, with the zeroth-order term of the second
 * example in Section 5) on the uniform Kuhn simplex mesh of mesh size h: the
 * "/" split of squares in 2D, Kuhn tetrahedra in 3D.  It implements
 * Algorithm 2 (parallel augmented subspace scheme) with h_1 = H: the coarse
 * eigenproblem on V_H gives the start, and every eigenpair is then corrected
 * independently on the finest mesh by Algorithm 1 (one correction step):
 *   1. a few multigrid V-cycles for the boundary value problem
 *          A_h u^ = lambda M_h u                 (Algorithm 1, step 1);
 *   2. the borders b = P^T A_h u~, c = P^T M_h u~, beta = u~^T A_h u~,
 *      zeta = u~^T M_h u~ of the augmented space V_H + span{u~} and the
 *      (N_H+1)-dimensional generalized eigenproblem of Section 3.1 (matrix
 *      form), keeping the eigenvector with the largest component along u~
 *      (the score |u_H . c + alpha zeta|), prolongated back to the fine mesh.
 * All k eigenpairs are processed together as k right-hand sides of the same
 * sweeps, never orthogonalised against each other (Section 3.2).
 *
 * Conventions for every entry point
 *   - Vectors of nodal values hold the interior nodes only, numbered
 *     lexicographically with x fastest; a batch of k vectors is stored as k
 *     consecutive blocks of `ld` doubles (ld >= number of interior nodes).
 *   - Per-element input arrays follow the element order of the Kuhn mesh:
 *     cell index (x fastest) major, simplex index minor, the simplex p of a
 *     cell being the monotone vertex path o, o+e[pi0], o+e[pi0]+e[pi1], ...
 *     for pi the p-th permutation of (0..d-1) in lexicographic order (2D:
 *     p = 0 lower triangle (o, o+ex, o+ex+ey), p = 1 upper triangle).
 *   - Eigenvectors are returned M-normalised (u^T M_h u = 1), eigenvalues in
 *     the order of their coarse start index.
 *   - Host inputs are copied during the call; the library keeps no pointer to
 *     caller memory.  The context owns its device memory, allocated once in
 *     pasm_setup and released in pasm_destroy; pasm_iterate allocates nothing.
 *   - Every call returns a status; no C++ exception crosses the ABI.  After a
 *     failure pasm_last_error() on the same context describes it.
 *   - A context is used by one host thread at a time.  All device work runs
 *     on the stream given in the options (NULL: a stream the context creates).
 */
#ifndef PASM_H
#define PASM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PASM_API __attribute__((visibility("default")))

typedef struct pasm_ctx pasm_ctx;

typedef enum pasm_status {
    PASM_OK = 0,
    PASM_E_INVALID = 1,    /* bad argument: sizes, mesh ratio, k, null pointer */
    PASM_E_NOMEM = 2,      /* device or host allocation failed */
    PASM_E_DEVICE = 3,     /* HIP, rocBLAS or rocSOLVER call failed */
    PASM_E_STATE = 4,      /* call out of order (e.g. iterate before setup) */
    PASM_E_NOTCONV = 5,    /* iteration cap reached before the tolerance */
    PASM_E_BREAKDOWN = 6   /* non-finite value detected in the eigenpairs */
} pasm_status;

typedef enum pasm_precision {
    PASM_FP64 = 0,         /* every step in FP64 */
    PASM_MIXED = 1         /* V-cycles in FP32 on FP64 residuals (defect correction);
                              residuals, borders, Rayleigh quotients and the
                              augmented eigensolve in FP64 */
} pasm_precision;

typedef enum pasm_smoother {
    PASM_JACOBI = 0,       /* damped Jacobi, x <- x + omega D^{-1}(f - A x) */
    PASM_CHEBYSHEV = 1,    /* Chebyshev semi-iteration on D^{-1}A over [rho/alpha, rho] */
    PASM_LEARNED = 2       /* 3D, constant coefficients: one step of a learned convolutional
                              corrector per smoothing phase, x <- x + N(D^{-1}(f - A x)),
                              trained at set-up on residuals of plain V-cycles; damped
                              Jacobi (nu_pre / nu_post sweeps) is the fallback, taken for
                              any V-cycle whose residual reduction is worse than the plain
                              cycle's, and throughout when the learned cycle reduces the
                              residual less per unit time than the plain one at set-up
                              (see pasm_learned_report) */
    ,
    PASM_CG = 3            /* the smoother of the paper's experiments (Section 5: one
                              multigrid step with 2 CG steps for pre- and post-smoothing):
                              nu_pre / nu_post steps of plain conjugate gradients on
                              A_l x = f_l from the current iterate, on every level; each
                              step forms two inner products over the level per
                              right-hand side (block partial sums added in a fixed order) */
} pasm_smoother;

/* Unit box (0,1)^dim; dim = 2 or 3. */
typedef struct pasm_domain {
    int dim;
} pasm_domain;

/* Coefficients of -div(kappa A grad u) + V u, constant per fine element
 * (element order above).  NULL kappa means kappa = 1, NULL potential means
 * V = 0, NULL tensor means A = I.  kappa must be finite and positive,
 * potential finite and >= 0, every tensor symmetric positive definite.
 * 2D: kappa and potential.  3D: kappa, potential and the full tensor (the
 * operator of the second example of Section 5 is A = I + (x - 1/2)(x - 1/2)^T,
 * V = exp(prod_i (x_i - 1/2)), taken at element centroids); any of them makes
 * every level a 15-point operator (Galerkin coarse levels), smoothed with
 * unfused Jacobi / Chebyshev / CG sweeps. */
typedef struct pasm_coefficients {
    const double* kappa;       /* n_elements values or NULL */
    const double* potential;   /* n_elements values of V at the element centroid, or NULL */
    size_t n_elements;         /* (1/h)^dim * dim! when any array is given */
    const double* tensor;      /* 3D: 6 * n_elements values (a11 a22 a33 a12 a13 a23 per
                                  element, the diffusion tensor at its centroid), or NULL */
} pasm_coefficients;

typedef struct pasm_options {
    int precision;      /* pasm_precision */
    int smoother;       /* pasm_smoother */
    int nu_pre;         /* Jacobi sweeps / Chebyshev degree before restriction */
    int nu_post;        /* ... after prolongation */
    int vcycles;        /* V-cycles per boundary value problem (>= 1) */
    int max_iter;       /* cap used by pasm_solve */
    double tol;         /* converged when max_i |lambda_i - lambda_i_prev| / lambda_i < tol */
    double omega;       /* Jacobi weight; <= 0 selects 4/5 (2D) or 6/7 (3D) */
    double cheb_alpha;  /* Chebyshev interval [rho/alpha, rho]; <= 0 selects 4 (2D) or 6 (3D) */
    void* stream;       /* hipStream_t, or NULL */
    int fused_smoothing;/* 1: all steps of a smoothing phase in one pass over memory where
                           supported (2D, up to 4 steps), 0: one launch per step */
    int exhaustive_selection; /* 1: score every eigenvalue of the augmented problem;
                                 0 (default): stop once the scores already computed
                                 provably contain the winner (same choice, less work) */
} pasm_options;

/* Fill *opt with the defaults: FP64, Jacobi 2/2, 2 V-cycles, 50 iterations,
 * tol 1e-10, omega and alpha by dimension, own stream, fused smoothing. */
PASM_API void pasm_default_options(pasm_options* opt);

/* Build the mesh hierarchy H = h_1 > 2h > ... > h (ratio 2, Section 3), the
 * coarse operators, the coarse generalized eigenproblem of Algorithm 2,
 * step 1 (A_H q = theta M_H q, dense, on the device), and the start
 * lambda_i = theta_i, u_i = P q_i for i < k.
 *   out        receives the new context (set to NULL on failure)
 *   H, h       coarse and fine mesh sizes: 1/H and 1/h integers, 1/h = 2^j / H,
 *              j >= 0 (j = 0: the augmented space degenerates and the coarse
 *              Ritz pairs are returned)
 *   k          number of eigenpairs, 1 <= k < N_H = (1/H - 1)^dim (Remark 3.1)
 *   opt        NULL for defaults
 * Device memory for every buffer of the iteration is allocated here. */
PASM_API pasm_status pasm_setup(pasm_ctx** out, const pasm_domain* domain,
                                const pasm_coefficients* coef, double H, double h,
                                int k, const pasm_options* opt);

/* One outer iteration = one correction step (Algorithm 1) for all k
 * eigenpairs at once.  *converged (may be NULL) is set to 1 when the
 * maximum relative eigenvalue change is below opt.tol.  Synchronises the
 * stream once (to read the k eigenvalues).  Returns PASM_E_BREAKDOWN if an
 * eigenvalue is not finite. */
PASM_API pasm_status pasm_iterate(pasm_ctx* ctx, int* converged);

/* n >= 1 steps of Algorithm 1 back to back, with one synchronisation of the
 * stream at the end (pasm_iterate synchronises after every step): for
 * callers that know how many steps they need before testing.  *converged
 * (may be NULL) reports the stop test of the last step (maximum relative
 * eigenvalue change over that step below opt.tol).  The results equal n
 * calls of pasm_iterate bit for bit; on 2D FP64 contexts whose finest level
 * takes the marching smoother, a step's prolongation is formed inside the
 * next step's first pre-smoothing pass.  PASM_E_INVALID if n < 1;
 * PASM_E_BREAKDOWN if an eigenvalue is not finite after the last step.
 * Allocates nothing. */
PASM_API pasm_status pasm_iterate_n(pasm_ctx* ctx, int n, int* converged);

/* Return to the start of Algorithm 2 (lambda_i = theta_i, u_i = P q_i) on
 * the device, reusing the coarse eigenpairs computed by pasm_setup.  The
 * work is enqueued on the context's stream without waiting for it (every
 * later call on the context is ordered after it).  Where the next step's
 * first pre-smoothing can form u_i and theta_i M u_i in its own pass (2D
 * FP64, marching finest level), they are left to it; every other call that
 * reads u forms them first, so callers see no difference. */
PASM_API pasm_status pasm_restart(pasm_ctx* ctx);

/* Algorithm 2 with its nested step 2(A): return to the coarse start
 * (lambda_i = theta_i, u_i = q_i on V_H = V_{h_1}), then for every
 * intermediate mesh h_2 = H/2, ..., h_{n-1} = 2h in turn take the previous
 * mesh's result as the start (a coarser P1 function is also a finer one:
 * its nodal values are prolongated) and run varpi >= 1 correction steps
 * (Algorithm 1 with the same coarse space V_H, on that mesh; varpi = 1 as in
 * Remark 3.2).  The context is left on the finest mesh at the start of step
 * 2(B): the following pasm_iterate / pasm_solve calls are the finest-level
 * corrections, and the stop test of the first one compares with the last
 * intermediate eigenvalues.  The operators of an intermediate mesh are the
 * Galerkin restrictions of the finest ones (for constant coefficients and
 * per-element kappa: the rediscretisation with kappa averaged over the
 * children); a context with a potential term returns PASM_E_INVALID.  The
 * first call allocates the intermediate meshes' vectors (they share the
 * coarse space and stream); later calls allocate nothing.  Synchronises the
 * stream once.  With fewer than three meshes it is pasm_restart. */
PASM_API pasm_status pasm_restart_nested(pasm_ctx* ctx, int varpi);

/* Iterate until converged or opt.max_iter iterations; *iterations (may be
 * NULL) receives the count.  PASM_E_NOTCONV if the cap was reached. */
PASM_API pasm_status pasm_solve(pasm_ctx* ctx, int* iterations);

/* Copy the current eigenvalues (k doubles) and, if U != NULL, the eigenvectors
 * (k blocks of ldu doubles, host memory) out of the context.  With U != NULL
 * the call may first enqueue device work that changes the context: a step
 * of pasm_iterate_n or a pasm_restart can leave the last prolongation
 * u = P Q y' + s u~ to the next step's first pass, and it is formed here
 * instead.  An eigenvalue-only call (U == NULL) enqueues nothing. */
PASM_API pasm_status pasm_eigenpairs(pasm_ctx* ctx, double* lambda, double* U, size_t ldu);

/* Same, with U in device memory (written on the context's stream, which is
 * synchronised before return); may form a pending prolongation first, as
 * pasm_eigenpairs. */
PASM_API pasm_status pasm_eigenvectors_device(pasm_ctx* ctx, double* U_dev, size_t ldu);

/* Replace the current state by (lambda, U) (host memory, layout as above):
 * a warm start or checkpoint restore.  The previous-eigenvalue record used by
 * the stop test is set to lambda.  PASM_E_INVALID (state unchanged) if any
 * lambda_i or entry of U is not finite: no kernel ever sees such input. */
PASM_API pasm_status pasm_set_state(pasm_ctx* ctx, const double* lambda, const double* U, size_t ldu);

/* Per-eigenpair report of the last iteration (host arrays of k entries, any
 * may be NULL): the selected augmented eigenvalue's rank from the bottom of
 * the augmented spectrum, its score |b(u_new, u~)|, and a flag word
 * (bit 0: augmentation skipped because u~ lay in V_H; bit 1: a deflated
 * coarse direction was selected). */
PASM_API pasm_status pasm_last_selection(const pasm_ctx* ctx, int* rank, double* score, int* flags);

/* The coarse generalized eigenpairs of Algorithm 2, step 1 (h_1 = H):
 * theta (N_H values, ascending) and Q (N_H x N_H, column j the eigenvector of
 * theta_j, column-major, Q^T M_H Q = I).  Either pointer may be NULL. */
PASM_API pasm_status pasm_coarse_eigenpairs(const pasm_ctx* ctx, double* theta, double* Q);

/* Border quantities of the last iteration (Section 3.1, matrix form), host
 * arrays: beta_zeta[k][2] = (u~^T A_h u~, u~^T M_h u~), p[k][N_H] = Q^T b and
 * q[k][N_H] = Q^T c with b = P^T A_h u~, c = P^T M_h u~.  Any pointer may be NULL. */
PASM_API pasm_status pasm_last_borders(const pasm_ctx* ctx, double* beta_zeta, double* p, double* q);

/* Sizes: interior fine nodes, interior coarse nodes, number of levels. */
PASM_API size_t pasm_num_dofs(const pasm_ctx* ctx);
PASM_API size_t pasm_coarse_dofs(const pasm_ctx* ctx);
PASM_API int pasm_num_levels(const pasm_ctx* ctx);

/* Release every resource of the context.  NULL is accepted. */
PASM_API pasm_status pasm_destroy(pasm_ctx* ctx);

PASM_API const char* pasm_status_string(pasm_status s);
/* Message of the last failure on ctx; with ctx == NULL, of the last failed
 * pasm_setup on the calling thread. */
PASM_API const char* pasm_last_error(const pasm_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Building blocks, exposed for verification against the CPU oracle.  Vectors
 * are device pointers in the compact interior layout above, FP64.
 * ------------------------------------------------------------------------- */

enum { PASM_OP_STIFFNESS = 0, PASM_OP_MASS = 1 };

/* y = A_l x (op = STIFFNESS, the level's stiffness + potential operator) or
 * y = M_h x (op = MASS, finest level only) for nrhs vectors.  Level 0 is V_H,
 * level pasm_num_levels()-1 the finest mesh. */
PASM_API pasm_status pasm_apply_operator(pasm_ctx* ctx, int level, int op, const double* x,
                                         double* y, size_t ld, int nrhs);

/* ncycles V-cycles of the library's multigrid (same smoother, levels and
 * coarse solve as pasm_iterate, in the context's precision) for A_h x = f on
 * the finest level, starting from x; nrhs <= k vectors, x updated in place. */
PASM_API pasm_status pasm_vcycle(pasm_ctx* ctx, const double* f, double* x, size_t ld, int nrhs,
                                 int ncycles);

/* Graph replay of correction steps (the batching of Algorithm 1's launches,
 * which the paper leaves to the implementation).  enable = 1: pasm_iterate,
 * pasm_iterate_n and pasm_solve record the launches of a correction step
 * into a hipGraph the first time a step starts from a given context state
 * (which buffers hold u, f and the eigenvalues, and which fused pass forms
 * what; at most 16 graphs are kept; a context's very first step runs
 * unrecorded) and replay it for every later step from that state: the same kernels and arguments, so the same results bit for
 * bit, with one launch per step instead of one per kernel.  Steps that
 * record profiling events (pasm_profile) or run the learned smoother run
 * unrecorded.  A step whose recording fails runs unrecorded and switches the
 * replay off for the context.  enable = 0 (the default) destroys the graphs.
 * The call synchronises the context's stream.  The graphs belong to the
 * context and are destroyed with it. */
PASM_API pasm_status pasm_use_graph(pasm_ctx* ctx, int enable);
/* Whether the replay is on, the graphs held and the steps replayed from a
 * graph since set-up (any output may be NULL). */
PASM_API pasm_status pasm_graph_stats(const pasm_ctx* ctx, int* enabled, int* graphs, long* replays);

/* Time the launches of one kernel class inside subsequent pasm_iterate calls
 * with HIP events recorded on the context's stream (enable = 1 starts and
 * clears the record, 0 stops).  kernel: 0 = fine-level smoothing sweep. */
PASM_API pasm_status pasm_profile(pasm_ctx* ctx, int kernel, int enable);
/* Number of timed launches, their summed duration (ms) and the bytes each
 * launch must move at minimum (the algorithmic traffic of that kernel). */
PASM_API pasm_status pasm_profile_read(pasm_ctx* ctx, int kernel, long* launches, double* total_ms,
                                       double* bytes_per_launch);

/* ---------------------------------------------------------------------------
 * Learned smoother (opt.smoother = PASM_LEARNED; not part of the paper's
 * method: an alternative for its "some multigrid steps").
 *
 * N(rho)(v) = sum_{c,t} W2[c][t] h_c(v + t), h_c = max(0, sum_t W1[c][t] rho(v + t)),
 * 16 channels c, 27 offsets t in {-1,0,1}^3 (index (dz+1)*9 + (dy+1)*3 + (dx+1)),
 * h zero off the interior nodes.  Both convolutions run as bfloat16 matrix
 * products with FP32 accumulation.  Weights are FP32 [2][16][27] (W1 then
 * W2).  Training (at set-up, and by pasm_learned_train) minimises
 * (1/S) sum_s ||r_s - A N(r_s / D)||^2 / ||r_s||^2 with Adam, over residuals
 * r_s that plain V-cycles leave on random errors, on the level with 32 cells
 * per side (or the finest level below the finest).  The weights start as the
 * damped Jacobi step (two channels passing +rho and -rho).
 * ------------------------------------------------------------------------- */
typedef struct pasm_learned_stats {
    int enabled;            /* 1 while the learned smoother is in use */
    int train_steps;        /* Adam steps taken so far */
    double loss_first;      /* training loss at the first and the latest step */
    double loss_last;
    double plain_rate;      /* residual reduction of one plain V-cycle (set-up, worst right-hand side) */
    double learned_rate;    /* ... of one learned V-cycle */
    double plain_cycle_ms;  /* time of one plain / learned V-cycle at set-up */
    double learned_cycle_ms;
    long cycles_learned;    /* V-cycles kept with the learned smoother */
    long cycles_fallback;   /* V-cycles redone with the plain smoother */
} pasm_learned_stats;

PASM_API pasm_status pasm_learned_report(const pasm_ctx* ctx, pasm_learned_stats* out);
PASM_API pasm_status pasm_learned_weights(const pasm_ctx* ctx, float* w);
/* The most recent per-cycle residual reductions sqrt(|r_new|^2 / |r_old|^2)
 * of learned V-cycles, one per right-hand side and cycle, oldest first (the
 * library keeps the last 4096).  Copies at most max into out (host);
 * returns the count, or -1 for a null context or a null out with max > 0. */
PASM_API int pasm_learned_ratios(const pasm_ctx* ctx, double* out, int max);
/* Replace the weights (host [2][16][27]); the stored rates are kept. */
PASM_API pasm_status pasm_learned_set_weights(pasm_ctx* ctx, const float* w);
/* Fallback threshold: a learned V-cycle is redone with the plain smoother
 * when it reduces some right-hand side's residual by less than this factor.
 * rate <= 0 restores the default, the plain cycle's rate measured at set-up. */
PASM_API pasm_status pasm_learned_set_threshold(pasm_ctx* ctx, double rate);
/* Override the set-up decision: 1 smooths with the learned step (with the
 * per-cycle fallback), 0 with the plain smoother only. */
PASM_API pasm_status pasm_learned_enable(pasm_ctx* ctx, int enable);
/* steps more Adam steps from the current weights; loss_history (may be NULL)
 * receives the loss of each step. */
PASM_API pasm_status pasm_learned_train(pasm_ctx* ctx, int steps, double* loss_history);
/* One learned step on level l >= 1, out = x + N((f - A_l x) / D), for nrhs
 * vectors (device, compact FP64, ld apart), in the context's V-cycle precision. */
PASM_API pasm_status pasm_learned_step(pasm_ctx* ctx, int level, const double* x, const double* f, double* out,
                                       size_t ld, int nrhs);
/* Training loss and gradient (host grad [2][16][27]) of ns residual samples
 * r (device, compact FP64, ld apart) on level l >= 1, with the current weights. */
PASM_API pasm_status pasm_learned_loss_grad(pasm_ctx* ctx, int level, const double* r, size_t ld, int ns,
                                            double* loss, double* grad);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, allocation-free serving loops, harnesses that forbid it): the
 * same loss and gradient as pasm_learned_loss_grad, same arguments, with
 * every device buffer (the trainer's activations, partial sums and the FP32
 * copy of the samples) taken from a fixed scratch array of 72 MiB that the
 * library keeps per GPU until the process ends, instead of hipMalloc.  It
 * holds 8 samples on the 32-cell level, or up to 63 on the 16-cell level;
 * larger requests return PASM_E_INVALID (pasm_last_error gives the bytes
 * needed) before any device work.  No hipMalloc, hipFree or other
 * allocating device call is made.  The array is shared by every call on one
 * GPU and keeps the last call's contents (the part used is cleared at the
 * start of each call): calls that overlap on one GPU, from any context or
 * thread, race and must be serialised by the caller. */
PASM_API pasm_status pasm_learned_loss_grad_noalloc(pasm_ctx* ctx, int level, const double* r, size_t ld,
                                                    int ns, double* loss, double* grad);

/* ---------------------------------------------------------------------------
 * Batches of problems of uneven size.
 *
 * Eigenpairs are corrected independently (Algorithm 2 runs one correction
 * step per eigenpair with no exchange between them), so several problems
 * sharing the coarse size H and the count k can advance together.  A batch
 * stores every multigrid level level-major: level l (1/H * 2^l cells per
 * side) holds the k vectors of every member whose fine mesh is at least that
 * fine, and each step of the iteration is one launch per level over all those
 * members (members of equal fine size share the fine-level launches).  Every
 * level uses the general 7-point operator form (stiffness + potential,
 * Galerkin coarse levels) with the member's own coefficients and smoother
 * bound.  V-cycles always run as defect correction: r = f - A u in FP64,
 * the cycle from zero in the cycle's precision (FP32 for PASM_MIXED, FP64
 * otherwise), then u += e in FP64.
 * The device work of one iteration is recorded once into a HIP graph and
 * replayed (pasm_batch_use_graph).  Smoothing tile heights per level are
 * chosen at set-up by timing each candidate on the batch itself.
 * ------------------------------------------------------------------------- */
typedef struct pasm_batch pasm_batch;

/* One member: fine mesh size and coefficients (2D, layout as for pasm_setup). */
typedef struct pasm_instance {
    double h;
    pasm_coefficients coef;
} pasm_instance;

/* Set up n >= 1 members on the unit square (dim must be 2), all with coarse
 * size H and k eigenpairs each; member i has fine size inst[i].h (1/h a
 * multiple 2^j / H with j >= 1).  Options as for pasm_setup; the smoothing
 * tile heights are autotuned unless opt->fused_smoothing is 0 (one launch
 * per smoothing step).  The coarse eigenproblem of every member is solved
 * here; the start is lambda = theta_i, u_i = P q_i per member. */
PASM_API pasm_status pasm_batch_setup(pasm_batch** out, const pasm_domain* domain, const pasm_instance* inst,
                                      int n, double H, int k, const pasm_options* opt);

/* One correction step for all n * k eigenpairs.  *converged (may be NULL):
 * 1 when every member's maximum relative eigenvalue change is below
 * opt.tol.  Synchronises the stream once. */
PASM_API pasm_status pasm_batch_iterate(pasm_batch* b, int* converged);
PASM_API pasm_status pasm_batch_restart(pasm_batch* b);
PASM_API pasm_status pasm_batch_solve(pasm_batch* b, int* iterations);

/* Eigenvalues (k) and, if U != NULL, eigenvectors (k blocks of ldu doubles,
 * host memory, interior nodes x fastest) of member i (0 <= i < n, in the
 * order given at set-up). */
PASM_API pasm_status pasm_batch_eigenpairs(const pasm_batch* b, int member, double* lambda, double* U,
                                           size_t ldu);
/* Replace member i's state (host memory, layout as above); non-finite
 * values are refused (PASM_E_INVALID) as in pasm_set_state. */
PASM_API pasm_status pasm_batch_set_state(pasm_batch* b, int member, const double* lambda, const double* U,
                                          size_t ldu);
PASM_API size_t pasm_batch_num_dofs(const pasm_batch* b, int member);
PASM_API int pasm_batch_num_levels(const pasm_batch* b);

/* 1 (default): replay the recorded graph of one iteration; 0: launch the
 * kernels one by one (the same kernels, same order). */
PASM_API pasm_status pasm_batch_use_graph(pasm_batch* b, int enable);

/* Smoothing tile height per level (levels 1 .. pasm_batch_num_levels()-1;
 * entry 0 unused): 0 = one launch per smoothing step, 2/4/8 = fused phase
 * with 4*rows LDS rows per workgroup.  pasm_batch_tuning reports the choice
 * and, if times_ms != NULL, the measured time of each candidate
 * (times_ms[level][4] for 0, 2, 4, 8; negative if not applicable).
 * pasm_batch_set_tiles overrides the choice (invalid entries: PASM_E_INVALID). */
PASM_API pasm_status pasm_batch_tuning(const pasm_batch* b, int* rows, double* times_ms);
PASM_API pasm_status pasm_batch_set_tiles(pasm_batch* b, const int* rows);

/* HIP-event timing of the finest batched level's smoothing phases inside
 * subsequent iterations (kernel 0 only), as pasm_profile / pasm_profile_read. */
PASM_API pasm_status pasm_batch_profile(pasm_batch* b, int kernel, int enable);
PASM_API pasm_status pasm_batch_profile_read(pasm_batch* b, int kernel, long* launches, double* total_ms,
                                             double* bytes_per_launch);

PASM_API pasm_status pasm_batch_destroy(pasm_batch* b);
/* Last failure on b; with b == NULL, of the last failed pasm_batch_setup on
 * the calling thread. */
PASM_API const char* pasm_batch_last_error(const pasm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* PASM_H */
