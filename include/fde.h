/*
 * fde.h -- C ABI of the MI355X (gfx950) hot path of ADMM for box-constrained
 * optimal control under a time-dependent 2-D fractional-diffusion constraint.
 *
 * Method: Pougkakiotis, Pearson, Leveque, Gondzio, "Fast Solution Methods for
 * Convex Fractional Differential Equation Optimization".  The discretised
 * problem is the QP of Sec. 3 (eq. (3.3)) with the constraint of Sec. 4:
 *
 *     min  1/2 (y - yhat)^T J1 (y - yhat) + 1/2 u^T J2 u,     J2 = gamma J1
 *     s.t. D y + s u = g,   ya <= y <= yb,   ua <= u <= ub,
 *
 *     D = C_t (x) I - I (x) (L_x (+) L_y)                        (eq. (4.9))
 *
 * with implicit Euler in time (the Grünwald matrix of eq. (4.5) at order 1),
 * shifted Grünwald two-sided operators L_a = (c_a/h^a)(diag(d+) G_a +
 * diag(d-) G_a^T) in space (eqs. (4.6)-(4.7)), c_a = -1/(2 cos(a pi/2)).
 *
 * Conventions for every entry point:
 *   - Fields are contiguous float64 arrays of nx*ny*nt values, layout
 *     [nt][ny][nx] (x fastest); index (k*ny + j)*nx + i is the node
 *     (x_i, y_j, t_k) = ((i+1) hx, (j+1) hy, (k+1) ht), hx = 1/(nx+1),
 *     hy = 1/(ny+1), ht = T/nt.
 *   - Field pointers are DEVICE pointers owned by the caller (e.g. a torch
 *     tensor's data_ptr()); pointers marked (host) are host memory.  The
 *     library never frees caller memory.  A context owns only its O(n)
 *     tables and its workspace (about 12 fields plus a half spectrum).
 *     Device fields must be 16-byte aligned (the kernels move adjacent
 *     pairs of doubles; any hipMalloc or torch allocation is); a misaligned
 *     field is rejected with FDE_EINVAL before any device work.
 *   - Work is enqueued on the context's stream.  Calls returning host
 *     results (iteration counts, stats) synchronise that stream; the others
 *     are asynchronous.  A context must be used by one host thread and one
 *     stream at a time.
 *   - Return value: FDE_OK, a positive warning (FDE_ENOTCONV: the iteration
 *     limit was reached, outputs hold the last iterate) or a negative error.
 *     After an error the outputs are unspecified and fde_last_error() gives
 *     a message (thread-local).  Parameter errors are detected before any
 *     device work is enqueued.
 */
#ifndef FDE_H
#define FDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fde_ctx fde_ctx;

typedef enum {
  FDE_OK = 0,
  FDE_ENOTCONV = 1,      /* warning: iteration limit reached                  */
  FDE_EINVAL = -1,       /* invalid parameter or unsupported size             */
  FDE_ENOMEM = -2,       /* device allocation failed                           */
  FDE_EHIP = -3,         /* HIP runtime error (no device, launch failure ...)  */
  FDE_ENONFINITE = -4    /* NaN/Inf met in a residual                          */
} fde_status;

/* Problem description (Sec. 4, eqs. (4.2)-(4.10)). */
typedef struct {
  int32_t nx, ny, nt;     /* interior nodes per axis; each 2^a 3^b with b <= 1,
                             4 <= n <= 1024, or one of 50, 80, 100, 160 (the
                             paper's grids of Sec. 6.2; radix-5 transforms in
                             the preconditioner, a longer circulant embedding
                             in the operator)                                   */
  double T;               /* final time (> 0); ht = T / nt                      */
  double alpha, beta;     /* fractional orders along x and y, each in (1, 2]    */
  const double* dplus;    /* (host) ny*nx coefficient field d+, row j = y_j;
                             NULL means d+ = 1.  Copied at create time.        */
  const double* dminus;   /* (host) same for d-                                 */
  double ctrl_sign;       /* s = +1: D y + u = g (eq. (4.8)); -1: D y - u = g    */
  int32_t psi_scaling;    /* 1: scale the constraints by psi = min{ht^alpha_t,
                             hx^alpha, hy^beta} and the copies of u by psi
                             (Sec. 5, 6.1);
                             2: scale the FDE constraint only (u copies
                             unscaled); 0: unscaled                             */
  int32_t obj_weights;    /* 0: J1 = I; 1: trapezoidal, 1/2 on the last time
                             block (eq. (4.10))                                 */
  int32_t precond_fp32;   /* 1: run the circulant preconditioner in float32
                             (operator, residuals, dots, ADMM stay float64)     */
  double alpha_t;         /* order of the Caputo time derivative, in (0, 1]:
                             the non-shifted Grünwald matrix of eq. (4.5),
                             (1/ht^alpha_t) lower-triangular Toeplitz of the
                             weights g_k(alpha_t); 1 (and 0, read as 1) is
                             implicit Euler.  psi then uses ht^alpha_t.        */
} fde_problem;

/* ADMM and Krylov settings (Algorithm 1; Sec. 6.1). */
typedef struct {
  double gamma;           /* > 0, J2 = gamma J1                                 */
  double delta;           /* > 0, the augmented term is 1/(2 delta)||.||^2      */
  double rho;             /* dual step, in (0, (1 + sqrt 5)/2)                   */
  double ya, yb, ua, ub;  /* bounds, +-INFINITY allowed, ya <= yb, ua <= ub     */
  double krylov_tol;      /* PCG stops when ||r||_2 <= tol ||b||_2              */
  int32_t krylov_maxit;   /* > 0                                                */
  int32_t tol_mode;       /* 0: fixed krylov_tol; 1: the paper's dynamic rule
                             0.05 max{min{three residuals}, 1e-4}              */
  double admm_tol;        /* stop when max of the three inf-norm residuals
                             <= admm_tol (0: run exactly admm_maxit iterations) */
  int32_t admm_maxit;     /* > 0                                                */
  int32_t pcg_cold_start; /* 0: each x-step's PCG starts from the previous y;
                             1: from zero (MATLAB pcg's default, Sec. 6.1)     */
  int32_t prox;           /* 0: Algorithm 1.  1: the generalized ADMM of
                             Sec. 3.3.2 (Algorithm 2): the x-step adds
                             1/2|y - y^j|^2_{R_y} + 1/2|u - u^j|^2_{R_u} with
                             R_y = c_y I - J1, R_u = c_u I - J2, so its (1,1)
                             and (2,2) blocks are the scaled identities
                             rho (c_y + e_y^2/delta) I, rho (c_u + e_u^2/delta) I
                             and the preconditioner's scalars are exact.
                             Needs rho in (0, 1].                            */
  double prox_cy;         /* c_y: 0 selects max diag J1 = 1 (R_y semi-definite,
                             zero off the last time block); else >= 1        */
  double prox_cu;         /* c_u: 0 selects gamma; else >= gamma              */
  int32_t precond_kind;   /* 0: S~ of eq. (3.10), a I + C^* C / mbar_p;
                             1: the matching approximation S^ of eq. (3.11)
                             with the same blocks, (C^* + c)(C + c) / mbar_p,
                             c = (a mbar_p)^{1/2} (C the 3-level T. Chan
                             circulant of B, eq. (5.2));
                             2: S~ with a diagonal scaling for variable
                             coefficients (the remark closing Sec. 4 points to
                             diagonal-times-structured forms): the inverse is
                             Delta S~^{-1} Delta, Delta = (s0 / diag S)^{1/2}
                             with the exact diagonal of S (eq. (3.9)) and s0
                             its mean; PCG x-step only (krylov_solver 0) */
  int32_t krylov_solver;  /* x-step solver: 0: PCG on the normal equations
                             (3.9) with S~ (or S^); 1: MINRES on the merged
                             saddle-point system (3.8) with the block-diagonal
                             K~ of eq. (3.12) (Sec. 3.3.1), see fde_minres;
                             krylov_tol, krylov_maxit, tol_mode and
                             pcg_cold_start apply to either               */
} fde_admm_params;

typedef struct {
  int32_t admm_iters;     /* iterations performed                                */
  int32_t pcg_total;      /* Krylov (PCG, or MINRES with krylov_solver = 1)
                             iterations summed over all x-steps              */
  int32_t pcg_last;       /* PCG iterations of the last x-step                   */
  int32_t pcg_max;        /* largest PCG count of one x-step                     */
  double r_p;             /* ||B y + k_u u - psi g||_inf  (scaled constraint)     */
  double r_y;             /* ||y - z_y||_inf                                      */
  double r_u;             /* ||u - z_u||_inf                                      */
  double J;               /* objective 1/2 (y-yhat)^T J1 (y-yhat) + 1/2 u^T J2 u at
                             the returned iterate                                */
  double t_total;         /* seconds, wall clock of the solve                    */
  double t_pcg;           /* seconds spent in the Krylov solves (host clock)     */
  double dual_inf;        /* dual infeasibility of the returned iterate (reported,
                             not a stopping test; Sec. 6.1):
                             max(||J1 (y - yhat) + D^T lambda + mu_y||_inf,
                                 ||gamma J1 u + ctrl_sign lambda + mu_u||_inf)
                             with lambda = psi p, mu_y = w_y, mu_u = e_u w_u     */
  /* GPU time per phase of Algorithm 1, seconds summed over the iterations
   * (HIP events on the context stream at the phase boundaries; host waits
   * between the Krylov chunks count in t_krylov):                           */
  double t_rhs;           /* right-hand side of the x-step (step 1, with the
                             B^T apply of eq. (3.9)'s right-hand side)         */
  double t_krylov;        /* the x-step's Krylov solve (step 2)                  */
  double t_update;        /* B y, recovery of p and u, box projection, dual
                             updates and residual maxima (steps 3-6)            */
  int32_t batched;        /* 1: the Krylov iterations ran as batched launches
                             (fde_batch_solve, lockstep mode); 0 otherwise     */
} fde_admm_stats;

/* Check a problem/parameter pair without touching the GPU.  FDE_OK or
 * FDE_EINVAL (message in fde_last_error()). */
fde_status fde_validate(const fde_problem* prob, const fde_admm_params* prm);

/* Host-only setup tables, for inspection and CPU tests (no GPU use).
 * Writes (host, caller-allocated):
 *   scal[8]         = {psi, hx, hy, ht, a, 1/mbar_p, e_u, k_u}
 *   lam_x[2*nx], lam_y[2*ny], lam_t[2*nt]  interleaved (re, im) T. Chan
 *                     eigenvalues, lambda_k = sum_m c_m exp(-2 pi i k m / n)
 *                     (Sec. 5, closed form under eq. (5.1) and Thm 2.2);
 *   gx[nx+1], gy[ny+1] Grünwald weights of orders alpha, beta (Sec. 4).
 * Any output pointer may be NULL. */
fde_status fde_host_tables(const fde_problem* prob, const fde_admm_params* prm, double* scal,
                           double* lam_x, double* lam_y, double* lam_t, double* gx, double* gy);

/* Host-only: the diagonal scaling Delta of precond_kind 2 (whatever prm's
 * precond_kind), written to delta (host, caller-allocated, nx*ny*nt values,
 * field layout).  diag S = M_y + psi^2 (sum of the squared entries of the
 * column of D, each over M_p of its row's time level) (eq. (3.9), (4.9)).
 * FDE_EINVAL on invalid arguments.  O(nx^2 ny + ny^2 nx) host work. */
fde_status fde_host_diag_scaling(const fde_problem* prob, const fde_admm_params* prm, double* delta);

/* Create a context on the current HIP device.  `stream` is a hipStream_t
 * (NULL = default stream).  Validates, builds the weights, embedding and
 * T. Chan eigen tables and twiddles on the host (FP64), copies them to the
 * device and allocates the workspace.  *out receives the context.  The PCG
 * iteration is replayed from a HIP graph captured on a private stream
 * (environment FDE_NO_GRAPH=1 at create time: plain kernel launches).  The
 * column tiles start at the widest variant (FDE_TILES=a,b,c at create time
 * fixes the three variants; see fde_autotune).  Coefficient fields that vary
 * along x only make every y-line constant-coefficient: the y-passes then use
 * per-column multipliers, two transforms per column pair instead of three
 * (FDE_YCOL=0 at create time keeps the general variable-coefficient y-pass).
 * The PCG convergence test rides in the preconditioner's y-forward pass, or
 * runs as its own one-block launch on large grids where every block's sum of
 * the residual partials would cost more (FDE_CONV_SEPARATE=1 / 0 forces
 * either; results are identical). */
fde_status fde_create(const fde_problem* prob, const fde_admm_params* prm, void* stream,
                      fde_ctx** out);
fde_status fde_destroy(fde_ctx* ctx);

/* Replace the ADMM/Krylov settings of a context (same validation as create;
 * gamma, delta, rho enter the preconditioner tables, which are rebuilt). */
fde_status fde_set_params(fde_ctx* ctx, const fde_admm_params* prm);

/* Per-point box bounds (Sec. 3 states the box constraints with bounds that
 * are functions of space and time; here one value per grid point): ya, yb, ua, ub are device fields of the grid's
 * size, [nt][ny][nx], +-INFINITY allowed; NULL keeps the scalar bound of
 * fde_admm_params for that side.  The fields are checked (lower <= upper at
 * every point, no NaN; FDE_EINVAL otherwise, leaving the previous bounds) and
 * copied into the context (the caller may free them afterwards); later
 * fde_set_params calls keep them and are checked against them.  All NULL
 * restores scalar bounds.  Used by fde_admm_solve (not by fde_batch).
 * Synchronises the stream. */
fde_status fde_set_bounds(fde_ctx* ctx, const double* ya, const double* yb, const double* ua, const double* ub);

/* y = D x (transpose = 0) or y = D^T x (transpose = 1), the unscaled
 * constraint matrix of eq. (4.9), by circulant embedding and FFT (Table 1).
 * x and y are device fields and must not alias. */
fde_status fde_apply_A(fde_ctx* ctx, const double* x, double* y, int transpose);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * fde_apply_A with its intermediate fields in a fixed static device array
 * (32 MiB = 2^22 doubles per GPU, held until the process ends) instead of the
 * context's workspace.  Calls no hipMalloc/hipFree.  Grids needing more than
 * 2^22 doubles of workspace (N points with implicit Euler, 2N with a
 * fractional time order) are rejected with FDE_EINVAL; the context's device
 * must be current (FDE_EINVAL otherwise).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams, or different host
 * threads) race and must be ordered by the caller.  Nothing in the array needs
 * to start at zero (each call writes it before reading).  Same arguments and
 * results as fde_apply_A. */
fde_status fde_apply_A_noalloc(fde_ctx* ctx, const double* x, double* y, int transpose);

/* y = S x with S = M_y + B^T M_p^{-1} B the normal-equations matrix of the
 * ADMM x-step (eq. (3.9), in the psi-scaled form B = psi D).  No aliasing. */
fde_status fde_apply_S(fde_ctx* ctx, const double* x, double* y);

/* z = S~^{-1} r, the Schur-complement approximation of eq. (3.10) built
 * from the 3-level T. Chan circulant of eq. (5.2): 3-D real FFT, division by
 * the eigenvalues a + |psi (lt - ly - lx)|^2 / mbar_p, inverse FFT.  Runs in
 * float32 when the problem asked for it.  r and z may alias. */
fde_status fde_precond(fde_ctx* ctx, const double* r, double* z);

/* Solve S x = b by PCG with S~ (Sec. 6.1 uses PCG on eq. (3.9)), Fletcher-
 * Reeves beta, stopping when the recursively updated ||r||_2 <= krylov_tol
 * ||b||_2.  x holds the initial guess on entry and the solution on exit.
 * *iters (host) receives the iteration count, *relres (host) the final
 * relative residual.  Synchronises the stream.  FDE_ENOTCONV after
 * krylov_maxit iterations. */
fde_status fde_krylov(fde_ctx* ctx, const double* b, double* x, int* iters, double* relres);

/* Solve the merged x-step system (3.8) in the scaled variables,
 *     [ M_y   0     B^T          ] [y]   [b_y]
 *     [ 0     M_u   k_u I        ] [u] = [b_u]      (B = psi D, k_u = psi s),
 *     [ B     k_u I -(delta/rho) I] [p]   [b_p]
 * by preconditioned MINRES (Sec. 3.3.1) with the block-diagonal K~ of
 * eq. (3.12): M_y and M_u exactly (they are diagonal) and, for the p block,
 * the circulant approximation of its Schur complement M_p + B M_y^{-1} B^T,
 * which with the scalar blocks a, mbar_p is (mbar_p / a) S~ (S^ when
 * precond_kind = 1).  Stops when the K~^{-1}-norm of the residual is at most
 * krylov_tol times that of b, or after krylov_maxit iterations
 * (FDE_ENOTCONV).  (y, u, p) hold the initial guess on entry and the solution
 * on exit; b_* are device fields of the grid's size, none aliasing an unknown.
 * *iters and *relres (host) receive the count and the final relative residual.
 * The workspace (22 fields) is allocated at fde_create / fde_set_params when
 * krylov_solver = 1, else by the first call.  Synchronises the stream. */
fde_status fde_minres(fde_ctx* ctx, const double* b_y, const double* b_u, const double* b_p, double* y, double* u,
                      double* p, int* iters, double* relres);

/* Algorithm 1 (2-block ADMM, Sec. 3.1) with the merged x-step: the normal
 * equations solved by fde_krylov's PCG (or, with krylov_solver = 1, the
 * merged system by fde_minres's MINRES), the z-step as the box projection,
 * the dual updates, and the stopping test of Sec. 6.1 on the scaled primal
 * residual and the two copy residuals.  prox = 1 runs Algorithm 2 instead
 * (Sec. 3.3.2).  yhat: desired state; g: FDE right-
 * hand side (NULL = 0).  y, u, zy, zu, p, wy, wu are the ADMM iterates
 * (p the scaled multiplier of B y + k_u u = psi g, wy/wu those of the copy
 * constraints): read as the starting point (all zeros for a cold start; a
 * previous call's outputs to resume) and overwritten with the last iterate.
 * *stats (host, may be NULL) receives counts and residuals.  Synchronises. */
fde_status fde_admm_solve(fde_ctx* ctx, const double* yhat, const double* g, double* y, double* u,
                          double* zy, double* zu, double* p, double* wy, double* wu,
                          fde_admm_stats* stats);

/* Gradients of the optimal value J*(yhat, alpha, beta) at an ADMM solution
 * (envelope theorem on the Lagrangian of eq. (3.5)):
 *   dJ/dyhat = -J1 (y - yhat)                       -> dyhat (device field, may be NULL)
 *   dJ/dalpha = lambda^T (dD/dalpha) y, dJ/dbeta likewise -> dab[2] (host)
 * with dD/dalpha = -dL_x/dalpha built from the derivative of the Grünwald
 * recurrence (and of c_a h^-a).  lambda, the multiplier of D y + s u = g:
 *   adjoint_solve = 1: from the adjoint equation D^T lambda = -J1 (y - yhat)
 *     - wy, solved by backward time stepping (the transposed time matrix is
 *     upper triangular: bidiagonal for implicit Euler, the Caputo weights of
 *     eq. (4.5) otherwise, whose history enters each step's right-hand side);
 *     each step is a 2-D transposed-Toeplitz solve (reversed weights) by
 *     BiCGSTAB preconditioned with the inverse of the transposed 2-D T. Chan
 *     circulant, to 1e-13 relative residual;
 *   adjoint_solve = 0: lambda = psi p from the ADMM iterate.
 * wy may be NULL when adjoint_solve = 0.  lambda_out (device field, may be
 * NULL) receives lambda.  Uses the context workspace.  Synchronises.
 * FDE_ENOTCONV if a time step's solve does not converge in 500 iterations. */
fde_status fde_grad(fde_ctx* ctx, const double* yhat, const double* y, const double* p,
                    const double* wy, int adjoint_solve, double* dyhat, double* dab,
                    double* lambda_out);

/* Measurement hook for the roofline figure: launch one internal pass of the
 * PCG iteration `reps` times back to back on the context stream between two
 * HIP events and report the mean duration per launch (*us, host) and the
 * algorithmic HBM bytes one launch must move (*bytes, host: every field the
 * pass reads or writes counted once).  The field passes alternate between two
 * disjoint sets of workspace fields, so a launch finds its inputs about as
 * warm in the last-level cache as inside an iteration.  The pass runs on the
 * context's workspace (contents are overwritten).  which:
 *   0 x-pass of B (time difference fused)   1 y-pass of B (scaled by M_p^-1)
 *   2 x-pass of B^T                          3 y-pass of B^T (+ M_y v, (v, Sv))
 *   4 preconditioner x-forward (fused alpha, r -= alpha q, x += alpha p, (r, r))
 *   5 preconditioner y-forward (fused convergence test)
 *   6 t-forward/divide/t-inverse (fused (r, z) partials from the spectrum)
 *   7 preconditioner y-inverse (fused (r, z) and beta)
 *   8 x-inverse writing the direction p = z + beta p
 * Synchronises the stream. */
fde_status fde_time_pass(fde_ctx* ctx, int which, int reps, double* us, double* bytes);

/* In-solve timing of the nine passes of the PCG iteration (the O(N log N)
 * applies of Table 1 and the preconditioner of eq. (3.10)), for the roofline
 * figure: with enable = 1, until disabled, every PCG iteration of fde_krylov
 * and fde_admm_solve on this context runs as plain launches (no graph) with a
 * pair of HIP events bound to each pass's own dispatch (hipExtLaunchKernel),
 * and the kernel durations accumulate per pass (cleared by enable = 1).
 * Results and iteration counts are those of the graph launches.  Implicit
 * Euler only (FDE_EINVAL for another time order).  Synchronises the stream. */
fde_status fde_pass_timing(fde_ctx* ctx, int enable);

/* Accumulated in-solve pass figures, pass order as in fde_time_pass (host
 * arrays of 9, each may be NULL): us = mean kernel duration per launch
 * (microseconds), launches = dispatches timed (iterations enqueued after the
 * solve's convergence return at once and are included, as in a kernel trace),
 * bytes = algorithmic bytes of one launch (as fde_time_pass). */
fde_status fde_pass_stats(fde_ctx* ctx, double* us, int32_t* launches, double* bytes);

/* Autotuner of the FFT column tiles: times the widest, half and quarter
 * column-tile variants of the y-direction Toeplitz passes, the y-direction
 * preconditioner passes and the t-direction pass on this context's grid
 * (HIP events, workspace overwritten) and keeps the fastest.  Choices are
 * cached per (nx, ny, nt, coefficient kind, precision) for the process and,
 * when the environment names a file in FDE_TUNE_DB, appended to / read from
 * it.  choices (host, 3 ints, may be NULL): column pairs per block of the
 * y-pass, and the variant indices of the two preconditioner passes.  The
 * results of every variant are identical up to the order of the partial
 * sums of the fused dot products.  Synchronises the stream. */
fde_status fde_autotune(fde_ctx* ctx, int32_t* choices);

/* Batched form: many independent problems of uneven sizes solved together.
 * Each instance has its own context (tables, workspace, graph-captured PCG
 * iteration, tiles chosen by fde_autotune) on its own stream (default
 * priority); one host thread drives
 * all of them as resumable state machines, polling a HIP event per instance
 * and enqueueing its next phase as soon as the previous one has finished,
 * so the instances' kernels overlap on the GPU and no instance waits for
 * another's host synchronisation (concurrent = 1).  concurrent = 0 runs the
 * same solves one after the other (the sequential reference).
 * concurrent = 2 (lockstep): the PCG iterations of all instances run as
 * batched launches, one launch per pass kind and position covering every
 * instance's blocks (each instance keeps its own tables, block decomposition
 * and done flag), the other ADMM phases as each instance's own launches; the
 * instances advance one ADMM iteration at a time together.  Instances whose
 * x-step has no batched form (MINRES, a fractional time order, lengths
 * without batched pass variants) make the call run the concurrent mode
 * instead.  Instances whose x-step has converged leave the batched launches
 * and go on with their own phases on their own streams while the others
 * iterate.  Results equal the single solves' bit for bit.
 * Arrays indexed by instance: yhat[i], g[i] (g may be NULL, or g[i] NULL),
 * and the iterate fields y[i] .. wu[i] (device fields of instance i's size,
 * read as the starting point, overwritten).  The caller makes the inputs
 * ready before the call (e.g. synchronises the stream that produced them);
 * the call synchronises every instance stream before returning.
 * stats[i], status[i] (host, may be NULL) receive per-instance results; the
 * return value is the first negative instance status, else FDE_ENOTCONV if
 * any instance hit its iteration limit, else FDE_OK. */
typedef struct fde_batch fde_batch;
fde_status fde_batch_create(int count, const fde_problem* probs, const fde_admm_params* prms,
                            fde_batch** out);
fde_status fde_batch_destroy(fde_batch* b);
fde_status fde_batch_solve(fde_batch* b, int concurrent, const double* const* yhat,
                           const double* const* g, double* const* y, double* const* u,
                           double* const* zy, double* const* zu, double* const* p,
                           double* const* wy, double* const* wu, fde_admm_stats* stats,
                           int32_t* status);

/* Last error message of the calling thread ("" if none). */
const char* fde_last_error(void);

/* Library version string. */
const char* fde_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FDE_H */
