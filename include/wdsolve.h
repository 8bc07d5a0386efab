/*
 * wdsolve -- Jacobi-preconditioned block BiCGGR for the O(a)-improved
 * (clover) Wilson-Dirac system A X = B with L right-hand sides, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Sec. 2, eq. (1)): A is an N x N complex sparse
 * non-Hermitian matrix with N = Lx*Ly*Lz*Lt*3*4; X and B are N x L.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ---------------------------------------------------------------------------
 * Lattice: extents Lx, Ly, Lz, Lt (each >= 2), V = Lx*Ly*Lz*Lt sites,
 *   site s = x + Lx*(y + Ly*(z + Lz*t)); directions mu = 0..3 are x, y, z, t.
 *
 * Gauge links (input of wd_set_links): complex128 (interleaved re, im)
 *   U[mu][s][a][b], i.e. 4*V*9 complex numbers; U_mu(x) is the SU(3) link
 *   from x to x + mu-hat.
 *
 * Block vectors (X, B, Y, R, Z below): N x L complex128 matrices stored
 *   column by column; within column i the row index is n = k*V + s, where
 *   k = 3*spin + colour (0..11) and s is the site.  Element (n, i) is at
 *   complex offset i*N + n.  Spin refers to the chiral gamma basis below.
 *   A context can be switched to the tiled layout instead (wd_set_layout),
 *   with n = (s/64)*768 + k*64 + s%64.
 *
 * Operator (the paper leaves the matrix to its companion paper; this is the
 *   standard hopping-parameter form):
 *     (A psi)(x) = T(x) psi(x)
 *        - kappa sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *     T(x) = 1 - kappa c_SW sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
 *     sigma_{mu nu} = (i/2)[g_mu, g_nu],
 *     F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag)/(8i), Q = sum of the
 *     four counter-clockwise plaquette leaves at x (no trace subtraction).
 *   Gamma matrices (chiral basis, s_k Pauli): g_k = [[0, -i s_k], [i s_k, 0]]
 *   for k = x, y, z and g_t = [[0, 1], [1, 0]]; gamma5 = diag(1, 1, -1, -1).
 *   Boundary conditions: periodic, or antiperiodic in t (bc_t = 1).
 *
 * Ownership and streams: every device pointer passed in is owned by the
 *   caller and must stay valid until the call returns; the library owns its
 *   gauge field, clover and workspace.  All device work is issued on the
 *   HIP stream given to wd_create and every function returns only after its
 *   results are complete.  A context is not thread-safe.
 *
 * Errors: 0 is success; negative values are API or runtime errors (nothing
 *   is modified on argument errors); positive values are numerical outcomes
 *   of the solver, which still returns an iterate: the last one when
 *   max_iter is reached, otherwise the run's recovery point or, after a
 *   breakdown, the iterate it stopped on.  No C++ exception or abort crosses
 *   this interface.
 */
#ifndef WDSOLVE_H
#define WDSOLVE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wd_ctx wd_ctx;

/* return codes */
#define WD_OK 0
#define WD_EINVAL (-1)         /* bad argument: dims, L, null, aliasing, zero column, unknown option */
#define WD_ENOMEM (-2)         /* device allocation failed */
#define WD_EHIP (-3)           /* HIP runtime error */
#define WD_ENAN (-4)           /* non-finite value met in a residual */
#define WD_ESTATE (-5)         /* call out of order (e.g. wd_apply before wd_set_params) */
#define WD_NOT_CONVERGED 1     /* max_iter reached */
#define WD_BREAKDOWN 2         /* singular L x L system (rank loss) or zero step */
#define WD_DIVERGED 3          /* max relative residual above diverge_at */
#define WD_STAGNATED 4         /* best residual not improved for stagnate_window iterations */

/* arithmetic/storage precision of an operator application */
#define WD_F64 0
#define WD_F32 1               /* FP32 storage of links, clover and spinors, FP32 arithmetic */
#define WD_BF16 2              /* BF16 storage, FP32 arithmetic */
/* Jacobi preconditioner only: FP64 iterates and arithmetic with the links and
 * A_D^{-1} stored in FP32 or BF16.  Unlike WD_F32 / WD_BF16, which round the
 * iterates, this M is a fixed linear operator to FP64 accuracy (the Jacobi
 * iteration of a nearby matrix), so block BiCGGR needs no Krylov cycles. */
#define WD_F64_COEF_F32 3
#define WD_F64_COEF_BF16 4

/* preconditioner M of the solver */
#define WD_PRECOND_NONE 0      /* M = I */
#define WD_PRECOND_JACOBI 1    /* j-step Jacobi */
#define WD_PRECOND_LEARNED 2   /* frozen linear gauge-covariant network (wd_set_learned), FP32 */

/* reading of "diagonal part A_D" for the Jacobi preconditioner */
#define WD_JACOBI_BLOCK 0      /* site-block diagonal: A_D = T(x) (12 x 12 per site) */
#define WD_JACOBI_POINT 1      /* point diagonal: A_D = diag(T(x)) */

#define WD_MAX_L 16            /* largest number of right-hand sides */

/* layout of the rows of a block vector (wd_set_layout) */
#define WD_LAYOUT_STANDARD 0   /* n = k*V + s (the default) */
#define WD_LAYOUT_TILED 1      /* n = (s/64)*768 + k*64 + s%64: the 12 spin-colour rows of a
                                  64-site tile of a column are contiguous */

/* Options of bbicggr_solve; zero-initialise and set what is needed. */
typedef struct wd_solve_opts {
    int j;                 /* Jacobi steps per application of M (>= 0); 0 means M = I */
    int precond;           /* WD_PRECOND_*; NONE forces j = 0 in the cost count */
    int prec_inner;        /* WD_F64 / WD_F32 / WD_BF16 / WD_F64_COEF_F32 / WD_F64_COEF_BF16
                              storage of the Jacobi preconditioner; WD_F64 / WD_F32 arithmetic
                              of the learned one */
    int use_x0;            /* 1: X holds the initial guess; 0: start from X = 0 */
    int max_iter;          /* outer iterations per run; <= 0 means 5000 */
    int max_restarts;      /* true-residual restarts; < 0 means 3 */
    int stagnate_window;   /* <= 0 means 200 */
    double diverge_at;     /* <= 0 means 1e2 */
    double* history;       /* optional host buffer: max relative recursive residual per iteration */
    int history_len;       /* its length in doubles */
    double cycle_tol;      /* Krylov cycle length for an inexact (low-precision) M: a cycle ends
                              once it has reduced its starting residual by this factor, or when it
                              stops improving (then X returns to the cycle's best iterate), and the
                              solver restarts from the FP64 true residual.  0: 1e-4 for FP32 and
                              1e-1 for BF16 storage of M (the learned M counts as FP32), no cycles
                              for FP64; < 0: no cycles */
    int no_fallback;       /* 0: when a cycle of an inexact M, or a run with the learned M in any
                              precision, stalls, diverges or breaks down, the solve starts again
                              from X = 0 with the FP64 Jacobi preconditioner of the same j (M = I
                              if j = 0); 1: the solve ends there with that status and X set to
                              the cycle's best iterate or the run's recovery point */
    void* x_snap;          /* optional device buffer of snap_count block vectors of L columns:
                              the iterate X_k is copied into slot i after outer iteration
                              k = (i + 1) * snap_every (counted over all runs of the solve), for
                              training pairs of the learned preconditioner (wd_learned_pairs) */
    int snap_count;        /* slots in x_snap (0: no snapshots) */
    int snap_every;        /* iterations between snapshots (>= 1 when snap_count > 0) */
    double* gap_history;   /* optional host buffer of history_len doubles: per outer iteration, the
                              largest per-column ||r_k - (b - A x_k)|| / ||b|| between the recursive
                              and the true residual (a diagnostic: one more application of A per
                              iteration) */
    double* cond_history;  /* optional host buffer of history_len doubles: per outer iteration, the
                              larger condition estimate (largest over smallest LU pivot modulus) of
                              the L x L matrices Rt_0^H V_k and Rt_0^H R_k (block BiCGSTAB: Rt_0^H V_k) */
    double cond_limit;     /* > 0: a condition estimate above this ends the run as a breakdown (rank
                              loss of the block); 0 or less: only singular systems do */
    int no_split;          /* block BiCGGR, FP64 runs: 0 (default) -- when a run of L > 1 columns breaks
                              down, diverges or stagnates, X returns to its recovery point (the last
                              iterate that had cut the largest residual tenfold) and the two halves
                              of the block are solved as blocks of their own, recursively: the remedy
                              of Sec. 3.3, a smaller L; 1 -- no splitting (a failed run of L = 1
                              columns, or with splitting off, restarts from its recovery point while
                              max_restarts allows) */
} wd_solve_opts;

/* Results of bbicggr_solve. */
typedef struct wd_solve_info {
    int status;                        /* the code the call returned: WD_OK, a positive outcome code, or a
                                          negative error met during the solve (e.g. WD_ENAN, WD_EHIP); the
                                          other fields then describe the work done until then */
    int iterations;                    /* outer iterations of the last run */
    int total_iterations;              /* over all restarts */
    int restarts;                      /* true-residual restarts made */
    int cycles;                        /* Krylov cycles run (1 without low-precision cycling) */
    int fallback;                      /* 1 if the FP64 fallback of an inexact M was taken */
    int snapshots;                     /* iterates copied into opts->x_snap */
    long long mvm_paper;               /* per column, counted as in Table 1: 2(j+1)k + 1 per run */
    long long mvm_actual;              /* per column: hopping-term applications actually made */
    double seconds;                    /* wall time of the solve (device synchronised) */
    double bytes_alg;                  /* algorithmic HBM bytes of every kernel launched by the solve */
    double true_residual[WD_MAX_L];    /* ||b - A x|| / ||b|| per column, FP64 */
    double recursive_residual[WD_MAX_L];
    double cond_max;                   /* largest condition estimate of the L x L systems over all runs */
    int splits;                        /* block splits made after failed runs */
    int min_block;                     /* smallest block width solved */
} wd_solve_info;

/* ---------------------------------------------------------------------------
 * Setup
 * ------------------------------------------------------------------------- */

/* Create a context for an Lx x Ly x Lz x Lt lattice (dims[0..3] = Lx, Ly,
 * Lz, Lt, each >= 2) with up to max_L right-hand sides (1..WD_MAX_L).
 * bc_t: 0 periodic, 1 antiperiodic in t.  hip_stream: a hipStream_t (NULL
 * for the default stream).  Workspace for max_L columns is allocated here.
 * The volume may not exceed 2^28 sites.
 * Errors: WD_EINVAL, WD_ENOMEM, WD_EHIP. */
int wd_create(wd_ctx** out, const int dims[4], int bc_t, int max_L, void* hip_stream);

/* Release the context and all library-owned device memory. */
int wd_destroy(wd_ctx* ctx);

/* Load the gauge field U[mu][s][a][b] (complex128, layout above); U is a
 * host pointer when on_device == 0, a device pointer otherwise.  The links
 * are copied; the caller's buffer is not kept. */
int wd_set_links(wd_ctx* ctx, const double* U, int on_device);

/* Set kappa and c_SW and build, on the GPU, the clover field strength, the
 * site matrices T(x) = T_+ (+) T_- (two 6 x 6 Hermitian chiral blocks) and
 * their inverses in FP64, plus FP32 and BF16 copies for the low-precision
 * preconditioner.  jacobi_kind: WD_JACOBI_BLOCK or WD_JACOBI_POINT (the
 * reading of A_D in Sec. 2's Jacobi preconditioner).  Needs wd_set_links. */
int wd_set_params(wd_ctx* ctx, double kappa, double csw, int jacobi_kind);

/* Copy the site matrices to host memory: which = 0 gives T, 1 gives T^{-1}.
 * out receives V*2*36 complex128: [s][chirality c][row][col] of the 6 x 6
 * block acting on spins (2c, 2c+1) x colours, row/col index 3*spin' + colour
 * with spin' = spin - 2c. */
int wd_get_clover(wd_ctx* ctx, int which, double* out_host);

/* Select the row layout of every block vector this context's entry points read
 * or write: WD_LAYOUT_STANDARD (the default) or WD_LAYOUT_TILED, in which the
 * twelve spin-colour rows of 64 consecutive sites of a column form one
 * contiguous 12 KB run.  The tiled layout is a memory layout of the same N x L
 * matrices (Sec. 2, eq. (1)): within a column it permutes the rows, so block
 * products and norms are unchanged, and the stencil kernels of the operator and
 * the Jacobi preconditioner touch one memory page per tile and column instead of
 * twelve (measured about 9 % faster at 32^3 x 64, L = 12).  bbicggr_solve and
 * bbicgstab_solve use it internally for a context in the standard layout when
 * the lattice allows it: B and X are copied into the tiled layout when the solve
 * starts, X back when it ends and each snapshot (opts->x_snap) as it is taken
 * (two N x max_L blocks of device memory, allocated on first use; without them
 * the solve keeps the standard layout).  The tiled layout needs V to be a
 * multiple of 64 and at most 22369621 sites; every entry point that takes block
 * vectors, the learned preconditioner's included, follows the selected layout.
 * Errors: WD_EINVAL (unknown layout, lattice not divisible into tiles). */
int wd_set_layout(wd_ctx* ctx, int layout);

/* ---------------------------------------------------------------------------
 * The hot path
 * ------------------------------------------------------------------------- */

/* Y = A X for L columns (1 <= L <= max_L).  X and Y are device pointers to
 * N x L block vectors and must not overlap.  prec selects the storage and
 * arithmetic precision of the application (WD_F64 for results at full
 * accuracy; WD_F32 / WD_BF16 round X, the links and the clover to that
 * format and accumulate in FP32; Y is always written in FP64). */
int wd_apply(wd_ctx* ctx, const void* X, void* Y, int L, int prec);

/* Z = M R with M the j-step Jacobi preconditioner of Sec. 2 (the display
 * after the algorithm box) with initial guess G_0 = 0:
 *   Z = sum_{i=0}^{j-1} (I - A_D^{-1} A)^i A_D^{-1} R  (j >= 1),  Z = R (j = 0),
 * evaluated as j sweeps Z_{i+1} = Z_i + A_D^{-1}(R - A Z_i).  prec selects the
 * storage of links, clover and the iterates (WD_F64, or WD_F32 / WD_BF16 with
 * FP32 accumulation), or FP64 iterates with FP32 / BF16 links and A_D^{-1}
 * (WD_F64_COEF_F32 / WD_F64_COEF_BF16); R and Z are FP64 device block vectors
 * and must not overlap. */
int jacobi_precond(wd_ctx* ctx, const void* R, void* Z, int L, int j, int prec);

/* Solve A X = B with preconditioned block BiCGGR (Sec. 2, algorithm box)
 * with Rt_0 = R_0 (Sec. 3.3), stopping when the largest relative recursive
 * residual max_i ||r^(i)|| / ||b^(i)|| falls to tol; the FP64 true residual is
 * then recomputed and the solver restarts from the current X while any
 * column's true residual exceeds tol (up to max_restarts times).  B and X are
 * device block vectors (X in/out); opts may be NULL (defaults, j = 0); info
 * may be NULL and is filled on every return after the arguments were
 * accepted.  Every column of B must be non-zero.  A run that breaks down,
 * diverges or stagnates is continued on the two halves of its block (see
 * no_split): the remedy of Sec. 3.3 for a failed block run, solving again
 * with fewer right-hand sides per block.
 * Returns WD_OK, a positive outcome code, or a negative error. */
int bbicggr_solve(wd_ctx* ctx, const void* B, void* X, int L, double tol,
                  const wd_solve_opts* opts, wd_solve_info* info);

/* Solve A X = B with preconditioned block BiCGSTAB: the published block
 * version of BiCGSTAB (Guennouni, Jbilou and Sadok, ETNA 16, 2003) with M on
 * the right, the method whose recursive residual drifts from the true one,
 * which block BiCGGR avoids (Sec. 1).  Per iteration, with Rt_0 = R_0:
 *   Ph = M P, V = A Ph, (Rt_0^H V) alpha = Rt_0^H R, S = R - V alpha,
 *   Sh = M S, T = A Sh, omega = Tr[T^H S] / Tr[T^H T],
 *   X += Ph alpha + omega Sh, R = S - omega T,
 *   (Rt_0^H V) beta = -Rt_0^H T, P = R + (P - omega V) beta.
 * Same arguments, stopping rule, true-residual restarts and cost count as
 * bbicggr_solve; of the options it takes j, precond (WD_PRECOND_NONE or
 * WD_PRECOND_JACOBI with prec_inner WD_F64), use_x0, max_iter, max_restarts,
 * stagnate_window, diverge_at, history, gap_history, cond_history and
 * cond_limit (no cycles, fallback, snapshots or splitting). */
int bbicgstab_solve(wd_ctx* ctx, const void* B, void* X, int L, double tol,
                    const wd_solve_opts* opts, wd_solve_info* info);

/* Throughput measurement: launch the hopping kernel nrep times back to back
 * on the context stream, then wait.  mode 0 is Y = A X (as wd_apply);
 * mode 1 is one Jacobi sweep Y = A_D^{-1} (R + kappa H X) (the kernel that
 * jacobi_precond runs j - 1 times).  X, R, Y: device block vectors of L
 * columns in FP64; R is ignored for mode 0.  With prec WD_F32 or WD_BF16, X
 * and R are first rounded into the library's low-precision buffers and the
 * low-precision kernel runs on them (mode 0 writes Y in FP64; mode 1 keeps
 * its low-precision output internal and leaves Y untouched).  Mode 1 also
 * takes WD_F64_COEF_F32 / WD_F64_COEF_BF16: the FP64 sweep with the links and
 * A_D^{-1} in that format, writing Y.  With FP64 vectors (WD_F64 and the two
 * coefficient formats) and L >= 3, mode 1 runs the middle sweep of
 * jacobi_precond, which keeps the iterates in a time-diagonal form: X and Y
 * hold u + d in planes 0-5 and u - d in planes 6-11 (u, d: the upper and lower
 * spin pairs), R the standard form. */
int wd_hop_repeat(wd_ctx* ctx, const void* X, const void* R, void* Y, int L, int mode, int prec, int nrep);

/* ---------------------------------------------------------------------------
 * Block kernels of the outer iteration, exposed for testing
 * ------------------------------------------------------------------------- */

/* C = P^H Q (L x L, complex128, row-major: C[i*L + j] = sum_n conj(P[n,i]) Q[n,j])
 * for device block vectors P, Q of L columns; C is a device pointer.  This is
 * the tall-skinny product behind Rt_0^H V_k and Rt_0^H R_k (Sec. 2). */
int wd_block_gram(wd_ctx* ctx, const void* P, const void* Q, int L, void* C);

/* Solve M Z = RHS for L x L complex128 row-major device matrices by LU with
 * partial pivoting in FP64 on the GPU (the alpha and gamma systems of
 * Sec. 2).  Returns WD_BREAKDOWN if a pivot is below 1e-14 max|M| or M is
 * not finite. */
int wd_small_solve(wd_ctx* ctx, const void* M, const void* RHS, int L, void* Z);

/* C = P^H Q as wd_block_gram computes it, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, hosts that
 * forbid hipMalloc): no context, no allocation.  P and Q are device block
 * vectors of N rows and L columns (column-major, N >= 1, 1 <= L <= WD_MAX_L),
 * C an L x L row-major complex128 device matrix; all are owned by the caller.
 * The reduction partials live in a fixed 2.2 MB device array of the library
 * (one per GPU, kept until the process ends, enough for any N); calls that
 * overlap on one GPU share it and race, so issue them one at a time.  Work
 * goes on hip_stream (NULL: the default stream) and the call returns after it
 * is complete.  Errors: WD_EINVAL (null pointer, N < 1, L out of range),
 * WD_EHIP. */
int wd_block_gram_static(const void* P, const void* Q, long long N, int L, void* C, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (linear, gauge covariant, frozen after training)
 * ------------------------------------------------------------------------- */

/* Number of layers and weights: theta is complex64 [layer][d][4][4] with
 * d = 0 the site term and d = 1 + 2 mu (+mu) / 2 + 2 mu (-mu) the hops.  A
 * layer maps psi to W_0 psi(x) + sum_mu [W_{+mu} U_mu(x) psi(x+mu)
 * + W_{-mu} U_mu(x-mu)^dag psi(x-mu)], W acting on spin; M_theta is the
 * product of the layers (layer 0 applied first). */
#define WD_LEARNED_LAYERS 3
#define WD_LEARNED_DIRS 9

/* Set theta (host pointer, 3*9*16 complex64 = interleaved float re, im). */
int wd_set_learned(wd_ctx* ctx, const float* theta_host);

/* Starting points for theta.  IDENTITY: W_0 = 1 and all hops 0 in every
 * layer, so M_theta = 1.  NEUMANN: the truncated Neumann series
 * 1 + x + x^2 + x^3 of (1 - x)^-1, x = kappa H (H the Wilson hopping term of
 * the operator, Sec. 2), written as the product (1 + x)(1 + i x)(1 - i x):
 * layer l has W_0 = 1, W_{+mu} = c_l kappa (1 - gamma_mu), W_{-mu} =
 * c_l kappa (1 + gamma_mu), c = (1, i, -i).  NEUMANN needs wd_set_params
 * (kappa) and ignores the clover term. */
#define WD_LEARNED_INIT_IDENTITY 0
#define WD_LEARNED_INIT_NEUMANN 1
int wd_learned_init(wd_ctx* ctx, int kind);

/* Z = M_theta R (FP64 in and out); prec WD_F64 runs the layers in FP64, WD_F32
 * in FP32 (arithmetic and intermediate storage).  R and Z are device block
 * vectors of L columns and must not overlap. */
int wd_learned_apply(wd_ctx* ctx, const void* R, void* Z, int L, int prec);

/* Training losses: the error of the proposed correction, mean ||M_theta r - e||^2 / ||e||^2, or
 * the residual it leaves, mean ||r - A M_theta r||^2 / ||r||^2 (e unused; needs wd_set_params). */
#define WD_LOSS_ERROR 0
#define WD_LOSS_RESIDUAL 1

/* Train theta on pairs (r, e) with A e ~ r: minimise the mean over columns of
 * the loss of loss_kind (WD_LOSS_ERROR: ||M_theta r - e||^2 / ||e||^2,
 * WD_LOSS_RESIDUAL: ||r - A M_theta r||^2 / ||r||^2, Ep may then be NULL)
 * with Adam (lr, beta1 0.9, beta2 0.999) for
 * `steps` steps; batch b uses columns [b*L, b*L + L) of the n_pairs columns
 * of Rp and Ep (device block vectors of n_pairs columns each, FP64), cycling.
 * Starts from the current theta and leaves the trained theta set.  loss_hist
 * (host, may be NULL) receives one loss per step.  Every column of Ep must be
 * non-zero and finite (WD_EINVAL otherwise, before any step). */
int wd_learned_train(wd_ctx* ctx, const void* Rp, const void* Ep, int n_pairs, int L,
                     int steps, double lr, int loss_kind, float* loss_hist);

/* Training pairs generated by the solver itself: for each of the n snapshots
 * X_k in Xsnap (device, n block vectors of L columns, as written by
 * bbicggr_solve with x_snap), Rp_k = B - A X_k and Ep_k = X - X_k, where X is
 * the converged solution of A X = B.  Rp and Ep are device buffers of n * L
 * columns (the layout wd_learned_train takes); none of the buffers may
 * overlap.  A pair satisfies A e = r exactly (up to rounding): e is the
 * correction that the residual r asks for.  A snapshot taken at the solve's
 * last iteration equals X and gives e = 0, which training rejects. */
int wd_learned_pairs(wd_ctx* ctx, const void* B, const void* X, const void* Xsnap, int n, int L, void* Rp,
                     void* Ep);

/* Copy the current theta to host memory (3*9*16 complex64). */
int wd_get_learned(wd_ctx* ctx, float* theta_host);

/* Loss of loss_kind (as in wd_learned_train) and its gradient with respect to theta on L
 * pairs, without updating theta: G_host receives 3*9*16 complex128 holding
 * dl/dRe(theta) + i dl/dIm(theta).  For testing the backward kernels. */
int wd_learned_grad(wd_ctx* ctx, const void* R, const void* E, int L, int loss_kind, double* loss,
                    double* G_host);

/* ---------------------------------------------------------------------------
 * Utilities
 * ------------------------------------------------------------------------- */

/* Static text for a return code. */
const char* wd_strerror(int code);

/* Lattice volume and N of a context. */
long long wd_volume(const wd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* WDSOLVE_H */
