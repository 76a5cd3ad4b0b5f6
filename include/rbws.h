/*
 * rbws.h -- C ABI of the MI355X reduced-basis warm-start solver (librbws.so).
 *
 * The library solves many instances of the parametrized linear system
 *     A_h(mu) u_h(mu) = f_h(mu)                     (paper, Eq. 1)
 * for the 3D diffusion problem -div(kappa(mu) grad u) = f on (0,1)^3 with
 * zero Dirichlet data (the paper's model PDE, Sec. 4), discretised by
 * 7-point finite differences on an n^3 grid of interior points.  The operator
 * is affine in the parameters, A_h(mu) = sum_q theta_q(mu) A_q.
 *
 * Calls follow the paper's statement of the method:
 *   - operator setup                       (Eq. 1; model PDE of Sec. 4)
 *   - offline greedy reduced-basis build   (Alg. 4: snapshots by Alg. 1,
 *     Gram-Schmidt, reduced matrices A_q^N = V^T A_q V)
 *   - batched solve from a zero, RB or learned initial value (Alg. 5 with
 *     the PCG of Alg. 1; RB value from the Galerkin system, Eq. "RB system").
 *
 * Conventions (all entry points):
 *   - Every call returns rbws_status; RBWS_OK is 0.  On failure
 *     rbws_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).  No exception crosses the ABI.
 *   - Handles are opaque and owned by the library until their *_destroy.
 *   - "host" pointers are ordinary CPU memory, read or written during the call.
 *     "device" pointers are GPU memory on the handle's device (e.g. the
 *     data_ptr() of a torch tensor); device work is ordered on `stream`
 *     (a hipStream_t, NULL = the default stream).
 *   - Vectors of one solve are n^3 contiguous values, x fastest:
 *     index (k-1) n^2 + (j-1) n + (i-1) for the interior point (i,j,k),
 *     1 <= i,j,k <= n, at coordinates (i,j,k)/(n+1).  A batch of B solves is
 *     B such vectors back to back.
 *   - Parameters mu are row-major (count, p) float64 host arrays.
 *   - Not reaching the tolerance within the iteration limit is not an error:
 *     it is reported per solve in rbws_solve_stat.status.
 *   - A handle may be used by one host thread at a time.
 */
#ifndef RBWS_H
#define RBWS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBWS_OK = 0,
  RBWS_EINVAL = -1,   /* invalid argument (null pointer, size, range, p mismatch) */
  RBWS_ENOMEM = -2,   /* device or host allocation failed */
  RBWS_EDEVICE = -3,  /* a HIP call failed */
  RBWS_ESTATE = -4,   /* the call needs state it was not given (e.g. RB start without a basis) */
  RBWS_ENUMERIC = -5  /* reduced matrix not positive definite, Gram-Schmidt breakdown */
} rbws_status;

/* problem kinds: how kappa(mu) depends on the parameters */
enum {
  RBWS_KIND_BLOCKS = 0,        /* kappa = 1, or mu_b inside axis-aligned block b (last listed
                                  block wins where blocks overlap); p = nblocks, Q = nblocks+1,
                                  theta = (1, mu_1, ..., mu_p) */
  RBWS_KIND_OCTANTS = 1,       /* kappa = mu_q on octant q = bx + 2 by + 4 bz of the 2x2x2
                                  split at 1/2; p = Q = 8, theta = mu */
  RBWS_KIND_OCTANTS_ANISO = 2  /* kappa = diag(mu[3q], mu[3q+1], mu[3q+2]) on octant q;
                                  Q = 24, p = 24 (+3 with the Gaussian source) */
};
/* right-hand sides: f_h = h^2 f(x_P), h = 1/(n+1) */
enum {
  RBWS_F_ONE = 0,   /* f = 1 */
  RBWS_F_GAUSS = 1  /* f = exp(-|x - x0|^2 / gauss_width), x0 = mu[24..26] (ANISO only); the
                       exponential rounded to nearest (the matrix-core projection V^T f uses
                       the device library's exp, within an ulp) */
};
enum { RBWS_INIT_ZERO = 0, RBWS_INIT_RB = 1, RBWS_INIT_LEARNED = 2 };
enum { RBWS_FP64 = 0, RBWS_FP32_IR = 1 };
/* the P of Alg. 1: identity, Jacobi (P r = r / diag A), or one multigrid
 * V-cycle (Alg. 2; see rbws_solve_opts.mg_nu) */
enum { RBWS_PREC_NONE = 0, RBWS_PREC_JACOBI = 1, RBWS_PREC_MG = 2 };
enum {
  RBWS_SOLVE_CONVERGED = 0,
  RBWS_SOLVE_MAXITER = 1,   /* the iteration limit (L_max of Alg. 1) was reached */
  RBWS_SOLVE_BREAKDOWN = 2, /* p^T A p <= 0 */
  RBWS_SOLVE_NAN = 3        /* a non-finite value appeared */
};
enum { RBWS_LIFT_EXACT = 0, RBWS_LIFT_MFMA = 1 };
/* FP32_IR variants: RESTART = classic refinement (each outer step solves the
 * correction equation from zero); RELIABLE = reliable updates (each outer
 * step folds the correction into u, replaces the FP32 residual by the true
 * FP64 one and continues CG with the current, rescaled search direction). */
enum { RBWS_IR_RESTART = 0, RBWS_IR_RELIABLE = 1 };
/* rbws_solve_opts.flags */
enum {
  RBWS_FLAG_FORCE_EXACT_DOTS = 1, /* take the exact integer path for every inner product
                                     (results are identical; for testing the fallback) */
  RBWS_FLAG_EXPLICIT_FALLBACK = 4, /* learned start, strict rule: compare explicit FP64
                                     residuals of both starts instead of the basis's
                                     residual decomposition */
  RBWS_FLAG_NO_GRAPH = 2          /* launch the iteration rounds one by one instead of
                                     replaying a captured HIP graph of them (results are
                                     identical; the graph is also skipped while kernel
                                     timing is on) */
};

typedef struct rbws_problem rbws_problem;
typedef struct rbws_basis rbws_basis;
typedef struct rbws_mlp rbws_mlp;

/* Problem description.  Coordinates of block bounds are in tenths of the unit
 * cube: blocks[6*b .. 6*b+5] = xlo, xhi, ylo, yhi, zlo, zhi (integers 0..10).
 * A face coefficient is kappa at the face midpoint; where the midpoint lies on
 * a sub-domain boundary along t axes it is the mean of the 2^t one-sided
 * values.  Copied during rbws_problem_create. */
typedef struct {
  int n;              /* interior points per axis, 1 <= n <= 1024 */
  int kind;           /* RBWS_KIND_* */
  int nblocks;        /* RBWS_KIND_BLOCKS: number of blocks, 1..31 */
  const int* blocks;  /* host, [nblocks][6], RBWS_KIND_BLOCKS only */
  int f_kind;         /* RBWS_F_* */
  double gauss_width; /* RBWS_F_GAUSS: the width w, at least 0.005 (EINVAL otherwise) */
} rbws_problem_desc;

/* Per-solve statistics (host output of rbws_solve). */
typedef struct {
  int iters;         /* CG iterations: SpMVs inside the loop of Alg. 1 (FP32_IR: inner, summed) */
  int outer_iters;   /* FP32_IR refinement steps (0 for FP64) */
  int extra_spmv;    /* true-residual evaluations beyond the initial one */
  int status;        /* RBWS_SOLVE_* */
  int init_used;     /* RBWS_INIT_* actually used (learned start may fall back to RB) */
  int vcycles;       /* V-cycles applied (RBWS_PREC_MG), else 0 */
  double init_rr;    /* ||f - A u0||^2 */
  double final_rr;   /* ||f - A u||^2 at exit (the true residual when converged) */
  double ff;         /* ||f||^2 */
  double t_done_ms;  /* completion time after the start of the solve phase (device clock) */
} rbws_solve_stat;

typedef struct {
  double tol;        /* stop when ||f - A u|| <= tol ||f|| (tested on squares) */
  int max_iter;      /* L_max (FP64); FP32_IR: cap on inner iterations per refinement step */
  int precond;       /* RBWS_PREC_* (the P of Alg. 1) */
  int precision;     /* RBWS_FP64 or RBWS_FP32_IR */
  int init;          /* RBWS_INIT_* */
  int lift;          /* RBWS_LIFT_EXACT (correctly rounded u0 = V c) or RBWS_LIFT_MFMA */
  double eta_inner;  /* FP32_IR: inner relative tolerance */
  int max_outer;     /* FP32_IR: refinement steps */
  int fallback;      /* learned start: 0 = start from whichever of u_MLP, u_RB has the smaller
                        true residual; 1 = use u_MLP unless its relative residual exceeds the
                        basis's final greedy indicator */
  int flags;         /* RBWS_FLAG_* */
  int check_every;   /* rounds between host checks for completion (0 = library default) */
  int ir_mode;       /* RBWS_IR_RESTART or RBWS_IR_RELIABLE (FP32_IR only) */
  int mg_nu;         /* RBWS_PREC_MG: damped-Jacobi sweeps before and after the coarse
                        correction on every level (1..8) */
  double mg_omega;   /* RBWS_PREC_MG: Jacobi damping, in (0, 1] */
} rbws_solve_opts;
/* The multigrid preconditioner (Alg. 2, V-cycle from a zero initial value):
 * levels n_0 = n, n_{l+1} = (n_l - 1) / 2 while n_l > 3; every level uses the
 * same 7-point face rule on its own grid (rediscretised, not P^T A P);
 * prolongation is trilinear interpolation between the vertex grids (which are
 * not nested when n + 1 is odd), restriction ((n_c+1)/(n_f+1)) P^T; the
 * coarsest level is solved exactly (dense Cholesky, at most 27 unknowns).
 * The V-cycle is a fixed symmetric positive definite operator, so PCG applies;
 * with RBWS_FP64 every step is evaluated in a fixed order and the trajectory
 * is reproducible bit for bit. */

/* ---- errors and defaults ------------------------------------------------ */
const char* rbws_last_error(void);
const char* rbws_version(void);
/* Fill *o with defaults: tol 1e-10, max_iter 50000, Jacobi, FP64, zero start,
 * exact lift, eta_inner 0.1, max_outer 40, fallback 0, flags 0, reliable updates
 * (classic restarted refinement works best with eta_inner about 1e-4),
 * mg_nu 1, mg_omega 6/7. */
void rbws_solve_opts_default(rbws_solve_opts* o);

/* ---- operator setup (Eq. 1; Sec. 4 model PDE) ----------------------------
 * Creates the face-class tables of the grid on `device`.  Errors: EINVAL for
 * an invalid description, EDEVICE/ENOMEM for HIP failures. */
rbws_status rbws_problem_create(const rbws_problem_desc* desc, int device, rbws_problem** out);
void rbws_problem_destroy(rbws_problem* p);
/* Sizes: any output pointer may be NULL. */
rbws_status rbws_problem_info(const rbws_problem* p, int* n, int* np, int* nq, long long* ndof);
/* theta(mu) of the affine form: host mu (nmu x p) -> host theta (nmu x Q). */
rbws_status rbws_theta(const rbws_problem* p, const double* mu, int nmu, double* theta);

/* y = A_h(mu_b) x_b for b < nmu.  x, y: device, nmu*ndof values of type
 * double (precision RBWS_FP64) or float (RBWS_FP32_IR: coefficients rounded
 * to float, float arithmetic).  The FP64 result is evaluated in a fixed order
 * (d_P x_P, then fma with the interior neighbours x-, x+, y-, y+, z-, z+) and
 * is bitwise reproducible. */
rbws_status rbws_spmv(rbws_problem* p, const double* mu, int nmu, const void* x, void* y,
                      int precision, void* stream);

/* s_b = MG(r_b) for b < nmu: one V-cycle from zero (Alg. 2 with nu damped
 * Jacobi sweeps of weight omega before and after the coarse correction; the
 * levels, transfers and coarsest solve of RBWS_PREC_MG), the preconditioner of
 * the multigrid path as an operator.  r, s: device, nmu*ndof values of type
 * double (RBWS_FP64: each step in a fixed order, bitwise reproducible) or
 * float (RBWS_FP32_IR: float coefficients and vectors; with nu = 1 the
 * smoothing multiplies by a float reciprocal of the diagonal).  r and s must
 * not overlap.  Blocks until done.  Errors: EINVAL (NULL, bad precision,
 * nu outside 1..8, omega outside (0, 1]), ENUMERIC (coarsest matrix not
 * positive definite), EDEVICE. */
rbws_status rbws_mg_apply(rbws_problem* p, const double* mu, int nmu, int nu, double omega, const void* r,
                          void* s, int precision, void* stream);

/* Correctly rounded dot products out[b] = sum_i x[b*len+i] y[b*len+i]
 * (exact sum of exact products rounded once to nearest-even), b < count.
 * x, y device (double); out host.  Used by every FP64 inner product. */
rbws_status rbws_exact_dots(const double* x, const double* y, long long len, int count,
                            double* out, int flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * correctly rounded dots as rbws_exact_dots, bit for bit, written to the
 * DEVICE array out (count doubles) on `stream`.  The call allocates nothing
 * and does not synchronise: its partial sums live in a fixed workspace of
 * RBWS_NOALLOC_SCRATCH_BYTES per GPU, inside the library, which holds
 * count * ceil(len / 4096) <= RBWS_NOALLOC_SCRATCH_BYTES / 24 partial sums
 * (e.g. 341 vectors of 128^3 entries).  Every call on one GPU uses that GPU's
 * workspace, so calls that overlap in time on one GPU (two streams or two
 * host threads) race; calls ordered on one stream do not.  The first call on
 * a device looks up the workspace's address there (not capturable; make one
 * call before capturing).  Errors: EINVAL (NULL pointer, negative size, more
 * partial sums than the workspace holds; nothing is launched), EDEVICE. */
#define RBWS_NOALLOC_SCRATCH_BYTES (4u << 20)
rbws_status rbws_exact_dots_noalloc(const double* x, const double* y, long long len, int count,
                                    double* out, int flags, void* stream);

/* dst[0:bytes) = src[0:bytes): a plain device copy with 16-byte
 * non-temporal loads and stores, each byte read and written once.  Not a step
 * of the method: the bandwidth a streaming kernel reaches on this device, the
 * reference that measured stencil and vector-update bandwidths and HBM
 * counters are compared with.  src, dst device, 16-byte aligned, not
 * overlapping; bytes a multiple of 16.  Stream-ordered, not synchronised.
 * Errors: EINVAL (NULL, misaligned, bytes negative or not a multiple of 16). */
rbws_status rbws_stream_copy(const void* src, void* dst, long long bytes, void* stream);

/* ---- offline: greedy reduced basis (Alg. 4 skeleton) ---------------------
 * Builds V (N orthonormal vectors), A_q^N = V^T A_q V and f^N = V^T f from the
 * training set mu_train (host, ntrain x p).  Step n: snapshot u(mu_l) by PCG
 * (Alg. 1) from zero to snap_tol with preconditioner `precond` and at most
 * snap_maxit iterations; two classical Gram-Schmidt passes against V; append
 * v / ||v||; then the indicator Delta(mu) = ||f - A(mu) V c(mu)|| / ||f|| on
 * the whole training set; the next parameter is the first maximiser.  The
 * first parameter is mu_train[0].  Stops early (n_reached < N) when the
 * maximiser is already selected or a snapshot adds nothing new (remainder
 * below 1e-10 of its norm).  All inner products are correctly rounded, so the
 * basis is reproducible.  With the Gaussian source (RBWS_F_GAUSS) the
 * reduced right-hand side V^T f(mu) is projected per parameter (FP64 matrix
 * cores, deterministic, not correctly rounded) and fN is unused.
 * Outputs (host, nullable): selected[N] (training indices), indicator_hist
 * [N x ntrain] (row k: indicator with k+1 vectors), n_reached.
 * Errors: EINVAL (N outside [1, min(64, ntrain)], snap_tol <= 0),
 * ENUMERIC (reduced matrix not positive definite), EDEVICE, ENOMEM. */
rbws_status rbws_rb_build(rbws_problem* p, const double* mu_train, int ntrain, int N, double snap_tol,
                          int precond, int snap_maxit, void* stream, rbws_basis** out, int* selected,
                          double* indicator_hist, int* n_reached);
/* L1-based reduced over-collocation (Sec. 3.1, Alg. 4), the paper's own RB
 * variant.  Same arguments as rbws_rb_build; N in [1, 60].
 * Step 1: snapshot u(mu_train[0]) by PCG; DEIM gives the first vector
 * w_1 = u / u(x_1), x_1 = argmax |u|.  Step n: the collocation least-squares
 * solve c(mu) = argmin || P (f - A(mu) W c) ||_2 at the collocation points X
 * (the distinct snapshot and residual DEIM points, ascending grid indices,
 * |X| <= 2n - 1) for every training parameter; the L1 indicator
 * ||c_U(mu)||_1 in the basis of the snapshots (W = U T); the first maximiser
 * mu_l; then (i) the residual r = f - A(mu_l) W c(mu_l) and its DEIM step
 * against the residual basis (a new residual point), (ii) the snapshot
 * u(mu_l) and its DEIM step against W (a new vector w_n, w_n(x_n) = 1, and a
 * new snapshot point).  DEIM step of x against vectors B with points x_i:
 * the unit lower-triangular interpolation system, r = x - B c (exact zeros
 * at the existing points), x_new = argmax |r| (lowest index on ties),
 * b_new = r / r(x_new).  Every inner product is correctly rounded and the
 * least-squares problem is solved by Householder QR with separately rounded
 * updates, so the basis is reproducible.  rbws_rb_coeffs, rbws_rb_lift and
 * rbws_solve accept the result like a Galerkin basis; the learned start's
 * cheap fallback rule, rbws_basis_save and the reduced matrices of
 * rbws_basis_get do not apply to it.  Errors as rbws_rb_build, plus EINVAL
 * for a non-constant source. */
rbws_status rbws_rb_build_l1roc(rbws_problem* p, const double* mu_train, int ntrain, int N, double snap_tol,
                                int precond, int snap_maxit, void* stream, rbws_basis** out, int* selected,
                                double* indicator_hist, int* n_reached);
/* The collocation points (npts <= 2N - 1, ascending grid indices), the
 * snapshot and residual DEIM points in selection order, and T (N x N, upper
 * triangular, W = U T) of an L1ROC basis; each output nullable; buffers of
 * 2N, N, N and N^2 entries suffice.  ESTATE for a Galerkin basis. */
rbws_status rbws_basis_l1roc(const rbws_basis* b, int* npts, long long* pts, int* nxs, long long* xs, int* nxr,
                             long long* xr, double* T);
void rbws_basis_destroy(rbws_basis* b);
/* N (reached), Q, ndof and the largest final indicator over the training set. */
rbws_status rbws_basis_info(const rbws_basis* b, int* N, int* nq, long long* ndof, double* final_max);
/* Host copies: V [N x ndof], AqN [Q x N x N], fN [N]; each may be NULL. */
rbws_status rbws_basis_get(const rbws_basis* b, double* V, double* AqN, double* fN);
/* Device pointer to V (N x ndof, row-major); valid until rbws_basis_destroy. */
rbws_status rbws_basis_device_v(const rbws_basis* b, const double** V);
/* Online RB solve (Eq. "RB system"): c(mu) from A_N(mu) = sum_q theta_q A_q^N
 * (accumulated with fma in q order), Cholesky and two triangular solves, every
 * inner sum correctly rounded; right-hand side f^N (f = 1) or V^T f(mu)
 * (Gaussian source).  For an L1ROC basis (rbws_rb_build_l1roc): the
 * collocation least-squares solution instead, one 64-thread block per
 * parameter.  mu host (nmu x p), c host (nmu x N).
 * ENUMERIC when a reduced matrix is not positive definite (or, for L1ROC, a
 * least-squares column vanishes). */
rbws_status rbws_rb_coeffs(const rbws_basis* b, const double* mu, int nmu, double* c, void* stream);
/* Lift u_b = V c_b for b < nmu: c device (nmu x N), u device (nmu x ndof).
 * mode RBWS_LIFT_EXACT: every entry a correctly rounded N-term dot;
 * RBWS_LIFT_MFMA: FP64 matrix cores (rounding depends on the blocking). */
rbws_status rbws_rb_lift(const rbws_basis* b, const double* c, int nmu, double* u, int mode, void* stream);
/* rel_b = ||f - A_h(mu_b) V c_b|| / ||f|| for b < nmu without forming V c_b: the
 * affine decomposition of the residual norm (Sec. 2.3's offline/online split
 * applied to r = f - sum_q theta_q(mu) A_q V c).  rbws_rb_build stores, for
 * f = 1 and when the Q N vectors A_q v_i fit in 8 GB, the correctly rounded
 * dots G = (A_q v_i)^T (A_q' v_j), g = (A_q v_i)^T f and f^T f; online,
 * ||r||^2 = f^T f - 2 y^T g + y^T G y with y = theta(mu) (x) c, O(Q^2 N^2) per
 * parameter.  mu host (nmu x p), c host (nmu x N), rel host (nmu).  Accurate
 * while ||r||^2 is not far below the terms' magnitude (relative residuals above
 * about 1e-4 of ||A V c|| / ||f||).  Errors: ESTATE when the basis has no
 * decomposition (Gaussian source, too large, or loaded from a file). */
rbws_status rbws_rb_residual_estimate(const rbws_basis* b, const double* mu, int nmu, const double* c, double* rel,
                                      void* stream);
/* Checkpoint: the basis, reduced matrices, selection and indicator history.
 * Loading checks that the file belongs to problem p. */
rbws_status rbws_basis_save(const rbws_basis* b, const char* path);
rbws_status rbws_basis_load(rbws_problem* p, const char* path, rbws_basis** out);

/* ---- learned start (an addition to the method; Sec. 1 cites neural-network
 * initial guesses as related work) --------------------------------------------
 * A multilayer perceptron maps the parameters to the reduced coefficients:
 *   x_i = (log10 mu_i - in_m) / in_s             for i < log_cols,
 *   x_i = (mu_i - (lin_lo + lin_hi)/2) / ((lin_hi - lin_lo)/2)   otherwise;
 *   h_1 = gelu(W_1 x + b_1), ..., h_D = gelu(W_D h_{D-1} + b_D)  (D = depth),
 *   y = W_o h_D + b_o,  gelu(z) = z Phi(z) (the erf form);
 *   c_j(mu) = (out_mean_j + out_std_j y_j) * 10^(-out_pow * l(mu)),
 *   l(mu) = mean of log10 mu_i over i < log_cols.
 * out_pow = 1 suits problems with A(t mu) = t A(mu) and f fixed (c(t mu) =
 * c(mu) / t); out_mean/out_std (default 0/1) standardise the targets.
 * Matrix products run on the BF16 matrix cores (weights and activations
 * rounded to nearest-even bfloat16, FP32 accumulation); master weights, Adam
 * moments and gradients are FP32.  Training minimises the mean over batch and
 * outputs of (y - y_target)^2 with Adam (bias-corrected, beta 0.9/0.999,
 * eps 1e-8) and a cosine step-size schedule.
 * Parameter vectors (host, float) are packed layer by layer: W_l (out x in,
 * row-major) then b_l, for l = 1..D, then W_o, b_o. */
typedef struct {
  int p;            /* inputs: the problem's parameter count */
  int nout;         /* outputs: the basis dimension, 1..64 */
  int hidden;       /* width of the hidden layers, a multiple of 32, <= 1024 */
  int depth;        /* hidden layers, 1..8 */
  int log_cols;     /* leading inputs that are log-scaled, 0..p */
  double in_m, in_s;        /* log scaling (in_s != 0) */
  double lin_lo, lin_hi;    /* linear scaling of the remaining inputs (lin_hi > lin_lo) */
  double out_pow;           /* output scale exponent (see above) */
} rbws_mlp_desc;
typedef struct {
  int epochs;       /* passes over the pairs */
  int batch;        /* minibatch size (a partial last minibatch of an epoch is dropped) */
  double lr;        /* initial step size; cosine decay to lr_min over all steps */
  double lr_min;
  unsigned long long seed;  /* minibatch order (a seeded shuffle per epoch) */
  int use_graph;    /* 1: each epoch is one captured HIP graph, replayed; 0: launches */
} rbws_mlp_train_cfg;
/* Create a network on `device`.  params: host, rbws_mlp_param_count values,
 * or NULL for a seeded initialisation (W uniform in +-1/sqrt(fan_in), b = 0).
 * Errors: EINVAL for an invalid description. */
rbws_status rbws_mlp_create(const rbws_mlp_desc* d, int device, const float* params,
                            unsigned long long seed, rbws_mlp** out);
void rbws_mlp_destroy(rbws_mlp* m);
rbws_status rbws_mlp_param_count(const rbws_mlp* m, long long* count);
/* The description the network was created with (host output). */
rbws_status rbws_mlp_info(const rbws_mlp* m, rbws_mlp_desc* d);
/* Host copies of the FP32 master parameters; set also resets Adam. */
rbws_status rbws_mlp_get_params(const rbws_mlp* m, float* params);
rbws_status rbws_mlp_set_params(rbws_mlp* m, const float* params);
/* Output scaling: mean/std host arrays of nout values (NULL = 0 and 1). */
rbws_status rbws_mlp_set_output_scaling(rbws_mlp* m, const double* mean, const double* stdev);
rbws_status rbws_mlp_get_output_scaling(const rbws_mlp* m, double* mean, double* stdev);
/* Set out_mean/out_std to the mean and standard deviation of the scaled
 * targets c * 10^(out_pow l(mu)) of the given pairs (computed on the GPU). */
rbws_status rbws_mlp_fit_output_scaling(rbws_mlp* m, const double* mu, const double* c, int npairs);
/* c (host, nmu x nout, double) = the network's prediction for mu (host, nmu x p). */
rbws_status rbws_mlp_predict(const rbws_mlp* m, const double* mu, int nmu, double* c);
/* Raw outputs y (host, nmu x nout, float) before output scaling. */
rbws_status rbws_mlp_forward(const rbws_mlp* m, const double* mu, int nmu, float* y);
/* Loss and gradient of one minibatch (mu host nb x p, c host nb x nout):
 * *loss = mean (y - y_target)^2 (accumulated in double); grads (host,
 * nullable) packed like the parameters.  Does not change the parameters. */
rbws_status rbws_mlp_grad(rbws_mlp* m, const double* mu, const double* c, int nb, double* loss,
                          float* grads);
/* One Adam step on one minibatch at step size lr (the gradient is the one
 * rbws_mlp_grad returns).  *loss (nullable) is the minibatch loss before the step. */
rbws_status rbws_mlp_adam_step(rbws_mlp* m, const double* mu, const double* c, int nb, double lr,
                               double* loss);
/* Train on npairs pairs (mu host npairs x p, c host npairs x nout, e.g. from
 * rbws_rb_coeffs).  loss_hist: host, nullable, epochs * (npairs / batch)
 * minibatch losses in step order.  Continues from the current parameters and
 * Adam state.  Errors: EINVAL (batch < 1 or > npairs, epochs < 1). */
rbws_status rbws_mlp_train(rbws_mlp* m, const double* mu, const double* c, int npairs,
                           const rbws_mlp_train_cfg* cfg, double* loss_hist);
/* Checkpoint: description, parameters, output scaling (not the Adam state). */
rbws_status rbws_mlp_save(const rbws_mlp* m, const char* path);
rbws_status rbws_mlp_load(const char* path, int device, rbws_mlp** out);

/* ---- batched solve (Alg. 5 driving Alg. 1) --------------------------------
 * Solves nmu systems in one batch.  problems[0..nprob) may have different
 * grid sizes (the uneven batch); problem_of[b] (NULL = all 0) picks the
 * problem of solve b; all problems must share p.  bases/mlps are indexed like
 * problems and may be NULL when init does not need them (ESTATE otherwise).
 * u_out: NULL, or nmu device pointers (double, ndof of that solve's problem)
 * that receive the solutions; stats: host, nmu entries (NULL allowed).
 * Returns after the stats are on the host; solutions are written on
 * `stream`.  */
rbws_status rbws_solve(rbws_problem* const* problems, const rbws_basis* const* bases,
                       const rbws_mlp* const* mlps, int nprob, const int* problem_of,
                       const double* mu, int nmu, const rbws_solve_opts* opts, void* stream,
                       void* const* u_out, rbws_solve_stat* stats);

/* ---- measurement ---------------------------------------------------------
 * Opt-in HIP-event timing of the library's kernel launches on the calling
 * thread, accumulated by kind: 0 A.p sweep (with the fused direction update),
 * 1 residual pass (initial / confirmation / refinement outer pass), 2 and 4
 * the per-solve scalar steps after each sweep, 3 update sweep (x, r and their
 * inner products), 5 SpMV, 6 MFMA lift, 7 reduced solves, 8 multigrid
 * V-cycle except its fused finest-level kernels (coarser levels, transfers,
 * the per-solve step after it), 9 the finest level's fused pre-smoothing and
 * residual, 10 its fused coarse correction, post-smoothing and r^T s,
 * 11 the projection V^T f(mu) of a parameter-dependent source (Galerkin
 * bases; L1ROC evaluates f at its collocation points inside 7).  The call
 * first waits for recorded events and returns the totals so far (ms[12],
 * launches[12], both nullable), then zeroes them if `reset`, then turns
 * timing on or off. */
rbws_status rbws_profile(int enable, double* ms, long long* launches, int reset);
/* How often a correctly rounded inner product could not be certified from
 * its double-double value and was recomputed exactly (current device):
 * counts[4] = solver and norm dots, basis dots, per-entry sums (Gram-Schmidt,
 * lift), reduced Cholesky/solves.  Diagnostics; results never depend on it. */
rbws_status rbws_exact_fallbacks(long long* counts, int reset);
/* Kernel-variant knobs (results are unaffected beyond FP32 rounding):
 * RBWS_TUNE_SWEEP32, value bit 0 / bit 1: the FP32 A.p / update sweeps keep
 * their face coefficients in registers (1) or look them up per plane (0).
 * RBWS_TUNE_GRID: the sweeps launch one workgroup per work item (0, default)
 * or a persistent grid of one full occupancy that loops over the items (1).
 * RBWS_TUNE_TZ: tile depth of every later batch, a power of two in [4, 64],
 * or 0 (default) for the autotuner's choice or the built-in rule; the coarser
 * levels of the multigrid preconditioner always take the built-in rule.
 * RBWS_TUNE_MG_PZ: where the tiles of a multigrid level span whole grid rows,
 * the FP32 post-smoothing interpolates the coarse correction itself (1,
 * default) or reads the z/y-interpolated rows from a separate pass (0); the
 * results are the same bits. */
enum { RBWS_TUNE_SWEEP32 = 0, RBWS_TUNE_GRID = 1, RBWS_TUNE_TZ = 2, RBWS_TUNE_MG_PZ = 3 };
rbws_status rbws_set_tuning(int key, int value);
/* Tile autotuner.  Work items are tiles of 1024 grid columns (32 x 32, or a
 * whole row when 32 < n <= 128) by TZ planes; a
 * deeper tile re-reads fewer halo planes, a shallower one gives more items
 * to spread over the 256 compute units.  Times y = A(mu) x for `nsolve` solves
 * of problem p (precision RBWS_FP64 or RBWS_FP32_IR) at TZ = 4, 8, ..., 64 and
 * keeps the fastest for later batches of this grid size whose solve count is
 * in the same power-of-two range (per process).  Each depth is timed in two
 * interleaved passes of five launches; its time is the faster pass's mean.
 * tz: host, the choice; ms: host, nullable, those 5 times in milliseconds (0
 * where not tried).  Results of the
 * solver do not depend on the tiling.  Errors: EINVAL, ENOMEM, EDEVICE.
 * rbws_autotune_clear drops every choice (back to the built-in rule). */
rbws_status rbws_autotune(rbws_problem* p, int nsolve, int precision, void* stream, int* tz, double* ms);
rbws_status rbws_autotune_clear(void);

#ifdef __cplusplus
}
#endif
#endif /* RBWS_H */
