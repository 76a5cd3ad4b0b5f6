/*
 * rbws_oracle.c -- CPU FP64 oracle for the reduced-basis warm-start solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, deliberately
 * unoptimised restatement of what the method computes.  It is used by the
 * test-suite, by the package's smoke check and by the benchmark's CPU
 * baseline, and by nothing else: the product path never calls it.  It shares
 * no code, headers or tables with the HIP library.
 *
 * What is computed, and where the paper defines it (Hou, Chen, Xia,
 * "A reduced basis warm-start iterative solver for the parameterized linear
 * systems"):
 *   - the parametrized system A_h(mu) u_h(mu) = f_h(mu)             (Eq. 1)
 *     here for -div(kappa(mu) grad u) = f on (0,1)^3 (model PDE, Sec. 4)
 *     discretised by 7-point finite differences with zero Dirichlet data;
 *   - preconditioned CG with a generic preconditioner P            (Alg. 1)
 *     with P = identity or Jacobi;
 *   - the greedy reduced-basis build (snapshots by Alg. 1, argmax of
 *     an error indicator over the training set)                    (Alg. 4)
 *     with a residual-norm indicator and Euclidean Gram-Schmidt;
 *   - the Galerkin reduced system A_N = W^T A W, b_N = W^T b and the
 *     RB solution W A_N^{-1} b_N                        (Eq. "RB system")
 *   - the warm-started solve: RB initial value, then PCG          (Alg. 5)
 *   - the L1-based reduced over-collocation method: DEIM of snapshots and
 *     residuals, the collocation least-squares online solve and the L1
 *     indicator of the greedy                            (Sec. 3.1, Alg. 4)
 *   - an FP32-inner / FP64-outer iterative refinement (an addition, not in
 *     the paper; the FP64 outer residual/update fixes the final accuracy).
 *
 * Readings of silent points:
 *   - every dot product is the exact sum of exact products rounded once to
 *     nearest-even (a "correctly rounded" dot), so that the result is a plain
 *     definition that does not depend on summation order;
 *   - the stencil is evaluated in one fixed order (below);
 *   - the loop of Alg. 1 runs while NOT converged (the printed inequality is
 *     reversed) and, when the recursive residual meets the tolerance, the true
 *     residual f - A x is recomputed; if it fails the test, CG restarts from it.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fopenmp -shared -fPIC ... -lquadmath
 * (-ffp-contract=off: every fused multiply-add below is an explicit fma()).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* problem description (plain data passed from Python)                 */
/* ------------------------------------------------------------------ */
enum { ORC_BLOCKS = 0, ORC_OCTANTS = 1, ORC_OCTANTS_ANISO = 2 };
enum { ORC_F_ONE = 0, ORC_F_GAUSS = 1 };
enum { ORC_PREC_NONE = 0, ORC_PREC_JACOBI = 1 };
enum { ORC_CONVERGED = 0, ORC_MAXITER = 1, ORC_BREAKDOWN = 2, ORC_NAN = 3 };

typedef struct {
    int n;              /* interior points per axis                       */
    int kind;           /* ORC_BLOCKS / ORC_OCTANTS / ORC_OCTANTS_ANISO    */
    int nblocks;        /* ORC_BLOCKS: number of blocks                    */
    const int *blocks;  /* [nblocks][6] = xlo,xhi,ylo,yhi,zlo,zhi (tenths) */
    int f_kind;         /* ORC_F_ONE / ORC_F_GAUSS                         */
    double gauss_width; /* width w in exp(-|x-x0|^2 / w)                   */
} orc_problem;

typedef struct {
    int iters;          /* SpMVs inside the CG loop                         */
    int extra_spmv;     /* true-residual confirmations                      */
    int status;         /* ORC_CONVERGED ...                                */
    int outer;          /* refinement steps (IR solver only)                */
    double init_rr;     /* ||r0||^2                                          */
    double final_rr;    /* ||r||^2 at exit (true residual when converged)    */
    double ff;          /* ||f||^2                                           */
} orc_stats;

int orc_nq(const orc_problem *P) {
    if (P->kind == ORC_BLOCKS) return P->nblocks + 1;
    if (P->kind == ORC_OCTANTS) return 8;
    return 24;
}

static long ndof_of(const orc_problem *P) { return (long)P->n * P->n * P->n; }

/* theta(mu): the affine coefficient functions.  BLOCKS: theta_0 = 1 (the
 * background), theta_b = mu_b.  OCTANTS: theta_q = mu_q.  ANISO: theta =
 * the 24 directional conductivities mu[3*octant + direction]. */
void orc_theta(const orc_problem *P, const double *mu, double *theta) {
    if (P->kind == ORC_BLOCKS) {
        theta[0] = 1.0;
        for (int b = 0; b < P->nblocks; b++) theta[b + 1] = mu[b];
    } else {
        int q = orc_nq(P);
        for (int i = 0; i < q; i++) theta[i] = mu[i];
    }
}

/* ------------------------------------------------------------------ */
/* exact accumulation: value = sum_i w[i] * 2^(32 i - XBIAS)           */
/* ------------------------------------------------------------------ */
#define XLIMBS 140
#define XBIAS 2240
typedef struct {
    int64_t w[XLIMBS];
    int bad;            /* a NaN or infinity was added */
} xacc;

static void xacc_clear(xacc *a) { memset(a, 0, sizeof *a); }

/* x = sgn * m * 2^e with m an integer below 2^53 */
static void split_double(double x, int *sgn, uint64_t *m, int *e) {
    uint64_t b;
    memcpy(&b, &x, 8);
    *sgn = (b >> 63) ? -1 : 1;
    int ex = (int)((b >> 52) & 0x7ff);
    uint64_t fr = b & ((1ull << 52) - 1);
    if (ex == 0) { *m = fr; *e = -1074; }
    else { *m = fr | (1ull << 52); *e = ex - 1075; }
}

/* add sgn * m * 2^e exactly; m < 2^128, e >= -2148 */
static void xacc_add_int(xacc *a, int sgn, unsigned __int128 m, int e) {
    int pos = e + XBIAS;
    int L = pos >> 5, s = pos & 31;
    for (int k = 0; m != 0; k++) {
        uint64_t chunk = (uint64_t)(m & 0xffffffffu);
        m >>= 32;
        uint64_t v = chunk << s;                    /* below 2^63 */
        a->w[L + k] += sgn * (int64_t)(v & 0xffffffffu);
        a->w[L + k + 1] += sgn * (int64_t)(v >> 32);
    }
}

static void xacc_add(xacc *a, double x) {
    if (!isfinite(x)) { a->bad = 1; return; }
    if (x == 0.0) return;
    int s; uint64_t m; int e;
    split_double(x, &s, &m, &e);
    xacc_add_int(a, s, m, e);
}

/* add the exact product x*y (integer mantissa product, no rounding) */
static void xacc_add_prod(xacc *a, double x, double y) {
    if (!isfinite(x) || !isfinite(y)) { a->bad = 1; return; }
    if (x == 0.0 || y == 0.0) return;
    int sx, sy; uint64_t mx, my; int ex, ey;
    split_double(x, &sx, &mx, &ex);
    split_double(y, &sy, &my, &ey);
    xacc_add_int(a, sx * sy, (unsigned __int128)mx * my, ex + ey);
}

/* round the exact value once to the nearest double, ties to even */
static double xacc_round(const xacc *a) {
    if (a->bad) return NAN;
    uint32_t d[XLIMBS];
    int64_t carry = 0;
    for (int i = 0; i < XLIMBS; i++) {
        int64_t t = a->w[i] + carry;
        int64_t low = t & 0xffffffff;               /* t mod 2^32, in [0,2^32) */
        d[i] = (uint32_t)low;
        carry = (t - low) / 4294967296LL;           /* exact */
    }
    int neg = 0;
    if (carry < 0) {                                /* value = D - 2^(32 XLIMBS) */
        neg = 1;
        uint64_t c = 1;                             /* magnitude = ~D + 1 */
        for (int i = 0; i < XLIMBS; i++) {
            uint64_t t = (uint64_t)(uint32_t)~d[i] + c;
            d[i] = (uint32_t)t;
            c = t >> 32;
        }
    }
    int top = -1;
    for (int i = XLIMBS - 1; i >= 0; i--) if (d[i]) { top = i; break; }
    if (top < 0) return 0.0;
    int msb = top * 32 + 31;
    while (!((d[msb >> 5] >> (msb & 31)) & 1u)) msb--;
    /* lowest kept bit: 53 significant bits, but never below 2^-1074 */
    int r = msb - 52;
    if (r < XBIAS - 1074) r = XBIAS - 1074;
    uint64_t M = 0;
    for (int b = msb; b >= r; b--) M = (M << 1) | ((d[b >> 5] >> (b & 31)) & 1u);
    int round_bit = 0, sticky = 0;
    if (r - 1 >= 0) round_bit = (d[(r - 1) >> 5] >> ((r - 1) & 31)) & 1u;
    for (int b = r - 2; b >= 0 && !sticky; b--)
        if ((d[b >> 5] >> (b & 31)) & 1u) sticky = 1;
    if (round_bit && (sticky || (M & 1u))) M++;
    double v = ldexp((double)M, r - XBIAS);       /* exact; inf on overflow */
    return neg ? -v : v;
}

/* correctly rounded dot product sum_i x_i y_i */
double orc_exact_dot(const double *x, const double *y, long n) {
    xacc a; xacc_clear(&a);
    for (long i = 0; i < n; i++) xacc_add_prod(&a, x[i], y[i]);
    return xacc_round(&a);
}

/* exp(x) rounded once to nearest (the Gaussian source): the binary128
 * exponential (error within a few units of its 113-bit last place) rounded
 * to double.  If that value lies so close to the midpoint between two
 * doubles that its own error could decide the rounding, the oracle cannot
 * certify the result and aborts. */
double orc_exp(double x) {
    __float128 q = expq((__float128)x);
    double d = (double)q;
    __float128 up = ((__float128)d + (__float128)nextafter(d, INFINITY)) / 2;
    __float128 dn = ((__float128)d + (__float128)nextafter(d, 0.0)) / 2;
    __float128 tol = q * 0x1p-104Q;
    if (fabsq(q - up) <= tol || fabsq(q - dn) <= tol) {
        fprintf(stderr, "orc_exp: rounding of exp(%a) not certified\n", x);
        abort();
    }
    return d;
}

/* correctly rounded sum */
double orc_exact_sum(const double *x, long n) {
    xacc a; xacc_clear(&a);
    for (long i = 0; i < n; i++) xacc_add(&a, x[i]);
    return xacc_round(&a);
}

/* The solvers' inner products (PCG, refinement): correctly rounded, or, for
 * timing a conventional CPU code only, a plain left-to-right FP64 loop.  The
 * switch is process-wide and is set before a solve starts. */
static int g_naive_dots = 0;
void orc_set_naive_dots(int on) { g_naive_dots = on ? 1 : 0; }

static double solver_dot(const double *x, const double *y, long n) {
    if (!g_naive_dots) return orc_exact_dot(x, y, n);
    double acc = 0.0;
    for (long i = 0; i < n; i++) acc = fma(x[i], y[i], acc);
    return acc;
}

/* ------------------------------------------------------------------ */
/* face coefficients                                                    */
/* Coordinates are scaled by 20(n+1) so that they are integers:          */
/*   node i (1..n)            -> 20 i                                     */
/*   face between i and i+1   -> 10 (2 i + 1)                              */
/*   a breakpoint of t tenths -> 2 (n+1) t                                 */
/* The coefficient of a face is kappa at its midpoint.  Where the midpoint */
/* lies on a sub-domain boundary along t axes, it is the mean of the 2^t   */
/* one-sided values (pairwise summed, then scaled by 2^-t).                */
/* ------------------------------------------------------------------ */
static int on_breakpoint(const orc_problem *P, int axis, long X) {
    long s = 2L * (P->n + 1);
    if (P->kind == ORC_BLOCKS) {
        for (int b = 0; b < P->nblocks; b++)
            if (X == s * P->blocks[6 * b + 2 * axis] || X == s * P->blocks[6 * b + 2 * axis + 1])
                return 1;
        return 0;
    }
    return X == 10L * (P->n + 1);
}

/* is coordinate X inside (lo, hi) when nudged to `side` (0 lower, 1 upper)? */
static int inside(long X, int side, long lo, long hi) {
    if (X > lo && X < hi) return 1;
    if (X == lo) return side == 1;
    if (X == hi) return side == 0;
    return 0;
}

/* region of the point X nudged to the given sides */
static int region_of(const orc_problem *P, const long X[3], const int side[3]) {
    if (P->kind == ORC_BLOCKS) {
        long s = 2L * (P->n + 1);
        for (int b = P->nblocks - 1; b >= 0; b--) {     /* last listed wins */
            const int *B = P->blocks + 6 * b;
            if (inside(X[0], side[0], s * B[0], s * B[1]) &&
                inside(X[1], side[1], s * B[2], s * B[3]) &&
                inside(X[2], side[2], s * B[4], s * B[5]))
                return b + 1;
        }
        return 0;
    }
    long mid = 10L * (P->n + 1);
    int o = 0;
    for (int a = 0; a < 3; a++)
        if (X[a] > mid || (X[a] == mid && side[a] == 1)) o |= 1 << a;
    return o;
}

static double pairwise_sum(const double *v, int cnt) {
    if (cnt == 1) return v[0];
    int h = cnt / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, h);
}

static double kappa_at(const orc_problem *P, const double *theta, const long X[3], int dir) {
    int tied[3], t = 0;
    for (int a = 0; a < 3; a++)
        if (on_breakpoint(P, a, X[a])) tied[t++] = a;
    double v[8];
    int nc = 1 << t;
    for (int c = 0; c < nc; c++) {
        int side[3] = {0, 0, 0};
        for (int m = 0; m < t; m++) side[tied[m]] = (c >> (t - 1 - m)) & 1;
        int reg = region_of(P, X, side);
        int idx = (P->kind == ORC_OCTANTS_ANISO) ? 3 * reg + dir : reg;
        v[c] = theta[idx];
    }
    return pairwise_sum(v, nc) * (1.0 / nc);
}

/* face arrays for a given theta:
 *   kx[((k-1) n + (j-1)) (n+1) + i],   i = 0..n   (face between i, i+1)
 *   ky[((k-1) (n+1) + j) n + (i-1)],   j = 0..n
 *   kz[(k n + (j-1)) n + (i-1)],       k = 0..n                        */
void orc_face_coeffs(const orc_problem *P, const double *theta, double *kx, double *ky, double *kz) {
    int n = P->n;
    for (int k = 1; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 0; i <= n; i++) {
                long X[3] = {10L * (2 * i + 1), 20L * j, 20L * k};
                kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + i] = kappa_at(P, theta, X, 0);
            }
    for (int k = 1; k <= n; k++)
        for (int j = 0; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                long X[3] = {20L * i, 10L * (2 * j + 1), 20L * k};
                ky[((long)(k - 1) * (n + 1) + j) * n + (i - 1)] = kappa_at(P, theta, X, 1);
            }
    for (int k = 0; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                long X[3] = {20L * i, 20L * j, 10L * (2 * k + 1)};
                kz[((long)k * n + (j - 1)) * n + (i - 1)] = kappa_at(P, theta, X, 2);
            }
}

typedef struct { double *kx, *ky, *kz; } faces;

static long nfaces_axis(int n) { return (long)(n + 1) * n * n; }

static faces faces_alloc(int n) {
    faces F;
    long m = nfaces_axis(n);
    F.kx = malloc(sizeof(double) * m);
    F.ky = malloc(sizeof(double) * m);
    F.kz = malloc(sizeof(double) * m);
    return F;
}
static void faces_free(faces F) { free(F.kx); free(F.ky); free(F.kz); }

static faces faces_for_mu(const orc_problem *P, const double *mu) {
    double theta[32];
    orc_theta(P, mu, theta);
    faces F = faces_alloc(P->n);
    orc_face_coeffs(P, theta, F.kx, F.ky, F.kz);
    return F;
}

/* the six face coefficients of unknown (i,j,k), 1-based */
static void six(const faces *F, int n, int i, int j, int k, double c[6]) {
    c[0] = F->kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + (i - 1)];
    c[1] = F->kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + i];
    c[2] = F->ky[((long)(k - 1) * (n + 1) + (j - 1)) * n + (i - 1)];
    c[3] = F->ky[((long)(k - 1) * (n + 1) + j) * n + (i - 1)];
    c[4] = F->kz[((long)(k - 1) * n + (j - 1)) * n + (i - 1)];
    c[5] = F->kz[((long)k * n + (j - 1)) * n + (i - 1)];
}

/* diagonal d_P = sum of the six faces, in the fixed order x-,x+,y-,y+,z-,z+ */
static double diag_of(const double c[6]) {
    return ((((c[0] + c[1]) + c[2]) + c[3]) + c[4]) + c[5];
}

/* y = A x, unscaled operator (A u)_P = sum_faces kappa_f (u_P - u_nb), u = 0
 * outside.  Order: acc = d_P x_P, then acc = fma(-kappa, x_nb, acc) for the
 * interior neighbours in the order x-, x+, y-, y+, z-, z+. */
static void apply_faces(const faces *F, int n, const double *x, double *y) {
    long n2 = (long)n * n;
    for (int k = 1; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                long P = (long)(k - 1) * n2 + (long)(j - 1) * n + (i - 1);
                double c[6];
                six(F, n, i, j, k, c);
                double acc = diag_of(c) * x[P];
                if (i > 1) acc = fma(-c[0], x[P - 1], acc);
                if (i < n) acc = fma(-c[1], x[P + 1], acc);
                if (j > 1) acc = fma(-c[2], x[P - n], acc);
                if (j < n) acc = fma(-c[3], x[P + n], acc);
                if (k > 1) acc = fma(-c[4], x[P - n2], acc);
                if (k < n) acc = fma(-c[5], x[P + n2], acc);
                y[P] = acc;
            }
}

static void diag_faces(const faces *F, int n, double *d) {
    long n2 = (long)n * n;
    for (int k = 1; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                double c[6];
                six(F, n, i, j, k, c);
                d[(long)(k - 1) * n2 + (long)(j - 1) * n + (i - 1)] = diag_of(c);
            }
}

/* public: y = A(theta) x */
void orc_apply_theta(const orc_problem *P, const double *theta, const double *x, double *y) {
    faces F = faces_alloc(P->n);
    orc_face_coeffs(P, theta, F.kx, F.ky, F.kz);
    apply_faces(&F, P->n, x, y);
    faces_free(F);
}

void orc_apply(const orc_problem *P, const double *mu, const double *x, double *y) {
    faces F = faces_for_mu(P, mu);
    apply_faces(&F, P->n, x, y);
    faces_free(F);
}

void orc_diag(const orc_problem *P, const double *mu, double *d) {
    faces F = faces_for_mu(P, mu);
    diag_faces(&F, P->n, d);
    faces_free(F);
}

/* right-hand side f_h = h^2 f(x_P), h = 1/(n+1) */
void orc_rhs(const orc_problem *P, const double *mu, double *f) {
    int n = P->n;
    double h = 1.0 / (n + 1);
    double h2 = h * h;
    for (int k = 1; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                long idx = ((long)(k - 1) * n + (j - 1)) * n + (i - 1);
                if (P->f_kind == ORC_F_ONE) {
                    f[idx] = h2;
                } else {
                    const double *x0 = mu + 24;
                    double dx = i * h - x0[0], dy = j * h - x0[1], dz = k * h - x0[2];
                    f[idx] = h2 * orc_exp(-(dx * dx + dy * dy + dz * dz) / P->gauss_width);
                }
            }
}

/* ------------------------------------------------------------------ */
/* Alg. 1: PCG, P in {identity, Jacobi}, FP64                           */
/* ------------------------------------------------------------------ */
static void precond_apply(int prec, const double *d, const double *r, double *s, long m) {
    if (prec == ORC_PREC_JACOBI) for (long i = 0; i < m; i++) s[i] = r[i] / d[i];
    else memcpy(s, r, sizeof(double) * m);
}

/* A preconditioner P(.) of Alg. 1: s = P(r). */
typedef void (*precond_fn)(void *ctx, const double *r, double *s);

typedef struct { int prec; const double *d; long m; } simple_prec;
static void simple_prec_apply(void *ctx, const double *r, double *s) {
    const simple_prec *c = ctx;
    precond_apply(c->prec, c->d, r, s, c->m);
}

/* Alg. 1 with a generic preconditioner.  Residual history: hist[0] =
 * ||r0||^2, hist[k] = recursive ||r||^2 after iteration k (at most maxit+1
 * entries).  rho = r^T s is a correctly rounded dot (for P = identity it is
 * ||r||^2). */
static int pcg_core(const faces *F, int n, const double *f, const double *u0, precond_fn pre, void *ctx,
                    double tol, int maxit, double *x, orc_stats *st, double *hist) {
    long m = (long)n * n * n;
    double *r = malloc(sizeof(double) * m), *s = malloc(sizeof(double) * m);
    double *p = malloc(sizeof(double) * m), *q = malloc(sizeof(double) * m);
    memset(st, 0, sizeof *st);
    double ff = solver_dot(f, f, m);
    double thr = (tol * tol) * ff;
    st->ff = ff;
    if (u0) memcpy(x, u0, sizeof(double) * m); else memset(x, 0, sizeof(double) * m);

    /* Alg. 1 step 2: r0 = f - A u0 */
    apply_faces(F, n, x, q);
    for (long i = 0; i < m; i++) r[i] = f[i] - q[i];
    double rr = solver_dot(r, r, m);
    st->init_rr = rr;
    if (hist) hist[0] = rr;
    int k = 0, extra = 0, status = ORC_MAXITER;
    double rho = 0.0;
    if (!isfinite(rr)) { status = ORC_NAN; goto done; }
    if (rr <= thr) { status = ORC_CONVERGED; goto done; }
    /* Alg. 1 steps 3-4: s0 = P(r0), p0 = s0 */
    pre(ctx, r, s);
    rho = solver_dot(r, s, m);
    memcpy(p, s, sizeof(double) * m);
    for (;;) {
        if (k >= maxit) { status = ORC_MAXITER; break; }
        apply_faces(F, n, p, q);
        double gamma = solver_dot(p, q, m);
        if (!isfinite(gamma)) { status = ORC_NAN; break; }
        if (!(gamma > 0.0)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / gamma;
        for (long i = 0; i < m; i++) {
            x[i] = fma(alpha, p[i], x[i]);
            r[i] = fma(-alpha, q[i], r[i]);
        }
        k++;
        rr = solver_dot(r, r, m);
        if (hist) hist[k] = rr;
        if (!isfinite(rr)) { status = ORC_NAN; break; }
        if (rr <= thr) {
            /* recursive residual meets the tolerance: confirm with f - A x */
            apply_faces(F, n, x, q);
            for (long i = 0; i < m; i++) r[i] = f[i] - q[i];
            extra++;
            rr = solver_dot(r, r, m);
            if (!isfinite(rr)) { status = ORC_NAN; break; }
            if (rr <= thr) { status = ORC_CONVERGED; break; }
            /* restart from the true residual */
            pre(ctx, r, s);
            rho = solver_dot(r, s, m);
            memcpy(p, s, sizeof(double) * m);
            continue;
        }
        pre(ctx, r, s);
        double rs = solver_dot(r, s, m);
        double beta = rs / rho;
        for (long i = 0; i < m; i++) p[i] = fma(beta, p[i], s[i]);
        rho = rs;
    }
done:
    st->iters = k;
    st->extra_spmv = extra;
    st->status = status;
    st->final_rr = rr;
    free(r); free(s); free(p); free(q);
    return status;
}

static int cg_faces(const faces *F, int n, const double *f, const double *u0, int prec,
                    double tol, int maxit, double *x, orc_stats *st, double *hist) {
    long m = (long)n * n * n;
    double *d = malloc(sizeof(double) * m);
    diag_faces(F, n, d);
    simple_prec c = {prec, d, m};
    int rc = pcg_core(F, n, f, u0, simple_prec_apply, &c, tol, maxit, x, st, hist);
    free(d);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Multigrid V-cycle preconditioner (Alg. 2) and MGCG                    */
/* ------------------------------------------------------------------ */
/* Levels: n_0 = n (finest), n_{l+1} = (n_l - 1) / 2 while n_l > 3.  Level
 * operators are the same 7-point rule on the coarser grid (rediscretised;
 * the paper forms P^T A P instead).  Vertex grids with n+1 intervals are not
 * nested when n+1 is odd, so the prolongation P is trilinear interpolation
 * between the grids: fine node i (at i/(nf+1)) lies in the coarse interval
 * [I, I+1] with I = floor(i (nc+1) / (nf+1)) and weight
 * w = (i (nc+1) - I (nf+1)) / (nf+1) on node I+1 (1 - w on node I); coarse
 * nodes 0 and nc+1 are on the boundary (value 0).  Restriction is
 * R = ((nc+1)/(nf+1)) P^T: with unscaled operators (A = h^2 L_h) this keeps
 * the coarse right-hand side consistent with the coarse operator.  The
 * coarsest level is solved exactly by a dense Cholesky factorisation.
 * Smoother: damped Jacobi e <- e + omega (b - A e) / d, nu sweeps before and
 * after the coarse correction, so the V-cycle is a symmetric operator.
 *
 * Fixed evaluation orders.  Alg. 2 fixes the transfer operators, not the
 * order of their sums; the separable x, y, z chains below are this oracle's
 * own definition of it (each output is a sum of at most 4^3 or 2^3 weighted
 * terms, and the tests pin every entry against the dense Kronecker form):
 *   Jacobi: q = A e (stencil order), t = b - q, t = t / d, e' = fma(omega, t, e)
 *   restriction, separable: ax = sum over i of px r (fma chain from 0, i
 *     ascending over the fine points whose weight on the coarse node may be
 *     nonzero), ay = sum over j of py ax, az = sum over k of pz ay, then
 *     az * ((nc+1)/(nf+1))
 *   prolongation, separable (interior corners only, each sum an fma chain
 *     from 0 over corner 0 then 1): az = sum over the z corners of wz e_c,
 *     ay = sum over the y corners of wy az, v = sum over the x corners of
 *     wx ay, then e = e + v
 *   coarse solve: Cholesky and the two triangular solves with sequential
 *     fma accumulation in index order. */
#define MG_MAXLEV 16
typedef struct {
    int nlev, nu;
    double omega;
    int n[MG_MAXLEV];
    faces F[MG_MAXLEV];
    double *d[MG_MAXLEV];
    int *ci[MG_MAXLEV];      /* transfer l -> l+1: coarse interval of fine index i (1..n_l) */
    double *cw[MG_MAXLEV];   /* its weight on the upper coarse node */
    double *b[MG_MAXLEV], *e[MG_MAXLEV], *t[MG_MAXLEV];
    double *L;               /* coarsest Cholesky factor (mc x mc, row-major) */
    int mc;
} mg_ctx;

int orc_mg_levels(int n, int *out) {
    int k = 0;
    out[k++] = n;
    while (out[k - 1] > 3 && k < MG_MAXLEV) { out[k] = (out[k - 1] - 1) / 2; k++; }
    return k;
}

static void mg_transfer_table(int nf, int nc, int *ci, double *cw) {
    for (int i = 1; i <= nf; i++) {
        long I = ((long)i * (nc + 1)) / (nf + 1);
        ci[i - 1] = (int)I;
        cw[i - 1] = (double)((long)i * (nc + 1) - I * (nf + 1)) / (double)(nf + 1);
    }
}

/* damped Jacobi sweep e_out = e_in + omega (b - A e_in) / d (e_in NULL = 0) */
static void mg_jacobi(const mg_ctx *c, int l, const double *b, const double *ein, double *eout) {
    int n = c->n[l];
    long m = (long)n * n * n;
    if (ein) apply_faces(&c->F[l], n, ein, c->t[l]);
    for (long i = 0; i < m; i++) {
        double q = ein ? c->t[l][i] : 0.0;
        double t = b[i] - q;
        t = t / c->d[l][i];
        eout[i] = fma(c->omega, t, ein ? ein[i] : 0.0);
    }
}

/* rc = ((nc+1)/(nf+1)) P^T rf */
static void mg_restrict(const mg_ctx *c, int l, const double *rf, double *rc) {
    int nf = c->n[l], nc = c->n[l + 1];
    const int *ci = c->ci[l];
    const double *cw = c->cw[l];
    double scale = (double)(nc + 1) / (double)(nf + 1);
    /* fine index ranges per coarse index: i with ci in {I-1, I} */
    int *lo = malloc(sizeof(int) * (nc + 2)), *hi = malloc(sizeof(int) * (nc + 2));
    for (int I = 1; I <= nc; I++) {
        lo[I] = nf + 1; hi[I] = 0;
        for (int i = 1; i <= nf; i++)
            if (ci[i - 1] == I - 1 || ci[i - 1] == I) { if (i < lo[I]) lo[I] = i; if (i > hi[I]) hi[I] = i; }
    }
    for (int K = 1; K <= nc; K++)
        for (int J = 1; J <= nc; J++)
            for (int I = 1; I <= nc; I++) {
                double az = 0.0;
                for (int k = lo[K]; k <= hi[K]; k++) {
                    double pz = ci[k - 1] == K ? 1.0 - cw[k - 1] : cw[k - 1];
                    double ay = 0.0;
                    for (int j = lo[J]; j <= hi[J]; j++) {
                        double py = ci[j - 1] == J ? 1.0 - cw[j - 1] : cw[j - 1];
                        double ax = 0.0;
                        for (int i = lo[I]; i <= hi[I]; i++) {
                            double px = ci[i - 1] == I ? 1.0 - cw[i - 1] : cw[i - 1];
                            ax = fma(px, rf[((long)(k - 1) * nf + (j - 1)) * nf + (i - 1)], ax);
                        }
                        ay = fma(py, ax, ay);
                    }
                    az = fma(pz, ay, az);
                }
                rc[((long)(K - 1) * nc + (J - 1)) * nc + (I - 1)] = az * scale;
            }
    free(lo); free(hi);
}

/* ef += P ec */
static void mg_prolong(const mg_ctx *c, int l, const double *ec, double *ef) {
    int nf = c->n[l], nc = c->n[l + 1];
    const int *ci = c->ci[l];
    const double *cw = c->cw[l];
    for (int k = 1; k <= nf; k++)
        for (int j = 1; j <= nf; j++)
            for (int i = 1; i <= nf; i++) {
                double v = 0.0;
                for (int cx = 0; cx < 2; cx++) {
                    int I = ci[i - 1] + cx;
                    if (I < 1 || I > nc) continue;
                    double wx = cx ? cw[i - 1] : 1.0 - cw[i - 1];
                    double ay = 0.0;
                    for (int cy = 0; cy < 2; cy++) {
                        int J = ci[j - 1] + cy;
                        if (J < 1 || J > nc) continue;
                        double wy = cy ? cw[j - 1] : 1.0 - cw[j - 1];
                        double az = 0.0;
                        for (int cz = 0; cz < 2; cz++) {
                            int K = ci[k - 1] + cz;
                            if (K < 1 || K > nc) continue;
                            double wz = cz ? cw[k - 1] : 1.0 - cw[k - 1];
                            az = fma(wz, ec[((long)(K - 1) * nc + (J - 1)) * nc + (I - 1)], az);
                        }
                        ay = fma(wy, az, ay);
                    }
                    v = fma(wx, ay, v);
                }
                long f = ((long)(k - 1) * nf + (j - 1)) * nf + (i - 1);
                ef[f] = ef[f] + v;
            }
}

/* dense Cholesky of the coarsest operator (mc <= 27), row-major lower factor */
static int mg_factor(mg_ctx *c) {
    int l = c->nlev - 1, n = c->n[l];
    int mc = n * n * n;
    c->mc = mc;
    double *A = calloc((size_t)mc * mc, sizeof(double));
    double *u = calloc(mc, sizeof(double)), *y = malloc(sizeof(double) * mc);
    for (int j = 0; j < mc; j++) {            /* column j = A e_j */
        u[j] = 1.0;
        apply_faces(&c->F[l], n, u, y);
        for (int i = 0; i < mc; i++) A[(long)i * mc + j] = y[i];
        u[j] = 0.0;
    }
    double *L = calloc((size_t)mc * mc, sizeof(double));
    int bad = 0;
    for (int j = 0; j < mc && !bad; j++) {
        double s = A[(long)j * mc + j];
        for (int k = 0; k < j; k++) s = fma(-L[(long)j * mc + k], L[(long)j * mc + k], s);
        if (!(s > 0.0)) { bad = 1; break; }
        double ljj = sqrt(s);
        L[(long)j * mc + j] = ljj;
        for (int i = j + 1; i < mc; i++) {
            double t = A[(long)i * mc + j];
            for (int k = 0; k < j; k++) t = fma(-L[(long)i * mc + k], L[(long)j * mc + k], t);
            L[(long)i * mc + j] = t / ljj;
        }
    }
    free(A); free(u); free(y);
    c->L = L;
    return bad;
}

static void mg_coarse_solve(const mg_ctx *c, const double *b, double *x) {
    int m = c->mc;
    const double *L = c->L;
    double *y = malloc(sizeof(double) * m);
    for (int i = 0; i < m; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s = fma(-L[(long)i * m + k], y[k], s);
        y[i] = s / L[(long)i * m + i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double s = y[i];
        for (int k = i + 1; k < m; k++) s = fma(-L[(long)k * m + i], x[k], s);
        x[i] = s / L[(long)i * m + i];
    }
    free(y);
}

/* Alg. 2 at level l: e = MG(b) */
static void mg_vcycle(const mg_ctx *c, int l, const double *b, double *e) {
    if (l == c->nlev - 1) { mg_coarse_solve(c, b, e); return; }
    int n = c->n[l];
    long m = (long)n * n * n;
    double *tmp = malloc(sizeof(double) * m);
    /* pre-smoothing from zero */
    mg_jacobi(c, l, b, NULL, e);
    for (int s = 1; s < c->nu; s++) { mg_jacobi(c, l, b, e, tmp); memcpy(e, tmp, sizeof(double) * m); }
    /* residual, restriction, coarse correction, prolongation */
    apply_faces(&c->F[l], n, e, c->t[l]);
    for (long i = 0; i < m; i++) tmp[i] = b[i] - c->t[l][i];
    mg_restrict(c, l, tmp, c->b[l + 1]);
    mg_vcycle(c, l + 1, c->b[l + 1], c->e[l + 1]);
    mg_prolong(c, l, c->e[l + 1], e);
    /* post-smoothing */
    for (int s = 0; s < c->nu; s++) { mg_jacobi(c, l, b, e, tmp); memcpy(e, tmp, sizeof(double) * m); }
    free(tmp);
}

static void mg_prec_apply(void *ctx, const double *r, double *s) { mg_vcycle(ctx, 0, r, s); }

static int mg_setup(mg_ctx *c, const orc_problem *P, const double *mu, int nu, double omega) {
    memset(c, 0, sizeof *c);
    c->nu = nu;
    c->omega = omega;
    c->nlev = orc_mg_levels(P->n, c->n);
    for (int l = 0; l < c->nlev; l++) {
        orc_problem Pl = *P;
        Pl.n = c->n[l];
        c->F[l] = faces_for_mu(&Pl, mu);
        long m = (long)c->n[l] * c->n[l] * c->n[l];
        c->d[l] = malloc(sizeof(double) * m);
        diag_faces(&c->F[l], c->n[l], c->d[l]);
        c->b[l] = malloc(sizeof(double) * m);
        c->e[l] = malloc(sizeof(double) * m);
        c->t[l] = malloc(sizeof(double) * m);
        if (l + 1 < c->nlev) {
            c->ci[l] = malloc(sizeof(int) * c->n[l]);
            c->cw[l] = malloc(sizeof(double) * c->n[l]);
        }
    }
    for (int l = 0; l + 1 < c->nlev; l++) mg_transfer_table(c->n[l], c->n[l + 1], c->ci[l], c->cw[l]);
    return mg_factor(c);
}

static void mg_free(mg_ctx *c) {
    for (int l = 0; l < c->nlev; l++) {
        faces_free(c->F[l]);
        free(c->d[l]); free(c->b[l]); free(c->e[l]); free(c->t[l]);
        free(c->ci[l]); free(c->cw[l]);
    }
    free(c->L);
}

/* One level pair's transfers on their own (for tests): dir 0 gives
 * out = ((nc+1)/(nf+1)) P^T in (in on the nf grid, out on the nc grid),
 * dir 1 gives out = P in (in on the nc grid, out on the nf grid). */
void orc_mg_transfer(int nf, int nc, int dir, const double *in, double *out) {
    mg_ctx c;
    memset(&c, 0, sizeof c);
    c.nlev = 2;
    c.n[0] = nf;
    c.n[1] = nc;
    c.ci[0] = malloc(sizeof(int) * nf);
    c.cw[0] = malloc(sizeof(double) * nf);
    mg_transfer_table(nf, nc, c.ci[0], c.cw[0]);
    if (dir == 0) {
        mg_restrict(&c, 0, in, out);
    } else {
        memset(out, 0, sizeof(double) * (size_t)nf * nf * nf);
        mg_prolong(&c, 0, in, out);
    }
    free(c.ci[0]);
    free(c.cw[0]);
}

/* s = MG(r) for one mu (the V-cycle as an operator, for tests) */
int orc_mg_apply(const orc_problem *P, const double *mu, int nu, double omega, const double *r, double *s) {
    mg_ctx c;
    int bad = mg_setup(&c, P, mu, nu, omega);
    if (!bad) mg_prec_apply(&c, r, s);
    mg_free(&c);
    return bad;
}

/* MGCG: Alg. 1 with s = MG(r) (Alg. 2), from u0 (NULL = 0) */
int orc_mgcg(const orc_problem *P, const double *mu, const double *f, const double *u0, int nu, double omega,
             double tol, int maxit, double *x, orc_stats *st) {
    mg_ctx c;
    if (mg_setup(&c, P, mu, nu, omega)) { mg_free(&c); memset(st, 0, sizeof *st); st->status = ORC_BREAKDOWN; return ORC_BREAKDOWN; }
    int s = pcg_core(&c.F[0], P->n, f, u0, mg_prec_apply, &c, tol, maxit, x, st, NULL);
    mg_free(&c);
    return s;
}

void orc_mgcg_batch(const orc_problem *P, const double *mu, int nmu, const double *f, const double *u0, int nu,
                    double omega, double tol, int maxit, double *x, orc_stats *st, int nthreads) {
    long m = ndof_of(P);
    int p = P->kind == ORC_BLOCKS ? P->nblocks : (P->kind == ORC_OCTANTS ? 8 : 24 + (P->f_kind == ORC_F_GAUSS ? 3 : 0));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < nmu; b++)
        orc_mgcg(P, mu + (long)b * p, f + b * m, u0 ? u0 + b * m : NULL, nu, omega, tol, maxit, x + b * m, st + b);
}

int orc_cg(const orc_problem *P, const double *mu, const double *f, const double *u0, int prec,
           double tol, int maxit, double *x, orc_stats *st, double *hist) {
    faces F = faces_for_mu(P, mu);
    int s = cg_faces(&F, P->n, f, u0, prec, tol, maxit, x, st, hist);
    faces_free(F);
    return s;
}

/* many independent solves, one per thread (f per solve: f + i*ndof) */
void orc_cg_batch(const orc_problem *P, const double *mu, int nmu, const double *f,
                  const double *u0, int prec, double tol, int maxit, double *x, orc_stats *st,
                  int nthreads) {
    long m = ndof_of(P);
    int p = P->kind == ORC_BLOCKS ? P->nblocks : (P->kind == ORC_OCTANTS ? 8 : 24 + (P->f_kind == ORC_F_GAUSS ? 3 : 0));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < nmu; b++)
        orc_cg(P, mu + (long)b * p, f + b * m, u0 ? u0 + b * m : NULL, prec, tol, maxit,
               x + b * m, st + b, NULL);
}

/* ------------------------------------------------------------------ */
/* Galerkin reduced system and its Cholesky solve (Eq. "RB system")     */
/* ------------------------------------------------------------------ */
/* A_N(mu)[i][j] = sum_q theta_q AqN[q][i][j], accumulated in q order with fma */
void orc_rb_assemble(int Q, int N, int ld, const double *AqN, const double *theta, double *AN) {
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            double a = 0.0;
            for (int q = 0; q < Q; q++) a = fma(theta[q], AqN[((long)q * ld + i) * ld + j], a);
            AN[i * N + j] = a;
        }
}

/* Cholesky A = L L^T and the two triangular solves, each inner sum one
 * correctly rounded dot.  Returns 0, or -1 when a pivot is not positive. */
int orc_chol_solve(int N, const double *A, const double *b, double *c) {
    double *L = calloc((size_t)N * N, sizeof(double));
    double *y = malloc(sizeof(double) * N);
    int ok = 0;
    for (int j = 0; j < N && !ok; j++) {
        xacc a; xacc_clear(&a);
        xacc_add(&a, A[j * N + j]);
        for (int k = 0; k < j; k++) xacc_add_prod(&a, -L[j * N + k], L[j * N + k]);
        double piv = xacc_round(&a);
        if (!(piv > 0.0) || !isfinite(piv)) { ok = -1; break; }
        double ljj = sqrt(piv);
        L[j * N + j] = ljj;
        for (int i = j + 1; i < N; i++) {
            xacc t; xacc_clear(&t);
            xacc_add(&t, A[i * N + j]);
            for (int k = 0; k < j; k++) xacc_add_prod(&t, -L[i * N + k], L[j * N + k]);
            L[i * N + j] = xacc_round(&t) / ljj;
        }
    }
    if (ok == 0) {
        for (int i = 0; i < N; i++) {              /* L y = b */
            xacc t; xacc_clear(&t);
            xacc_add(&t, b[i]);
            for (int k = 0; k < i; k++) xacc_add_prod(&t, -L[i * N + k], y[k]);
            y[i] = xacc_round(&t) / L[i * N + i];
        }
        for (int i = N - 1; i >= 0; i--) {         /* L^T c = y */
            xacc t; xacc_clear(&t);
            xacc_add(&t, y[i]);
            for (int k = i + 1; k < N; k++) xacc_add_prod(&t, -L[k * N + i], c[k]);
            c[i] = xacc_round(&t) / L[i * N + i];
        }
    }
    free(L); free(y);
    return ok;
}

/* u = V c, each entry a correctly rounded N-term dot.  V is N x m, row-major. */
void orc_lift(int N, long m, const double *V, const double *c, double *u) {
    for (long i = 0; i < m; i++) {
        xacc a; xacc_clear(&a);
        for (int j = 0; j < N; j++) xacc_add_prod(&a, V[(long)j * m + i], c[j]);
        u[i] = xacc_round(&a);
    }
}

/* reduced right-hand side b_N = V^T f */
static void project(int N, long m, const double *V, const double *f, double *bN) {
    for (int j = 0; j < N; j++) bN[j] = orc_exact_dot(V + (long)j * m, f, m);
}

/* RB coefficients for one mu with a basis of dimension N (leading dimension
 * ld of AqN).  fN is used for f = 1; for the Gaussian source b_N = V^T f(mu). */
int orc_rb_coeffs(const orc_problem *P, int N, int ld, const double *AqN, const double *fN,
                  const double *V, const double *mu, double *c) {
    int Q = orc_nq(P);
    double theta[32];
    orc_theta(P, mu, theta);
    double *AN = malloc(sizeof(double) * N * N), *bN = malloc(sizeof(double) * N);
    orc_rb_assemble(Q, N, ld, AqN, theta, AN);
    if (P->f_kind == ORC_F_ONE) memcpy(bN, fN, sizeof(double) * N);
    else {
        long m = ndof_of(P);
        double *f = malloc(sizeof(double) * m);
        orc_rhs(P, mu, f);
        project(N, m, V, f, bN);
        free(f);
    }
    int s = orc_chol_solve(N, AN, bN, c);
    free(AN); free(bN);
    return s;
}

/* error indicator Delta(mu) = ||f - A(mu) V c(mu)|| / ||f||, evaluated directly */
static double indicator(const orc_problem *P, int N, int ld, const double *AqN, const double *fN,
                        const double *V, const double *mu, int *err) {
    long m = ndof_of(P);
    double c[128];
    if (orc_rb_coeffs(P, N, ld, AqN, fN, V, mu, c) != 0) { *err = 1; return NAN; }
    double *u = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    double *f = malloc(sizeof(double) * m);
    orc_lift(N, m, V, c, u);
    orc_apply(P, mu, u, r);
    orc_rhs(P, mu, f);
    for (long i = 0; i < m; i++) r[i] = f[i] - r[i];
    double rr = orc_exact_dot(r, r, m), ff = orc_exact_dot(f, f, m);
    free(u); free(r); free(f);
    return sqrt(rr / ff);
}

void orc_indicators(const orc_problem *P, int N, int ld, const double *AqN, const double *fN,
                    const double *V, const double *mu, int nmu, double *delta, int nthreads) {
    int p = P->kind == ORC_BLOCKS ? P->nblocks : (P->kind == ORC_OCTANTS ? 8 : 24 + (P->f_kind == ORC_F_GAUSS ? 3 : 0));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < nmu; b++) {
        int err = 0;
        delta[b] = indicator(P, N, ld, AqN, fN, V, mu + (long)b * p, &err);
    }
}

/* ------------------------------------------------------------------ */
/* Alg. 4 skeleton: greedy basis build                                   */
/* ------------------------------------------------------------------ */
/* Outputs: V (N x m), AqN (Q x N x N, leading dim N), fN (N), selected (N),
 * hist (N x ntrain; row k = indicator with k+1 basis vectors), nreached.
 * Returns 0, or -1 on a reduced-matrix breakdown. */
int orc_greedy(const orc_problem *P, const double *mu_train, int ntrain, int N, double snap_tol,
               int prec, int snap_maxit, double *V, double *AqN, double *fN, int *selected,
               double *hist, int *nreached, orc_stats *snap_stats, int nthreads) {
    long m = ndof_of(P);
    int Q = orc_nq(P);
    int p = P->kind == ORC_BLOCKS ? P->nblocks : (P->kind == ORC_OCTANTS ? 8 : 24 + (P->f_kind == ORC_F_GAUSS ? 3 : 0));
    faces *Fq = malloc(sizeof(faces) * Q);
    for (int q = 0; q < Q; q++) {                 /* A_q = A(theta = e_q) */
        double e[32] = {0};
        e[q] = 1.0;
        Fq[q] = faces_alloc(P->n);
        orc_face_coeffs(P, e, Fq[q].kx, Fq[q].ky, Fq[q].kz);
    }
    double *u = malloc(sizeof(double) * m), *v = malloc(sizeof(double) * m);
    double *w = malloc(sizeof(double) * m), *f = malloc(sizeof(double) * m);
    double cc[128];
    memset(AqN, 0, sizeof(double) * Q * N * N);
    int nb = 0, l = 0, rc = 0;
    for (;;) {
        /* snapshot u(mu_l) by Alg. 1 from zero */
        const double *mul = mu_train + (long)l * p;
        orc_rhs(P, mul, f);
        orc_stats st;
        orc_cg(P, mul, f, NULL, prec, snap_tol, snap_maxit, u, &st, NULL);
        if (snap_stats) snap_stats[nb] = st;
        /* two classical Gram-Schmidt passes against V, each entry one dot */
        memcpy(v, u, sizeof(double) * m);
        for (int pass = 0; pass < 2; pass++) {
            for (int j = 0; j < nb; j++) cc[j] = orc_exact_dot(V + (long)j * m, v, m);
            for (long i = 0; i < m; i++) {
                xacc a; xacc_clear(&a);
                xacc_add(&a, v[i]);
                for (int j = 0; j < nb; j++) xacc_add_prod(&a, -cc[j], V[(long)j * m + i]);
                v[i] = xacc_round(&a);
            }
        }
        double nrm = sqrt(orc_exact_dot(v, v, m));
        double unrm = sqrt(orc_exact_dot(u, u, m));
        if (!(nrm >= 1e-10 * unrm)) break;        /* nothing new in this snapshot */
        for (long i = 0; i < m; i++) V[(long)nb * m + i] = v[i] / nrm;
        selected[nb] = l;
        /* reduced matrices: AqN[q][i][nb] = AqN[q][nb][i] = v_i . (A_q v_nb) */
        const double *vn = V + (long)nb * m;
        for (int q = 0; q < Q; q++) {
            apply_faces(&Fq[q], P->n, vn, w);
            for (int i = 0; i <= nb; i++) {
                double a = orc_exact_dot(V + (long)i * m, w, m);
                AqN[((long)q * N + i) * N + nb] = a;
                AqN[((long)q * N + nb) * N + i] = a;
            }
        }
        orc_rhs(P, mu_train, f);                  /* f = 1: same for every mu */
        fN[nb] = orc_exact_dot(vn, f, m);
        nb++;
        /* indicator over the training set with nb basis vectors */
        double *row = hist + (long)(nb - 1) * ntrain;
        orc_indicators(P, nb, N, AqN, fN, V, mu_train, ntrain, row, nthreads);
        for (int b = 0; b < ntrain; b++) if (!isfinite(row[b])) rc = -1;
        if (rc || nb == N) break;
        int best = 0;
        for (int b = 1; b < ntrain; b++) if (row[b] > row[best]) best = b;
        int dup = 0;
        for (int j = 0; j < nb; j++) if (selected[j] == best) dup = 1;
        if (dup) break;
        l = best;
    }
    *nreached = nb;
    for (int q = 0; q < Q; q++) faces_free(Fq[q]);
    free(Fq); free(u); free(v); free(w); free(f);
    return rc;
}

/* ------------------------------------------------------------------ */
/* FP32-inner / FP64-outer iterative refinement                        */
/* ------------------------------------------------------------------ */
/* Inner solve: PCG in FP32 on A32 d = b32 from d = 0 (face coefficients
 * rounded once to FP32, stencil in FP32 in the same order as FP64, dots
 * accumulated in FP64 where products of two floats are exact), stopped at
 * ||r|| <= eta ||b|| or kin_max iterations.  Outer: r = f - A u in FP64,
 * b32 = fl32(r * 2^-e) with 2^e ~ ||r||, u += 2^e d. */
static void apply32(const float *kx, const float *ky, const float *kz, int n, const float *x, float *y) {
    long n2 = (long)n * n;
    for (int k = 1; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                long P = (long)(k - 1) * n2 + (long)(j - 1) * n + (i - 1);
                float c0 = kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + (i - 1)];
                float c1 = kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + i];
                float c2 = ky[((long)(k - 1) * (n + 1) + (j - 1)) * n + (i - 1)];
                float c3 = ky[((long)(k - 1) * (n + 1) + j) * n + (i - 1)];
                float c4 = kz[((long)(k - 1) * n + (j - 1)) * n + (i - 1)];
                float c5 = kz[((long)k * n + (j - 1)) * n + (i - 1)];
                float d = ((((c0 + c1) + c2) + c3) + c4) + c5;
                float acc = d * x[P];
                if (i > 1) acc = fmaf(-c0, x[P - 1], acc);
                if (i < n) acc = fmaf(-c1, x[P + 1], acc);
                if (j > 1) acc = fmaf(-c2, x[P - n], acc);
                if (j < n) acc = fmaf(-c3, x[P + n], acc);
                if (k > 1) acc = fmaf(-c4, x[P - n2], acc);
                if (k < n) acc = fmaf(-c5, x[P + n2], acc);
                y[P] = acc;
            }
}

/* reliable = 1: reliable updates.  Each outer step folds the correction d
 * into u, replaces the FP32 residual by the true one (rescaled) and continues
 * CG with the current search direction p (rescaled by the same power of two)
 * instead of restarting from zero; beta uses the new residual. */
int orc_ir_solve2(const orc_problem *P, const double *mu, const double *f, const double *u0, int prec,
                  double tol, double eta, int kin_max, int max_outer, int reliable, double *u,
                  orc_stats *st);

int orc_ir_solve(const orc_problem *P, const double *mu, const double *f, const double *u0, int prec,
                 double tol, double eta, int kin_max, int max_outer, double *u, orc_stats *st) {
    return orc_ir_solve2(P, mu, f, u0, prec, tol, eta, kin_max, max_outer, 0, u, st);
}

int orc_ir_solve2(const orc_problem *P, const double *mu, const double *f, const double *u0, int prec,
                  double tol, double eta, int kin_max, int max_outer, int reliable, double *u,
                  orc_stats *st) {
    int n = P->n;
    long m = ndof_of(P), nf = nfaces_axis(n);
    faces F = faces_for_mu(P, mu);
    float *kx = malloc(sizeof(float) * nf), *ky = malloc(sizeof(float) * nf), *kz = malloc(sizeof(float) * nf);
    for (long i = 0; i < nf; i++) { kx[i] = (float)F.kx[i]; ky[i] = (float)F.ky[i]; kz[i] = (float)F.kz[i]; }
    double *r = malloc(sizeof(double) * m), *q64 = malloc(sizeof(double) * m);
    float *d = malloc(sizeof(float) * m), *ri = malloc(sizeof(float) * m), *s = malloc(sizeof(float) * m);
    float *p = malloc(sizeof(float) * m), *q = malloc(sizeof(float) * m), *dg = malloc(sizeof(float) * m);
    long n2 = (long)n * n;
    for (int k = 1; k <= n; k++)
        for (int j = 1; j <= n; j++)
            for (int i = 1; i <= n; i++) {
                float c0 = kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + (i - 1)];
                float c1 = kx[((long)(k - 1) * n + (j - 1)) * (n + 1) + i];
                float c2 = ky[((long)(k - 1) * (n + 1) + (j - 1)) * n + (i - 1)];
                float c3 = ky[((long)(k - 1) * (n + 1) + j) * n + (i - 1)];
                float c4 = kz[((long)(k - 1) * n + (j - 1)) * n + (i - 1)];
                float c5 = kz[((long)k * n + (j - 1)) * n + (i - 1)];
                dg[(long)(k - 1) * n2 + (long)(j - 1) * n + (i - 1)] = ((((c0 + c1) + c2) + c3) + c4) + c5;
            }
    memset(st, 0, sizeof *st);
    double ff = solver_dot(f, f, m), thr = (tol * tol) * ff;
    st->ff = ff;
    if (u0) memcpy(u, u0, sizeof(double) * m); else memset(u, 0, sizeof(double) * m);
    int outer = 0, inner = 0, status = ORC_MAXITER;
    double rr = 0, rho_prev = 0.0, sc_prev = 1.0;
    int have_dir = 0;
    for (;;) {
        apply_faces(&F, n, u, q64);
        for (long i = 0; i < m; i++) r[i] = f[i] - q64[i];
        rr = solver_dot(r, r, m);
        if (outer == 0) st->init_rr = rr;
        if (!isfinite(rr)) { status = ORC_NAN; break; }
        if (rr <= thr) { status = ORC_CONVERGED; break; }
        if (outer >= max_outer || inner >= kin_max * max_outer) { status = ORC_MAXITER; break; }
        int e = ilogb(sqrt(rr));
        double sc = ldexp(1.0, -e);
        for (long i = 0; i < m; i++) { ri[i] = (float)(r[i] * sc); d[i] = 0.0f; }
        double bb = 0.0;
        for (long i = 0; i < m; i++) bb += (double)ri[i] * (double)ri[i];
        /* the inner solve reduces the residual by eta, and at least to eta ||f||
         * (in the scaled units): a start whose residual exceeds ||f|| (a reduced
         * basis start with a small error but a large residual) then needs no
         * more outer steps than the zero start */
        double thr_in = (eta * eta) * fmin(bb, ff * sc * sc);
        for (long i = 0; i < m; i++) s[i] = (prec == ORC_PREC_JACOBI) ? ri[i] / dg[i] : ri[i];
        double rho_new = 0.0;
        for (long i = 0; i < m; i++) rho_new += (double)ri[i] * (double)s[i];
        if (reliable && have_dir) {
            /* p (old units) times sc/sc_old is the direction in new units; with
             * beta = rho_new / (rho_old (sc/sc_old)^2) the update is
             * p = s + rho_new / (rho_old sc/sc_old) p_old */
            float b = (float)(rho_new / (rho_prev * (sc / sc_prev)));
            for (long i = 0; i < m; i++) p[i] = fmaf(b, p[i], s[i]);
        } else {
            memcpy(p, s, sizeof(float) * m);
        }
        double rho = rho_new;
        have_dir = 0;
        for (int k = 0; k < kin_max; k++) {
            apply32(kx, ky, kz, n, p, q);
            double g = 0.0;
            for (long i = 0; i < m; i++) g += (double)p[i] * (double)q[i];
            if (!(g > 0.0)) { have_dir = 0; break; }
            float a = (float)(rho / g);
            for (long i = 0; i < m; i++) { d[i] = fmaf(a, p[i], d[i]); ri[i] = fmaf(-a, q[i], ri[i]); }
            inner++;
            double rri = 0.0, rs = 0.0;
            for (long i = 0; i < m; i++) {
                s[i] = (prec == ORC_PREC_JACOBI) ? ri[i] / dg[i] : ri[i];
                rri += (double)ri[i] * (double)ri[i];
                rs += (double)ri[i] * (double)s[i];
            }
            have_dir = 1;
            rho_prev = rho;
            if (rri <= thr_in) break;
            float b = (float)(rs / rho);
            for (long i = 0; i < m; i++) p[i] = fmaf(b, p[i], s[i]);
            rho = rs;
        }
        sc_prev = sc;
        double inv = ldexp(1.0, e);
        for (long i = 0; i < m; i++) u[i] = fma(inv, (double)d[i], u[i]);
        outer++;
    }
    st->iters = inner;
    st->outer = outer;
    st->extra_spmv = outer + 1;
    st->status = status;
    st->final_rr = rr;
    faces_free(F);
    free(kx); free(ky); free(kz); free(r); free(q64); free(d); free(ri); free(s); free(p); free(q); free(dg);
    return status;
}

void orc_ir_batch(const orc_problem *P, const double *mu, int nmu, const double *f, const double *u0,
                  int prec, double tol, double eta, int kin_max, int max_outer, int reliable, double *u,
                  orc_stats *st, int nthreads) {
    long m = ndof_of(P);
    int p = P->kind == ORC_BLOCKS ? P->nblocks : (P->kind == ORC_OCTANTS ? 8 : 24 + (P->f_kind == ORC_F_GAUSS ? 3 : 0));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int b = 0; b < nmu; b++)
        orc_ir_solve2(P, mu + (long)b * p, f + b * m, u0 ? u0 + b * m : NULL, prec, tol, eta, kin_max,
                      max_outer, reliable, u + b * m, st + b);
}

/* ------------------------------------------------------------------ */
/* L1-based reduced over-collocation, L1ROC (Sec. 3.1, Alg. 4)         */
/* ------------------------------------------------------------------ */
/* Readings:
 *  - DEIM vectors are normalised under point evaluation: B_j[pt_j] = 1 and
 *    B_j[pt_i] = 0 for i < j, so [B_j[pt_i]] is unit lower triangular.  A DEIM
 *    step interpolates x at the existing points (forward substitution), forms
 *    r = x - B c (zero at the existing points by construction, stored as exact
 *    zeros), takes the point of largest |r_i| (lowest index on ties) and the
 *    new vector r / r[pt].  Every sum is correctly rounded.
 *  - The online problem is a minimisation (the printed argmax is a typo):
 *    c = argmin || P (b - A(mu) W c) ||_2 over the distinct points of
 *    X = X_s u X_r in ascending grid order, by Householder QR.
 *  - The L1 indicator uses the coefficients in the basis of the snapshots
 *    themselves: W = U T with T upper triangular from the DEIM steps, so
 *    c_U = T c_W and Delta = sum_i |c_U,i|.
 *  - The first parameter is the training set's first (the set is seeded
 *    random); the greedy stops early when a parameter would be chosen twice
 *    or a snapshot's DEIM residual vanishes. */

/* (A(mu) x)_P at one unknown, with the order of apply_faces */
static double stencil_at(const faces *F, int n, const double *x, long P) {
    long n2 = (long)n * n;
    int i = (int)(P % n) + 1, j = (int)((P / n) % n) + 1, k = (int)(P / n2) + 1;
    double c[6];
    six(F, n, i, j, k, c);
    double acc = diag_of(c) * x[P];
    if (i > 1) acc = fma(-c[0], x[P - 1], acc);
    if (i < n) acc = fma(-c[1], x[P + 1], acc);
    if (j > 1) acc = fma(-c[2], x[P - n], acc);
    if (j < n) acc = fma(-c[3], x[P + n], acc);
    if (k > 1) acc = fma(-c[4], x[P - n2], acc);
    if (k < n) acc = fma(-c[5], x[P + n2], acc);
    return acc;
}

/* One DEIM step against the nb vectors B (rows of length m) and their points
 * pt.  Writes the interpolation coefficients c (nb), the new normalised vector
 * out and its scale *s = r[point]; returns the point, or -1 if r vanishes. */
static long deim_step(const double *B, const long *pt, int nb, long m, const double *x, double *c,
                      double *out, double *s) {
    for (int i = 0; i < nb; i++) {
        xacc a; xacc_clear(&a);
        xacc_add(&a, x[pt[i]]);
        for (int j = 0; j < i; j++) xacc_add_prod(&a, -B[(long)j * m + pt[i]], c[j]);
        c[i] = xacc_round(&a);
    }
    for (long k = 0; k < m; k++) {
        xacc a; xacc_clear(&a);
        xacc_add(&a, x[k]);
        for (int j = 0; j < nb; j++) xacc_add_prod(&a, -c[j], B[(long)j * m + k]);
        out[k] = xacc_round(&a);
    }
    for (int i = 0; i < nb; i++) out[pt[i]] = 0.0;
    long best = -1;
    double bv = 0.0;
    for (long k = 0; k < m; k++)
        if (fabs(out[k]) > bv) { bv = fabs(out[k]); best = k; }
    if (best < 0) return -1;
    *s = out[best];
    for (long k = 0; k < m; k++) out[k] = out[k] / *s;
    return best;
}

/* min || A c - b ||_2 for A (M x N row-major, overwritten), M >= N, by
 * Householder QR; b (M) is overwritten.  Returns -1 on a zero column. */
static int lsq_qr(int M, int N, double *A, double *b, double *c) {
    for (int k = 0; k < N; k++) {
        xacc a; xacc_clear(&a);
        for (int i = k; i < M; i++) xacc_add_prod(&a, A[(long)i * N + k], A[(long)i * N + k]);
        double nrm = sqrt(xacc_round(&a));
        if (!(nrm > 0.0)) return -1;
        double akk = A[(long)k * N + k];
        double alpha = akk > 0.0 ? -nrm : nrm;
        /* v = (akk - alpha, A[k+1..][k]); v^T v = 2 nrm (nrm + |akk|) */
        double vk = akk - alpha;
        double vtv = 2.0 * nrm * (nrm + fabs(akk));
        for (int j = k + 1; j <= N; j++) {            /* j == N: the right-hand side */
            xacc d; xacc_clear(&d);
            xacc_add_prod(&d, vk, j < N ? A[(long)k * N + j] : b[k]);
            for (int i = k + 1; i < M; i++) xacc_add_prod(&d, A[(long)i * N + k], j < N ? A[(long)i * N + j] : b[i]);
            double t = 2.0 * xacc_round(&d) / vtv;
            if (j < N) {
                A[(long)k * N + j] -= t * vk;
                for (int i = k + 1; i < M; i++) A[(long)i * N + j] -= t * A[(long)i * N + k];
            } else {
                b[k] -= t * vk;
                for (int i = k + 1; i < M; i++) b[i] -= t * A[(long)i * N + k];
            }
        }
        A[(long)k * N + k] = alpha;
    }
    for (int k = N - 1; k >= 0; k--) {
        xacc a; xacc_clear(&a);
        xacc_add(&a, b[k]);
        for (int j = k + 1; j < N; j++) xacc_add_prod(&a, -A[(long)k * N + j], c[j]);
        c[k] = xacc_round(&a) / A[(long)k * N + k];
    }
    return 0;
}

/* the collocation least-squares problem at mu: rows (A(mu) w_j)[x_i] and
 * f_h(x_i) for the npts points; c (nb).  Returns -1 on breakdown. */
static int l1roc_solve(const orc_problem *P, const double *mu, int nb, const double *W, const long *pts,
                       int npts, double *c) {
    long m = ndof_of(P);
    if (npts < nb) return -1;
    faces F = faces_for_mu(P, mu);
    double *A = malloc(sizeof(double) * npts * nb), *b = malloc(sizeof(double) * npts);
    double *f = malloc(sizeof(double) * m);
    orc_rhs(P, mu, f);
    for (int i = 0; i < npts; i++) {
        for (int j = 0; j < nb; j++) A[(long)i * nb + j] = stencil_at(&F, P->n, W + (long)j * m, pts[i]);
        b[i] = f[pts[i]];
    }
    int rc = lsq_qr(npts, nb, A, b, c);
    free(A); free(b); free(f);
    faces_free(F);
    return rc;
}

int orc_l1roc_coeffs(const orc_problem *P, int nb, const double *W, const long *pts, int npts,
                     const double *mu, double *c) {
    return l1roc_solve(P, mu, nb, W, pts, npts, c);
}

/* L1 indicator: || T c_W ||_1 with T (ld x ld, upper triangular) */
static double l1_indicator(int nb, int ld, const double *T, const double *cw) {
    double cu[128];
    for (int i = 0; i < nb; i++) {
        xacc a; xacc_clear(&a);
        for (int j = i; j < nb; j++) xacc_add_prod(&a, T[(long)i * ld + j], cw[j]);
        cu[i] = fabs(xacc_round(&a));
    }
    return orc_exact_sum(cu, nb);
}

static int cmp_long(const void *a, const void *b) {
    long x = *(const long *)a, y = *(const long *)b;
    return x < y ? -1 : x > y;
}

/* distinct points of Xs u Xr in ascending order */
static int point_set(const long *xs, int ns, const long *xr, int nr, long *out) {
    int k = 0;
    for (int i = 0; i < ns; i++) out[k++] = xs[i];
    for (int i = 0; i < nr; i++) out[k++] = xr[i];
    qsort(out, k, sizeof(long), cmp_long);
    int u = 0;
    for (int i = 0; i < k; i++)
        if (u == 0 || out[i] != out[u - 1]) out[u++] = out[i];
    return u;
}

/* Outputs: W (N x m), T (N x N), pts (2N) and *npts (the point set X), the
 * snapshot points xs (N) and residual points xr (N) with their counts nsr[2],
 * selected (N), hist (N x ntrain; row k = L1 indicator with k+1 vectors),
 * *nreached.  Returns 0, or -1 on a least-squares breakdown or N > 120. */
int orc_l1roc_greedy(const orc_problem *P, const double *mu_train, int ntrain, int N, double snap_tol,
                     int prec, int snap_maxit, double *W, double *T, long *pts, int *npts, long *xs,
                     long *xr, int *nsr, int *selected, double *hist, int *nreached, int nthreads) {
    if (N > 120) return -1;
    long m = ndof_of(P);
    int p = P->kind == ORC_BLOCKS ? P->nblocks : (P->kind == ORC_OCTANTS ? 8 : 24 + (P->f_kind == ORC_F_GAUSS ? 3 : 0));
    double *R = malloc(sizeof(double) * N * m);
    double *u = malloc(sizeof(double) * m), *f = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    double *tmp = malloc(sizeof(double) * m);
    double c[128], cl[128], s = 0.0;
    int ns = 0, nr = 0, nb = 0, rc = 0;
    memset(T, 0, sizeof(double) * N * N);
    *npts = 0;
    /* first snapshot */
    orc_rhs(P, mu_train, f);
    orc_stats st;
    orc_cg(P, mu_train, f, NULL, prec, snap_tol, snap_maxit, u, &st, NULL);
    long pt = deim_step(W, xs, 0, m, u, c, W, &s);
    if (pt >= 0) {
        T[0] = 1.0 / s;
        xs[ns++] = pt;
        selected[nb++] = 0;
        *npts = point_set(xs, ns, xr, nr, pts);
    }
    while (nb > 0) {
        double *row = hist + (long)(nb - 1) * ntrain;
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
        for (int b = 0; b < ntrain; b++) {
            double cw[128];
            if (l1roc_solve(P, mu_train + (long)b * p, nb, W, pts, *npts, cw) != 0) {
#pragma omp atomic write
                bad = 1;
                row[b] = NAN;
            } else {
                row[b] = l1_indicator(nb, N, T, cw);
            }
        }
        if (bad) { rc = -1; break; }
        if (nb == N) break;
        int best = 0;
        for (int b = 1; b < ntrain; b++) if (row[b] > row[best]) best = b;
        int dup = 0;
        for (int j = 0; j < nb; j++) if (selected[j] == best) dup = 1;
        if (dup) break;
        const double *mul = mu_train + (long)best * p;
        /* residual of the current approximation at the chosen parameter */
        if (l1roc_solve(P, mul, nb, W, pts, *npts, cl) != 0) { rc = -1; break; }
        orc_lift(nb, m, W, cl, tmp);
        orc_apply(P, mul, tmp, r);
        orc_rhs(P, mul, f);
        for (long i = 0; i < m; i++) r[i] = f[i] - r[i];
        /* the snapshot and its DEIM step */
        orc_cg(P, mul, f, NULL, prec, snap_tol, snap_maxit, u, &st, NULL);
        pt = deim_step(W, xs, nb, m, u, c, W + (long)nb * m, &s);
        if (pt < 0) break;
        /* W_new = (u - sum_j c_j W_j) / s  =>  T[:, nb] = (e_nb - sum_j c_j T[:, j]) / s */
        for (int i = 0; i < nb; i++) {
            xacc a; xacc_clear(&a);
            for (int j = i; j < nb; j++) xacc_add_prod(&a, -c[j], T[(long)i * N + j]);
            T[(long)i * N + nb] = xacc_round(&a) / s;
        }
        T[(long)nb * N + nb] = 1.0 / s;
        xs[ns++] = pt;
        /* the residual's DEIM step adds a second point */
        double sr = 0.0;
        long ptr = deim_step(R, xr, nr, m, r, c, R + (long)nr * m, &sr);
        if (ptr >= 0) xr[nr++] = ptr;
        selected[nb++] = best;
        *npts = point_set(xs, ns, xr, nr, pts);
    }
    *nreached = nb;
    nsr[0] = ns;
    nsr[1] = nr;
    free(R); free(u); free(f); free(r); free(tmp);
    return rc;
}
