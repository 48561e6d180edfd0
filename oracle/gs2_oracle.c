/*
 * CPU oracle for two-stage Gauss-Seidel (GS2) relaxation and GS2-preconditioned
 * restarted GMRES.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded
 * statement of what the HIP library computes.  Only the test suite, the smoke
 * check and the CPU baseline leg of the benchmark may load it; the library
 * never does.  It shares no code, header or table with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no OpenMP).
 * With contraction off every a*b+c is a rounded multiply then a rounded add,
 * and every row sum runs in CSR order, so results are reproducible.
 *
 * Matrix: CSR, 0-based int32 row pointers and column indices (sorted within a
 * row), float64 values, diagonal present.  Splitting A = L + D + U with L, U
 * the strictly lower / upper parts and D the diagonal (Section 3).
 *
 * Paper: Thomas et al., "Two-Stage Gauss-Seidel Preconditioners and Smoothers
 * for Krylov Solvers on a GPU cluster" (arXiv 2104.01196).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_FORWARD 0
#define OR_BACKWARD 1
#define OR_SYMMETRIC 2

#define OR_PREC_NONE 0
#define OR_PREC_GS2 1
#define OR_PREC_JR 2
#define OR_PREC_SOR 3
#define OR_PREC_MTGS 4

#define OR_FP64 0
#define OR_FP32 1
#define OR_FP16S 2

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_ZERO_DIAG (-3)
#define OR_ERR_NONFINITE (-4)
#define OR_ERR_NOMEM (-5)
#define OR_ERR_FP16_RANGE (-7)
#define OR_NOT_CONVERGED 1
#define OR_BREAKDOWN 2

typedef struct {
    int n;
    const int32_t *rp, *ci;
    const double *va;
} or_csr;

int or_mtgs_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int variant, int sweeps, double w,
                  const double *b, double *x);
int or_gs2_block_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int blocks, int variant,
                       int sweeps, int local_sweeps, int inner, double w, double gamma, const double *b, double *x);

/* ------------------------------------------------------------------ basics */

/* y = A x, each row summed in CSR order. */
void or_spmv(int n, const int32_t *rp, const int32_t *ci, const double *va, const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) s += va[k] * x[ci[k]];
        y[i] = s;
    }
}

/* Diagonal of A (Section 3 splitting).  Missing or zero entry: error. */
int or_diag(int n, const int32_t *rp, const int32_t *ci, const double *va, double *d)
{
    for (int i = 0; i < n; ++i) {
        d[i] = 0.0;
        int found = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) { d[i] = va[k]; found = 1; }
        if (!found || d[i] == 0.0) return OR_ERR_ZERO_DIAG;
        if (!isfinite(d[i])) return OR_ERR_NONFINITE;
    }
    return OR_OK;
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

/* --------------------------------------------------- GS2, FP64 (Section 4)
 *
 * One "half" of a two-stage sweep, non-compact form, eq. (two-stage):
 *   r = b - A x                                   (outer residual)
 *   g0 = D^{-1} r                                 eq. (jr-initial-guess)
 *   g_{j+1} = D^{-1}(r - w T g_j), j < inner      eq. (jacobi), with the
 *                                                  damped splitting D + wL
 *   x = x + w g_inner                             (damped update, Section 4)
 * T is L for a forward half and U for a backward half.  With inner damping
 * gamma the inner step is g_{j+1} = (1-gamma) g_j + gamma D^{-1}(r - w T g_j)
 * (Section 4, damping factor).  inner = 0 gives Jacobi-Richardson.
 */
static void gs2_half(const or_csr *A, const double *d, int lower, int inner, double w, double gamma,
                     const double *b, double *x, double *r, double *g, double *gn)
{
    const int n = A->n;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) s += A->va[k] * x[A->ci[k]];
        r[i] = b[i] - s;
    }
    for (int i = 0; i < n; ++i) g[i] = r[i] / d[i];
    for (int j = 0; j < inner; ++j) {
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
                int c = A->ci[k];
                if (lower ? (c < i) : (c > i)) s += A->va[k] * g[c];
            }
            double jac = (r[i] - w * s) / d[i];
            gn[i] = (gamma == 1.0) ? jac : (1.0 - gamma) * g[i] + gamma * jac;
        }
        double *t = g; g = gn; gn = t;
    }
    for (int i = 0; i < n; ++i) x[i] = x[i] + w * g[i];
}

/*
 * Stand-alone GS2 iteration (Fig. code:two-stage with n_k = 1 on one process):
 * `sweeps` outer sweeps on A x = b starting from the x passed in.  A symmetric
 * sweep is a forward half then a backward half; the backward residual uses the
 * x produced by the forward half, as the composed SGS2 residual operator of
 * Section 5 requires.  Both halves run exactly `inner` inner sweeps.
 */
int or_gs2_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int variant, int sweeps,
                 int inner, double w, double gamma, const double *b, double *x)
{
    if (n < 0 || sweeps < 0 || inner < 0 || variant < 0 || variant > 2) return OR_ERR_ARG;
    or_csr A = {n, rp, ci, va};
    double *d = malloc(sizeof(double) * (size_t)n * 4 + 8);
    if (!d) return OR_ERR_NOMEM;
    double *r = d + n, *g = r + n, *gn = g + n;
    int st = or_diag(n, rp, ci, va, d);
    if (st == OR_OK) {
        for (int t = 0; t < sweeps; ++t) {
            if (variant != OR_BACKWARD) gs2_half(&A, d, 1, inner, w, gamma, b, x, r, g, gn);
            if (variant != OR_FORWARD) gs2_half(&A, d, 0, inner, w, gamma, b, x, r, g, gn);
        }
    }
    free(d);
    return st;
}

/* Preconditioner form: z = GS2 applied to v from a zero initial guess. */
int or_gs2_apply(int n, const int32_t *rp, const int32_t *ci, const double *va, int variant, int sweeps,
                 int inner, double w, double gamma, const double *v, double *z)
{
    memset(z, 0, sizeof(double) * (size_t)n);
    return or_gs2_sweep(n, rp, ci, va, variant, sweeps, inner, w, gamma, v, z);
}

/*
 * Compact two-stage form, eq. (two-stage-3) with damping (Section 4):
 *   x_{k+1} = w (D + wL)^{-1} (b - [U + (1 - 1/w) D] x_k)
 * where the approximate inverse is `inner` JR steps from g0 = D^{-1} r.
 * Backward halves swap L and U.
 */
static void gs2c_half(const or_csr *A, const double *d, int lower, int inner, double w, double gamma,
                      const double *b, double *x, double *r, double *g, double *gn)
{
    const int n = A->n;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int c = A->ci[k];
            if (lower ? (c > i) : (c < i)) s += A->va[k] * x[c];
        }
        r[i] = b[i] - s - (1.0 - 1.0 / w) * d[i] * x[i];
    }
    for (int i = 0; i < n; ++i) g[i] = r[i] / d[i];
    for (int j = 0; j < inner; ++j) {
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
                int c = A->ci[k];
                if (lower ? (c < i) : (c > i)) s += A->va[k] * g[c];
            }
            double jac = (r[i] - w * s) / d[i];
            gn[i] = (gamma == 1.0) ? jac : (1.0 - gamma) * g[i] + gamma * jac;
        }
        double *t = g; g = gn; gn = t;
    }
    for (int i = 0; i < n; ++i) x[i] = w * g[i];
}

int or_gs2c_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int variant, int sweeps,
                  int inner, double w, double gamma, const double *b, double *x)
{
    if (n < 0 || sweeps < 0 || inner < 0 || variant < 0 || variant > 2) return OR_ERR_ARG;
    or_csr A = {n, rp, ci, va};
    double *d = malloc(sizeof(double) * (size_t)n * 4 + 8);
    if (!d) return OR_ERR_NOMEM;
    double *r = d + n, *g = r + n, *gn = g + n;
    int st = or_diag(n, rp, ci, va, d);
    if (st == OR_OK) {
        for (int t = 0; t < sweeps; ++t) {
            if (variant != OR_BACKWARD) gs2c_half(&A, d, 1, inner, w, gamma, b, x, r, g, gn);
            if (variant != OR_FORWARD) gs2c_half(&A, d, 0, inner, w, gamma, b, x, r, g, gn);
        }
    }
    free(d);
    return st;
}

/*
 * Jacobi-Richardson, the n_j = 0 case of GS2 (Section 4):
 *   x = x + w D^{-1}(b - A x), `sweeps` times.
 */
int or_jr_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int sweeps, double w,
                const double *b, double *x)
{
    double *d = malloc(sizeof(double) * (size_t)n * 2 + 8);
    if (!d) return OR_ERR_NOMEM;
    double *r = d + n;
    int st = or_diag(n, rp, ci, va, d);
    for (int t = 0; st == OR_OK && t < sweeps; ++t) {
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = rp[i]; k < rp[i + 1]; ++k) s += va[k] * x[ci[k]];
            r[i] = b[i] - s;
        }
        for (int i = 0; i < n; ++i) x[i] = x[i] + w * (r[i] / d[i]);
    }
    free(d);
    return st;
}

/*
 * Classical (one-stage) Gauss-Seidel / SOR as the sequential in-place row loop
 * of Section 6 (sequential Gauss-Seidel), compact form eq. (one-stage-2), with
 * damping w:  x_i = (1 - w) x_i + w (b_i - sum_{j != i} a_ij x_j) / a_ii,
 * rows ascending (forward) or descending (backward); symmetric = forward then
 * backward.  w = 1 is plain Gauss-Seidel.
 */
int or_sor_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int variant, int sweeps,
                 double w, const double *b, double *x)
{
    double *d = malloc(sizeof(double) * (size_t)n + 8);
    if (!d) return OR_ERR_NOMEM;
    int st = or_diag(n, rp, ci, va, d);
    for (int t = 0; st == OR_OK && t < sweeps; ++t) {
        for (int pass = 0; pass < 2; ++pass) {
            int fwd = (pass == 0);
            if (fwd && variant == OR_BACKWARD) continue;
            if (!fwd && variant == OR_FORWARD) continue;
            for (int q = 0; q < n; ++q) {
                int i = fwd ? q : n - 1 - q;
                double s = 0.0;
                for (int k = rp[i]; k < rp[i + 1]; ++k)
                    if (ci[k] != i) s += va[k] * x[ci[k]];
                x[i] = (1.0 - w) * x[i] + w * ((b[i] - s) / d[i]);
            }
        }
    }
    free(d);
    return st;
}

/*
 * Level sets of the dependency DAG of L (lower = 1) or U (lower = 0):
 * level_i = 1 + max level_j over the entries a_ij of the triangle (0 if the
 * row has none).  Rows of one level can be solved in parallel (level-set
 * scheduling, Section 3).  Returns the number of levels; the longest path in
 * the DAG is that number minus one.
 */
int or_levels(int n, const int32_t *rp, const int32_t *ci, int lower, int32_t *level)
{
    int nlev = 0;
    for (int q = 0; q < n; ++q) {
        int i = lower ? q : n - 1 - q;
        int lv = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            int c = ci[k];
            if (lower ? (c < i) : (c > i)) if (level[c] + 1 > lv) lv = level[c] + 1;
        }
        level[i] = lv;
        if (lv + 1 > nlev) nlev = lv + 1;
    }
    return nlev;
}

/*
 * Inner-iteration diagnostic of Section 8 (inner JR convergence): for a fixed
 * r, the relative residual ||r - (wL + D) g_j|| / ||r|| of the lower
 * triangular system after j = 0..inner inner steps.  out has inner+1 entries.
 */
int or_inner_residuals(int n, const int32_t *rp, const int32_t *ci, const double *va, int inner, double w,
                       const double *r, double *out)
{
    double *d = malloc(sizeof(double) * (size_t)n * 4 + 8);
    if (!d) return OR_ERR_NOMEM;
    double *g = d + n, *gn = g + n, *t = gn + n;
    int st = or_diag(n, rp, ci, va, d);
    double rn = nrm2(n, r);
    for (int i = 0; st == OR_OK && i < n; ++i) g[i] = r[i] / d[i];
    for (int j = 0; st == OR_OK && j <= inner; ++j) {
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] < i) s += va[k] * g[ci[k]];
            t[i] = r[i] - (w * s + d[i] * g[i]);
        }
        out[j] = nrm2(n, t) / rn;
        if (j == inner) break;
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] < i) s += va[k] * g[ci[k]];
            gn[i] = (r[i] - w * s) / d[i];
        }
        double *tt = g; g = gn; gn = tt;
    }
    free(d);
    return st;
}

/* ------------------------------------------- reduced-precision preconditioner
 *
 * The paper runs the preconditioner in single precision while the Krylov
 * solver stays in double (Section 10).  Its GS2 code keeps D^{-1}L prescaled
 * (Section 6, two-stage Gauss-Seidel).  The reduced-precision forms here are
 * defined in symmetrically scaled variables, which GS2 is invariant under in
 * exact arithmetic:
 *   s_r[i] = 1/sqrt(|a_ii|), s_l[i] = sign(a_ii) s_r[i]      (float64)
 *   Ah_ij  = round_p((s_l[i] * a_ij) * s_r[j]),  i != j        (unit diagonal)
 * with round_p = round to binary32 (FP32 form) or binary16 (FP16 form,
 * round to nearest even).  Then, all in binary32 arithmetic:
 *   rh = round32(v_i * s_l[i]) - xh_i - sum_{j != i} Ah_ij xh_j   (CSR order)
 *   g0 = rh;  g_{j+1} = rh - w * sum_{T} Ah_ij g_j
 *   (with inner damping gamma != 1, Section 9: g_{j+1} = (1 - gamma) g_j +
 *    gamma (rh - w * sum_{T} Ah_ij g_j), the float64 form's update in
 *    scaled variables, where D^{-1} is the identity)
 *   xh = xh + w g
 * and the output is z_i = (double) xh_i * s_r[i] in float64.  The first
 * residual of an apply from zero is round32(v_i s_l[i]) exactly.
 */

/* binary16 round-to-nearest-even of a double, returned as a double.  Written
 * from the IEEE 754 binary16 format: 10 fraction bits, exponent range
 * [-14, 15], subnormal quantum 2^-24, overflow to infinity at 65520. */
double or_round_f16(double x)
{
    if (isnan(x)) return x;
    double ax = fabs(x);
    if (ax >= 65520.0) return copysign(INFINITY, x);
    if (ax == 0.0) return x;
    int e;
    frexp(ax, &e); /* ax in [2^(e-1), 2^e) */
    int E = e - 1;
    if (E < -14) E = -14;
    double q = ldexp(1.0, E - 10);
    double m = rint(ax / q); /* default rounding mode: nearest even */
    double r = m * q;
    return copysign(r, x);
}

typedef struct {
    int n;
    int32_t *rp, *ci; /* off-diagonal pattern only */
    float *va;
    double *sl, *sr;
    float w, gamma;
} or_scaled;

static void scaled_free(or_scaled *S)
{
    free(S->rp); free(S->ci); free(S->va); free(S->sl); free(S->sr);
    memset(S, 0, sizeof(*S));
}

static int scaled_build(const or_csr *A, int precision, double w, double gamma, or_scaled *S)
{
    const int n = A->n;
    memset(S, 0, sizeof(*S));
    S->n = n;
    S->w = (float)w;
    S->gamma = (float)gamma;
    int64_t nnz = A->rp[n];
    S->rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    S->ci = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    S->va = malloc(sizeof(float) * (size_t)(nnz + 1));
    S->sl = malloc(sizeof(double) * (size_t)(n + 1));
    S->sr = malloc(sizeof(double) * (size_t)(n + 1));
    if (!S->rp || !S->ci || !S->va || !S->sl || !S->sr) { scaled_free(S); return OR_ERR_NOMEM; }
    double *d = malloc(sizeof(double) * (size_t)(n + 1));
    if (!d) { scaled_free(S); return OR_ERR_NOMEM; }
    int st = or_diag(n, A->rp, A->ci, A->va, d);
    if (st != OR_OK) { free(d); scaled_free(S); return st; }
    for (int i = 0; i < n; ++i) {
        S->sr[i] = 1.0 / sqrt(fabs(d[i]));
        S->sl[i] = d[i] < 0.0 ? -S->sr[i] : S->sr[i];
    }
    int32_t p = 0;
    S->rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int c = A->ci[k];
            if (c == i) continue;
            double s = (S->sl[i] * A->va[k]) * S->sr[c];
            double q = (precision == OR_FP16S) ? or_round_f16(s) : (double)(float)s;
            if (!isfinite(q)) { free(d); scaled_free(S); return precision == OR_FP16S ? OR_ERR_FP16_RANGE : OR_ERR_NONFINITE; }
            S->ci[p] = c;
            S->va[p] = (float)q;
            ++p;
        }
        S->rp[i + 1] = p;
    }
    free(d);
    return OR_OK;
}

static void scaled_half(const or_scaled *S, int lower, int inner, int from_zero, const double *v, float *xh,
                        float *r, float *g, float *gn)
{
    const int n = S->n;
    const float w = S->w, gamma = S->gamma;
    for (int i = 0; i < n; ++i) {
        float base = (float)(v[i] * S->sl[i]);
        if (from_zero) { r[i] = base; continue; }
        float s = base - xh[i];
        for (int k = S->rp[i]; k < S->rp[i + 1]; ++k) s = s - S->va[k] * xh[S->ci[k]];
        r[i] = s;
    }
    for (int i = 0; i < n; ++i) g[i] = r[i];
    for (int j = 0; j < inner; ++j) {
        for (int i = 0; i < n; ++i) {
            float s = 0.0f;
            for (int k = S->rp[i]; k < S->rp[i + 1]; ++k) {
                int c = S->ci[k];
                if (lower ? (c < i) : (c > i)) s = s + S->va[k] * g[c];
            }
            const float jac = r[i] - w * s;
            gn[i] = (gamma == 1.0f) ? jac : (1.0f - gamma) * g[i] + gamma * jac;
        }
        float *t = g; g = gn; gn = t;
    }
    for (int i = 0; i < n; ++i) xh[i] = xh[i] + w * g[i];
}

static int scaled_apply(const or_scaled *S, int variant, int sweeps, int inner, const double *v, double *z,
                        float *work)
{
    const int n = S->n;
    float *xh = work, *r = xh + n, *g = r + n, *gn = g + n;
    for (int i = 0; i < n; ++i) xh[i] = 0.0f;
    int first = 1;
    for (int t = 0; t < sweeps; ++t) {
        if (variant != OR_BACKWARD) { scaled_half(S, 1, inner, first, v, xh, r, g, gn); first = 0; }
        if (variant != OR_FORWARD) { scaled_half(S, 0, inner, first, v, xh, r, g, gn); first = 0; }
    }
    for (int i = 0; i < n; ++i) z[i] = (double)xh[i] * S->sr[i];
    return OR_OK;
}

/* Reduced-precision GS2 apply (FP32 or FP16-scaled form, inner damping
 * gamma), zero initial guess. */
int or_gs2_apply_lp(int n, const int32_t *rp, const int32_t *ci, const double *va, int precision, int variant,
                    int sweeps, int inner, double w, double gamma, const double *v, double *z)
{
    if (precision != OR_FP32 && precision != OR_FP16S) return OR_ERR_ARG;
    or_csr A = {n, rp, ci, va};
    or_scaled S;
    int st = scaled_build(&A, precision, w, gamma, &S);
    if (st != OR_OK) return st;
    float *work = malloc(sizeof(float) * (size_t)n * 4 + 16);
    if (!work) { scaled_free(&S); return OR_ERR_NOMEM; }
    st = scaled_apply(&S, variant, sweeps, inner, v, z, work);
    free(work);
    scaled_free(&S);
    return st;
}

/* ------------------------------------------------------------------ GMRES
 *
 * Restarted GMRES(m), right-preconditioned in the flexible form that stores
 * Z = [M^{-1} v_j] (so x = x0 + Z y matches what the Arnoldi process saw),
 * modified Gram-Schmidt (or CGS2) Arnoldi, Givens rotations on the
 * Hessenberg matrix.  The Krylov solver is the outer loop the paper pairs
 * with GS2 (Sections 1 and 8).
 *
 * Stopping: a cycle ends when |g_{j+1}| <= rtol ||b|| (the residual estimate),
 * when h_{j+1,j} <= 1e-14 ||A z_j|| (breakdown: the Krylov space is
 * invariant), when j = m, or when maxit Arnoldi steps have run.  After each
 * cycle x += Z y and the true residual ||b - A x|| / ||b|| decides
 * convergence.  iterations counts Arnoldi steps (preconditioner applications
 * inside cycles).
 */
typedef struct {
    int kind;      /* OR_PREC_* */
    int variant;   /* forward / backward / symmetric */
    int sweeps;
    int inner;
    double omega;
    double gamma;
    int precision; /* OR_FP64 / OR_FP32 / OR_FP16S (GS2 and JR only) */
    int compact;   /* GS2 compact form (FP64 only) */
    int blocks;    /* hybrid relaxation: row blocks (<= 1: global), FP64 GS2 / JR */
    int local_sweeps;
} or_prec;

typedef struct {
    int iterations;
    int restarts;
    double relres;
    int converged;
    int status;
} or_info;

typedef struct {
    const or_prec *P;
    const or_csr *A;
    or_scaled S;
    int have_scaled;
    float *work;
} prec_ctx;

static int prec_apply(prec_ctx *C, const double *v, double *z)
{
    const or_prec *P = C->P;
    const or_csr *A = C->A;
    const int n = A->n;
    switch (P->kind) {
    case OR_PREC_NONE:
        memcpy(z, v, sizeof(double) * (size_t)n);
        return OR_OK;
    case OR_PREC_GS2:
    case OR_PREC_JR: {
        int inner = P->kind == OR_PREC_JR ? 0 : P->inner;
        int variant = P->kind == OR_PREC_JR ? OR_FORWARD : P->variant;
        if (C->have_scaled) return scaled_apply(&C->S, variant, P->sweeps, inner, v, z, C->work);
        memset(z, 0, sizeof(double) * (size_t)n);
        if (P->blocks > 1)
            return or_gs2_block_sweep(n, A->rp, A->ci, A->va, P->blocks, variant, P->sweeps,
                                      P->local_sweeps > 1 ? P->local_sweeps : 1, inner, P->omega, P->gamma, v, z);
        if (P->kind == OR_PREC_JR) return or_jr_sweep(n, A->rp, A->ci, A->va, P->sweeps, P->omega, v, z);
        if (P->compact) return or_gs2c_sweep(n, A->rp, A->ci, A->va, variant, P->sweeps, inner, P->omega, P->gamma, v, z);
        return or_gs2_sweep(n, A->rp, A->ci, A->va, variant, P->sweeps, inner, P->omega, P->gamma, v, z);
    }
    case OR_PREC_SOR:
        memset(z, 0, sizeof(double) * (size_t)n);
        return or_sor_sweep(n, A->rp, A->ci, A->va, P->variant, P->sweeps, P->omega, v, z);
    case OR_PREC_MTGS:
        memset(z, 0, sizeof(double) * (size_t)n);
        return or_mtgs_sweep(n, A->rp, A->ci, A->va, P->variant, P->sweeps, P->omega, v, z);
    }
    return OR_ERR_ARG;
}

int or_gmres(int n, const int32_t *rp, const int32_t *ci, const double *va, const double *b, double *x, int m,
             double rtol, int maxit, const or_prec *P, int cgs2, or_info *info, double *hist)
{
    or_csr A = {n, rp, ci, va};
    memset(info, 0, sizeof(*info));
    if (n <= 0 || m <= 0 || maxit < 0) return info->status = OR_ERR_ARG;
    for (int i = 0; i < n; ++i)
        if (!isfinite(b[i]) || !isfinite(x[i])) return info->status = OR_ERR_NONFINITE;
    prec_ctx C;
    memset(&C, 0, sizeof(C));
    C.P = P;
    C.A = &A;
    if ((P->kind == OR_PREC_GS2 || P->kind == OR_PREC_JR) && P->precision != OR_FP64) {
        /* the reduced-precision forms are defined for the non-compact, single-block sweep only */
        if (P->compact || P->blocks > 1) return info->status = OR_ERR_ARG;
        int st = scaled_build(&A, P->precision, P->omega, P->gamma, &C.S);
        if (st != OR_OK) return info->status = st;
        C.have_scaled = 1;
        C.work = malloc(sizeof(float) * (size_t)n * 4 + 16);
        if (!C.work) { scaled_free(&C.S); return info->status = OR_ERR_NOMEM; }
    }
    size_t N = (size_t)n;
    double *V = malloc(sizeof(double) * N * (size_t)(m + 1));
    double *Z = malloc(sizeof(double) * N * (size_t)m);
    double *w = malloc(sizeof(double) * N);
    double *H = calloc((size_t)(m + 1) * (size_t)m, sizeof(double)); /* H[k*m + j] */
    double *cs = malloc(sizeof(double) * (size_t)m), *sn = malloc(sizeof(double) * (size_t)m);
    double *g = malloc(sizeof(double) * (size_t)(m + 1)), *y = malloc(sizeof(double) * (size_t)m);
    double *hc = malloc(sizeof(double) * (size_t)(m + 1));
    int status = OR_OK;
    int total = 0, cycles = 0;
    double bnorm = 0.0;
    if (!V || !Z || !w || !H || !cs || !sn || !g || !y || !hc) { status = OR_ERR_NOMEM; goto done; }

    bnorm = nrm2(n, b);
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * N);
        info->converged = 1;
        info->relres = 0.0;
        goto done;
    }
    for (;;) {
        /* true residual */
        or_spmv(n, rp, ci, va, x, w);
        for (int i = 0; i < n; ++i) w[i] = b[i] - w[i];
        double beta = nrm2(n, w);
        info->relres = beta / bnorm;
        if (hist) hist[total] = info->relres;
        if (!isfinite(beta)) { status = OR_ERR_NONFINITE; break; }
        if (info->relres <= rtol) { info->converged = 1; break; }
        if (total >= maxit) { status = OR_NOT_CONVERGED; break; }
        if (cycles > 0) info->restarts++;
        cycles++;
        for (int i = 0; i < n; ++i) V[i] = w[i] / beta;
        memset(g, 0, sizeof(double) * (size_t)(m + 1));
        g[0] = beta;
        int kk = 0;
        int breakdown = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N;
            int st = prec_apply(&C, vj, zj);
            if (st != OR_OK) { status = st; goto done; }
            or_spmv(n, rp, ci, va, zj, w);
            double wnorm0 = nrm2(n, w);
            if (cgs2) {
                for (int k = 0; k <= j; ++k) hc[k] = 0.0;
                for (int pass = 0; pass < 2; ++pass) {
                    double hh[1024];
                    double *h = (j + 1 <= 1024) ? hh : malloc(sizeof(double) * (size_t)(j + 1));
                    for (int k = 0; k <= j; ++k) h[k] = dot(n, V + (size_t)k * N, w);
                    for (int k = 0; k <= j; ++k) {
                        const double *vk = V + (size_t)k * N;
                        for (int i = 0; i < n; ++i) w[i] = w[i] - h[k] * vk[i];
                        hc[k] += h[k];
                    }
                    if (h != hh) free(h);
                }
            } else {
                for (int k = 0; k <= j; ++k) {
                    const double *vk = V + (size_t)k * N;
                    double h = dot(n, vk, w);
                    for (int i = 0; i < n; ++i) w[i] = w[i] - h * vk[i];
                    hc[k] = h;
                }
            }
            double hnext = nrm2(n, w);
            total++;
            /* apply previous rotations, then a new one */
            for (int k = 0; k < j; ++k) {
                double t = cs[k] * hc[k] + sn[k] * hc[k + 1];
                hc[k + 1] = -sn[k] * hc[k] + cs[k] * hc[k + 1];
                hc[k] = t;
            }
            double rho = hypot(hc[j], hnext);
            if (!isfinite(rho) || !isfinite(hnext)) { status = OR_ERR_NONFINITE; goto done; }
            if (rho == 0.0) { status = OR_BREAKDOWN; goto done; }
            cs[j] = hc[j] / rho;
            sn[j] = hnext / rho;
            hc[j] = rho;
            for (int k = 0; k <= j; ++k) H[(size_t)k * m + j] = hc[k];
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            kk = j + 1;
            breakdown = hnext <= 1e-14 * wnorm0;
            if (!breakdown)
                for (int i = 0; i < n; ++i) V[(size_t)(j + 1) * N + i] = w[i] / hnext;
            if (hist) hist[total] = fabs(g[j + 1]) / bnorm;
            if (fabs(g[j + 1]) <= rtol * bnorm || breakdown || total >= maxit) break;
        }
        /* y = R^{-1} g, x += Z y */
        for (int k = kk - 1; k >= 0; --k) {
            double s = g[k];
            for (int l = k + 1; l < kk; ++l) s -= H[(size_t)k * m + l] * y[l];
            y[k] = s / H[(size_t)k * m + k];
        }
        for (int k = 0; k < kk; ++k) {
            const double *zk = Z + (size_t)k * N;
            for (int i = 0; i < n; ++i) x[i] = x[i] + y[k] * zk[i];
        }
        (void)breakdown;
    }
done:
    info->iterations = total;
    if (status == OR_OK && !info->converged) status = OR_NOT_CONVERGED;
    if (info->converged) status = OR_OK;
    info->status = status;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y); free(hc);
    if (C.have_scaled) { scaled_free(&C.S); free(C.work); }
    return status;
}

/* ------------------------------------------- hybrid (block-Jacobi) GS2
 *
 * The hybrid relaxation of Section 3 on P contiguous row blocks of size
 * ceil(n/P) (the rows one process would own): in each of n_t global sweeps
 * the values outside a row's block are frozen (y = x, the neighbourhood
 * exchange), then n_k local sweeps run on the block system
 * A_loc x = b - E y, each a GS2 half (or a forward and a backward half)
 * whose inner JR sweeps use only the block's own triangle.  Coupling to
 * other blocks enters only through the frozen y (the multiple local sweeps
 * with a frozen halo of Section 3).  The interface is exchanged once per
 * global sweep (Fig. code:two-stage), so the backward half of a symmetric
 * sweep also sees the frozen values.  P = 1 is plain GS2; a global sweep of a
 * single forward or backward half uses the global residual b - A x.
 */
static void block_half(const or_csr *A, const double *d, int bs, int lower, int inner, double w, double gamma,
                       const double *b, const double *y, double *x, double *r, double *g, double *gn)
{
    const int n = A->n;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int c = A->ci[k];
            s += A->va[k] * ((c / bs == i / bs) ? x[c] : y[c]);
        }
        r[i] = b[i] - s;
    }
    for (int i = 0; i < n; ++i) g[i] = r[i] / d[i];
    for (int j = 0; j < inner; ++j) {
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
                int c = A->ci[k];
                if (c / bs == i / bs && (lower ? (c < i) : (c > i))) s += A->va[k] * g[c];
            }
            double jac = (r[i] - w * s) / d[i];
            gn[i] = (gamma == 1.0) ? jac : (1.0 - gamma) * g[i] + gamma * jac;
        }
        double *t = g; g = gn; gn = t;
    }
    for (int i = 0; i < n; ++i) x[i] = x[i] + w * g[i];
}

int or_gs2_block_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int blocks, int variant,
                       int sweeps, int local_sweeps, int inner, double w, double gamma, const double *b, double *x)
{
    if (n <= 0 || blocks < 1 || sweeps < 0 || local_sweeps < 1 || inner < 0 || variant < 0 || variant > 2)
        return OR_ERR_ARG;
    or_csr A = {n, rp, ci, va};
    const int bs = (n + blocks - 1) / blocks;
    double *d = malloc(sizeof(double) * (size_t)n * 5 + 8);
    if (!d) return OR_ERR_NOMEM;
    double *r = d + n, *g = r + n, *gn = g + n, *y = gn + n;
    int st = or_diag(n, rp, ci, va, d);
    for (int t = 0; st == OR_OK && t < sweeps; ++t) {
        memcpy(y, x, sizeof(double) * (size_t)n); /* exchange: freeze off-block values */
        for (int k = 0; k < local_sweeps; ++k) {
            if (variant != OR_BACKWARD) block_half(&A, d, bs, 1, inner, w, gamma, b, y, x, r, g, gn);
            if (variant != OR_FORWARD) block_half(&A, d, bs, 0, inner, w, gamma, b, y, x, r, g, gn);
        }
    }
    free(d);
    return st;
}

/* ------------------------------------------------------- multicolor GS
 *
 * Multicolor Gauss-Seidel (Section 6, multi-threaded Gauss-Seidel): rows get
 * colors such that two rows of one color are never coupled (a_ij = a_ji = 0);
 * colors are then swept one after the other and the rows of a color are
 * independent.  Coloring: greedy first fit in natural row order on the
 * symmetrised pattern (row i takes the smallest color not used by any
 * earlier row j < i with a_ij != 0 or a_ji != 0).  Returns the color count.
 */
int or_colors(int n, const int32_t *rp, const int32_t *ci, int32_t *color)
{
    /* transpose pattern to see a_ji */
    int32_t *tp = calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *tc = malloc(sizeof(int32_t) * ((size_t)rp[n] + 1));
    int32_t *fill = malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *mark = malloc(sizeof(int32_t) * ((size_t)n + 2));
    if (!tp || !tc || !fill || !mark) { free(tp); free(tc); free(fill); free(mark); return OR_ERR_NOMEM; }
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) tp[ci[k] + 1]++;
    for (int i = 0; i < n; ++i) tp[i + 1] += tp[i];
    for (int i = 0; i < n; ++i) fill[i] = tp[i];
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) tc[fill[ci[k]]++] = i;
    for (int c = 0; c <= n; ++c) mark[c] = -1;
    int ncol = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] < i) mark[color[ci[k]]] = i;
        for (int k = tp[i]; k < tp[i + 1]; ++k)
            if (tc[k] < i) mark[color[tc[k]]] = i;
        int c = 0;
        while (mark[c] == i) ++c;
        color[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(tp); free(tc); free(fill); free(mark);
    return ncol;
}

/* Multicolor GS/SOR sweeps: colors ascending (forward), descending
 * (backward) or both (symmetric); within a color every row takes the same
 * damped update as the sequential loop, x_i = (1-w) x_i + w (b_i -
 * sum_{j != i} a_ij x_j) / a_ii. */
int or_mtgs_sweep(int n, const int32_t *rp, const int32_t *ci, const double *va, int variant, int sweeps, double w,
                  const double *b, double *x)
{
    int32_t *color = malloc(sizeof(int32_t) * ((size_t)n + 1));
    double *d = malloc(sizeof(double) * ((size_t)n + 1));
    if (!color || !d) { free(color); free(d); return OR_ERR_NOMEM; }
    int st = or_diag(n, rp, ci, va, d);
    int ncol = st == OR_OK ? or_colors(n, rp, ci, color) : 0;
    if (ncol < 0) st = ncol;
    for (int t = 0; st == OR_OK && t < sweeps; ++t) {
        for (int pass = 0; pass < 2; ++pass) {
            int fwd = (pass == 0);
            if (fwd && variant == OR_BACKWARD) continue;
            if (!fwd && variant == OR_FORWARD) continue;
            for (int q = 0; q < ncol; ++q) {
                int c = fwd ? q : ncol - 1 - q;
                for (int i = 0; i < n; ++i) {
                    if (color[i] != c) continue;
                    double s = 0.0;
                    for (int k = rp[i]; k < rp[i + 1]; ++k)
                        if (ci[k] != i) s += va[k] * x[ci[k]];
                    x[i] = (1.0 - w) * x[i] + w * ((b[i] - s) / d[i]);
                }
            }
        }
    }
    free(color);
    free(d);
    return st;
}

/* ---------------------------------------------------------------------- CG
 *
 * Preconditioned conjugate gradients (the Krylov solver of the paper's
 * symmetric positive definite experiments, Sections 9 and 10) in the
 * textbook form:
 *   r = b - A x, z = M^{-1} r, p = z, rz = r.z
 *   repeat: q = A p, alpha = rz / p.q, x += alpha p, r -= alpha q,
 *           stop if ||r|| <= rtol ||b||, z = M^{-1} r, beta = r.z_new / rz,
 *           p = z + beta p
 * The recurrence residual decides when to stop; the true residual is then
 * checked and, if it has drifted above rtol, the iteration restarts from it.
 * iterations counts preconditioner applications after the first
 * (= the number of A p products).
 */
int or_pcg(int n, const int32_t *rp, const int32_t *ci, const double *va, const double *b, double *x, double rtol,
           int maxit, const or_prec *P, or_info *info)
{
    or_csr A = {n, rp, ci, va};
    memset(info, 0, sizeof(*info));
    if (n <= 0 || maxit < 0) return info->status = OR_ERR_ARG;
    for (int i = 0; i < n; ++i)
        if (!isfinite(b[i]) || !isfinite(x[i])) return info->status = OR_ERR_NONFINITE;
    prec_ctx C;
    memset(&C, 0, sizeof(C));
    C.P = P;
    C.A = &A;
    if ((P->kind == OR_PREC_GS2 || P->kind == OR_PREC_JR) && P->precision != OR_FP64) {
        /* the reduced-precision forms are defined for the non-compact, single-block sweep only */
        if (P->compact || P->blocks > 1) return info->status = OR_ERR_ARG;
        int st = scaled_build(&A, P->precision, P->omega, P->gamma, &C.S);
        if (st != OR_OK) return info->status = st;
        C.have_scaled = 1;
        C.work = malloc(sizeof(float) * (size_t)n * 4 + 16);
        if (!C.work) { scaled_free(&C.S); return info->status = OR_ERR_NOMEM; }
    }
    size_t N = (size_t)n;
    double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
    int status = OR_OK, total = 0;
    double bnorm = 0.0;
    if (!r || !z || !p || !q) { status = OR_ERR_NOMEM; goto done; }
    bnorm = nrm2(n, b);
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * N);
        info->converged = 1;
        goto done;
    }
    for (;;) {
        or_spmv(n, rp, ci, va, x, r);
        for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double rn = nrm2(n, r);
        info->relres = rn / bnorm;
        if (!isfinite(rn)) { status = OR_ERR_NONFINITE; break; }
        if (info->relres <= rtol) { info->converged = 1; break; }
        if (total >= maxit) { status = OR_NOT_CONVERGED; break; }
        if (total > 0) info->restarts++;
        int st = prec_apply(&C, r, z);
        if (st != OR_OK) { status = st; break; }
        memcpy(p, z, sizeof(double) * N);
        double rz = dot(n, r, z);
        while (total < maxit) {
            or_spmv(n, rp, ci, va, p, q);
            double pq = dot(n, p, q);
            double alpha = rz / pq;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            total++;
            double rr = nrm2(n, r);
            if (!isfinite(rr) || !isfinite(alpha)) { status = OR_ERR_NONFINITE; goto done; }
            if (rr <= rtol * bnorm) break;
            st = prec_apply(&C, r, z);
            if (st != OR_OK) { status = st; goto done; }
            double rzn = dot(n, r, z);
            double beta = rzn / rz;
            rz = rzn;
            for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
    }
done:
    info->iterations = total;
    if (status == OR_OK && !info->converged) status = OR_NOT_CONVERGED;
    if (info->converged) status = OR_OK;
    info->status = status;
    free(r); free(z); free(p); free(q);
    if (C.have_scaled) { scaled_free(&C.S); free(C.work); }
    return status;
}
