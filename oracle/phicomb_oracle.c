/*
 * phicomb_oracle.c -- TEST INFRASTRUCTURE ONLY; not part of the product path.
 *
 * A plain, slow, single-threaded IEEE-double reference implementation of
 * the method of A. H. Al-Mohy, "Computing Linear Combinations of
 * phi-Function Actions for Exponential Integrators" (arXiv 2509.26475):
 *
 *   w_i = sum_{j=0..p} beta_ij phi_j(t_i A) v_j,  i = 1..r      (Sec. 1, (phi.comb))
 *
 * with beta_ij = alpha_i^j in the paper.  It contains
 *   - orc_params:       Algorithm 1 (Sec. 3): safe power basis, s0,
 *                       normalised basis, objective f, Brent minimisation,
 *                       scaling s;
 *   - orc_solve:        Algorithm 3 (Sec. 4), the block variant, in two
 *                       forms: the literal alpha-form (J (x) Delta) and the
 *                       beta-prescaled form for a general weight table
 *                       (Corollary of Theorem 1: D_exp(A, aJ, V) =
 *                       D_exp(A, J, V Delta^-1) Delta);
 *   - orc_solve_single: Algorithm 2 (Sec. 4), one combination;
 *   - orc_brent_min:    Brent's local minimiser, used by Algorithm 1.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no source with the HIP library.
 * Compiled with -O2 -ffp-contract=off: no fused multiply-adds.
 *
 * Layout: every n x c block is column-major, column q at X + q*n.
 * Readings where the paper is silent or inconsistent (documented in the
 * design notes as R1..R19):
 *   R1  Algorithm 3 forms J (x) Delta - xi I (x) T without the division by
 *       s that Algorithm 2 has; the division is applied (r = 1 must reduce
 *       to Algorithm 2, and the augmented-exponential check needs it).
 *   R2  The recovery uses S exp(kJ/s) at step k (as the listings do).
 *   R5  The stopping test is evaluated after every term (as the listings).
 *   R6  Each Taylor loop is capped at kcap terms; hitting it is an error.
 *   R7  s_int = max(1, ceil(s max|t_i|)).
 *   R9  Fallbacks for a short power basis (see orc_params).
 *   R13 p = 0 returns exp(tA) v_0 (the tracked last block is zero).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-4)
#define ORC_EOVERFLOW (-5)

typedef struct {
    int64_t n;
    int32_t kind;             /* 0: CSR, 1: dense row-major, 2: low rank U W^T */
    int32_t rank;             /* low rank: columns of U and W */
    const int32_t *rowptr;    /* CSR: n+1 */
    const int32_t *col;       /* CSR: nnz */
    const double *val;        /* CSR: nnz */
    const double *dense;      /* dense: n*n row-major */
    const double *lr_u;       /* low rank: U, n x rank row-major */
    const double *lr_w;       /* low rank: W, n x rank row-major */
} orc_op;

typedef struct {
    double shift;    /* xi* */
    double s0;       /* preliminary scale */
    double zstar;    /* minimiser in z = -xi/s0 */
    double fstar;    /* f(xi*) */
    double s;        /* scaling parameter (real) */
    int32_t m;
    int32_t r_acc;   /* last accepted power */
    int32_t n_feval;
    int32_t status;
} orc_params_t;

typedef struct {
    int32_t s_int;
    int32_t terms_S;     /* k at exit of the S-series loop */
    int32_t terms_rec;   /* total Taylor terms over all recovery steps */
    int32_t max_terms_step;
    int32_t status;
    int32_t pad;
} orc_stats_t;

/* ---------------------------------------------------------------- basics */

/* Inner product sum_i a_i b_i (ascending i) evaluated as if in twice the
 * working precision: the compensated dot product Dot2 of Ogita, Rump and
 * Oishi (SIAM J. Sci. Comput. 26, 2005), with the exact product split by
 * fma and the exact sum split by Knuth's TwoSum.  The result is the exact
 * inner product rounded once, up to a relative error of order u plus
 * n^2 u^2 times its condition number, instead of the n u of a plain sum. */
static double dot2(const double *a, int64_t sa, const double *b, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double p = a[i * sa] * b[i];
        const double pe = fma(a[i * sa], b[i], -p);   /* p + pe = a_i b_i exactly */
        const double t = s + p;
        const double z = t - s;
        const double te = (s - (t - z)) + (p - z);    /* t + te = s + p exactly */
        s = t;
        c += te + pe;
    }
    return s + c;
}

/* y = A x (row sums in stored order).  The low-rank operator of the third
 * experiment (Sec. 5) is applied matrix-free as x -> U (W^T x): first the
 * rank inner products c_k = sum_i W_ik x_i, compensated (dot2 above: a row
 * order plain sum carries an error of n u, which the non-normal cores
 * amplify beyond the method's own error at the paper's n), then y_i =
 * sum_k U_ik c_k. */
static void apply_A(const orc_op *A, const double *x, double *y)
{
    const int64_t n = A->n;
    if (A->kind == 2) {
        const int r = A->rank;
        double c[16];
        for (int k = 0; k < r; ++k)
            c[k] = dot2(A->lr_w + k, r, x, n);
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k)
                acc += A->lr_u[i * r + k] * c[k];
            y[i] = acc;
        }
        return;
    }
    if (A->kind == 0) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int32_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q)
                acc += A->val[q] * x[A->col[q]];
            y[i] = acc;
        }
    } else {
        for (int64_t i = 0; i < n; ++i) {
            const double *row = A->dense + i * n;
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j)
                acc += row[j] * x[j];
            y[i] = acc;
        }
    }
}

/* y = A_1 x = A x - xi x  (the shifted operator, Sec. 3). */
static void apply_A1(const orc_op *A, double xi, const double *x, double *y)
{
    apply_A(A, x, y);
    for (int64_t i = 0; i < A->n; ++i)
        y[i] = y[i] - xi * x[i];
}

/* Matrix infinity norm of an n x c block: max_i sum_q |X(i,q)|. */
static double norm_inf(const double *X, int64_t n, int c)
{
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = 0; q < c; ++q)
            s += fabs(X[(int64_t)q * n + i]);
        if (s > best || isnan(s))
            best = s;
        if (isnan(best))
            return best;
    }
    return best;
}

/* Euclidean norm, evaluated with a max-abs scaling so that it neither
 * overflows nor underflows before the result itself would. */
static double norm_2(const double *x, int64_t n)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(x[i]);
        if (a > mx || isnan(a))
            mx = a;
    }
    if (mx == 0.0 || isnan(mx) || isinf(mx))
        return mx;
    double ssq = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double q = x[i] / mx;
        ssq += q * q;
    }
    return mx * sqrt(ssq);
}

/* binom(m,k) as the correctly rounded double of the exact integer. */
static double binom_exact(int m, int k)
{
    unsigned __int128 b = 1;
    if (k > m - k)
        k = m - k;
    for (int j = 1; j <= k; ++j)
        b = b * (unsigned __int128)(m - k + j) / (unsigned __int128)j;
    return (double)b;
}

/* -------------------------------------------------------- Brent localmin */

typedef double (*orc_fun)(double x, void *ctx);

/*
 * Brent's minimiser without derivatives (R. P. Brent, "Algorithms for
 * Minimization without Derivatives", 1973, ch. 5): golden-section steps
 * combined with parabolic interpolation through the three best points.
 * Tolerance at x is rel*|x| + abs_tol.  Returns the minimiser.
 */
double orc_brent_min(orc_fun f, void *ctx, double a, double b, double rel,
                     double abs_tol, int max_iter, double *fmin, int *nfev)
{
    const double golden = 0.5 * (3.0 - sqrt(5.0));
    double x = a + golden * (b - a);
    double w = x, v = x;
    double fx = f(x, ctx);
    double fw = fx, fv = fx;
    double d = 0.0, e = 0.0;
    int evals = 1;
    for (int it = 0; it < max_iter; ++it) {
        const double mid = 0.5 * (a + b);
        const double tol1 = rel * fabs(x) + abs_tol;
        const double tol2 = 2.0 * tol1;
        if (fabs(x - mid) <= tol2 - 0.5 * (b - a))
            break;
        int use_golden = 1;
        if (fabs(e) > tol1) {
            /* parabola through (v,fv), (w,fw), (x,fx) */
            double r = (x - w) * (fx - fv);
            double q = (x - v) * (fx - fw);
            double pnum = (x - v) * q - (x - w) * r;
            q = 2.0 * (q - r);
            if (q > 0.0)
                pnum = -pnum;
            else
                q = -q;
            const double e_prev = e;
            e = d;
            if (fabs(pnum) < fabs(0.5 * q * e_prev) && pnum > q * (a - x) &&
                pnum < q * (b - x)) {
                d = pnum / q;
                const double u = x + d;
                if (u - a < tol2 || b - u < tol2)
                    d = (x < mid) ? tol1 : -tol1;
                use_golden = 0;
            }
        }
        if (use_golden) {
            e = (x < mid) ? b - x : a - x;
            d = golden * e;
        }
        const double u = (fabs(d) >= tol1) ? x + d : (d > 0.0 ? x + tol1 : x - tol1);
        const double fu = f(u, ctx);
        ++evals;
        if (fu <= fx) {
            if (u < x)
                b = x;
            else
                a = x;
            v = w; fv = fw;
            w = x; fw = fx;
            x = u; fx = fu;
        } else {
            if (u < x)
                a = u;
            else
                b = u;
            if (fu <= fw || w == x) {
                v = w; fv = fw;
                w = u; fw = fu;
            } else if (fu <= fv || v == x || v == w) {
                v = u; fv = fu;
            }
        }
    }
    if (fmin)
        *fmin = fx;
    if (nfev)
        *nfev = evals;
    return x;
}

/* ------------------------------------------------------------ Algorithm 1 */

typedef struct {
    const double *basis;   /* n x (m+1), column k = V_k */
    int64_t n;
    int m;
    const double *b;       /* binomials */
    double *y;             /* workspace n */
} objective_ctx;

/* f(xi) = || V (b .* p(xi)) ||_2^(1/m), z = -xi/s0, p = [z^m .. z 1]. */
static double objective(double z, void *vctx)
{
    objective_ctx *c = (objective_ctx *)vctx;
    const int m = c->m;
    double *coef = (double *)malloc(sizeof(double) * (m + 1));
    double pw = 1.0;                      /* z^(m-k), built from k = m down */
    for (int k = m; k >= 0; --k) {
        coef[k] = c->b[k] * pw;
        pw = pw * z;
    }
    for (int64_t i = 0; i < c->n; ++i) {
        double acc = 0.0;
        for (int k = 0; k <= m; ++k)
            acc += coef[k] * c->basis[(int64_t)k * c->n + i];
        c->y[i] = acc;
    }
    free(coef);
    const double nrm = norm_2(c->y, c->n);
    if (nrm == 0.0)
        return 0.0;
    return exp(log(nrm) / (double)m);
}

/*
 * Algorithm 1: choose the shift xi* and the scaling s.
 *   v_in     start vector (normalised here to unit 2-norm)
 *   L_out    optional [m+1]: L_k = log ||W_k||_2 for computed k (0 beyond)
 *   basis_out optional [n*(m+1)] column-major: the normalised basis.
 * Brent runs on z in [-sqrt(n), sqrt(n)] with relative tolerance
 * brent_rel, absolute tolerance brent_abs and at most brent_maxit steps.
 */
int orc_params(const orc_op *A, double tol, int m, const double *v_in,
               double brent_rel, double brent_abs, int brent_maxit,
               orc_params_t *out, double *L_out, double *basis_out)
{
    const int64_t n = A->n;
    memset(out, 0, sizeof(*out));
    out->m = m;
    if (n < 1 || m < 1 || m > 120 || !(tol > 0.0) || !isfinite(tol)) {
        out->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    const double gmax = 0.8 * log(DBL_MAX);
    const double gmin = 0.8 * log(DBL_MIN);
    double lmax = -INFINITY;
    for (int j = 0; j <= m; ++j) {
        double lj = lgamma(m + 1.0) - lgamma(j + 1.0) - lgamma(m - j + 1.0);
        if (lj > lmax)
            lmax = lj;
    }
    double *basis = (double *)calloc((size_t)n * (m + 1), sizeof(double));
    double *L = (double *)calloc((size_t)m + 1, sizeof(double));
    double *b = (double *)malloc(sizeof(double) * (m + 1));
    double *y = (double *)malloc(sizeof(double) * n);
    if (!basis || !L || !b || !y) {
        free(basis); free(L); free(b); free(y);
        out->status = ORC_ENOMEM;
        return ORC_ENOMEM;
    }
    /* V_0 = v / ||v||_2 */
    const double vn = norm_2(v_in, n);
    if (!(vn > 0.0) || !isfinite(vn)) {
        free(basis); free(L); free(b); free(y);
        out->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i)
        basis[i] = v_in[i] / vn;
    L[0] = 0.0;

    /* safe powers: W_k = A V_{k-1}, L_k = log||W_k||, guarded */
    int r = 0;
    int nonfinite = 0;
    for (int k = 1; k <= m; ++k) {
        double *Wk = basis + (int64_t)k * n;
        apply_A(A, basis + (int64_t)(k - 1) * n, Wk);
        const double Lk = log(norm_2(Wk, n));
        L[k] = Lk;
        if (isnan(Lk)) {
            nonfinite = 1;
            break;
        }
        if (Lk + 0.5 * log(k + 1.0) + lmax > gmax || Lk < gmin)
            break;
        r = k;
    }
    if (nonfinite) {
        free(basis); free(L); free(b); free(y);
        out->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    out->r_acc = r;
    if (L_out)
        for (int k = 0; k <= m; ++k)
            L_out[k] = (k <= r + 1) ? L[k] : 0.0;
    if (r == 0) {
        if (L[1] < gmin) {
            /* A v vanishes to working precision: A is treated as zero. */
            out->shift = 0.0;
            out->s0 = 0.0;
            out->s = 1.0;
            out->fstar = 0.0;
            out->status = ORC_OK;
            free(basis); free(L); free(b); free(y);
            return ORC_OK;
        }
        free(basis); free(L); free(b); free(y);
        out->status = ORC_EOVERFLOW;
        return ORC_EOVERFLOW;
    }
    /* preliminary scale s0: mean log growth over the last accepted ratios */
    double s0;
    if (r >= 3) {
        const int jr = (r - 5 > 2) ? r - 5 : 2;
        double sum = 0.0;
        for (int j = jr; j <= r - 1; ++j)
            sum += L[j + 1] - L[j];
        s0 = exp(sum / (double)(r - jr));
    } else {
        s0 = exp(L[r] / (double)r);   /* R9: fewer than three powers */
    }
    out->s0 = s0;
    /* normalise V_j by s0^-j, then extend to degree m */
    const double ls0 = log(s0);
    for (int j = 1; j <= r; ++j) {
        const double sc = exp(-(double)j * ls0);
        double *Vj = basis + (int64_t)j * n;
        for (int64_t i = 0; i < n; ++i)
            Vj[i] = Vj[i] * sc;
    }
    for (int k = r + 1; k <= m; ++k) {
        double *Vk = basis + (int64_t)k * n;
        apply_A(A, basis + (int64_t)(k - 1) * n, Vk);
        for (int64_t i = 0; i < n; ++i)
            Vk[i] = Vk[i] / s0;
    }
    for (int k = 0; k <= m; ++k)
        b[k] = binom_exact(m, k);
    objective_ctx ctx = {basis, n, m, b, y};
    const double zmax = sqrt((double)n);
    double fz = 0.0;
    int nfev = 0;
    const double zs = orc_brent_min(objective, &ctx, -zmax, zmax, brent_rel,
                                    brent_abs, brent_maxit, &fz, &nfev);
    out->zstar = zs;
    out->shift = -zs * s0;
    out->fstar = fz;
    out->n_feval = nfev;
    out->s = s0 * fz / exp((log(tol) + lgamma(m + 1.0)) / (double)m);
    out->status = ORC_OK;
    if (basis_out)
        memcpy(basis_out, basis, sizeof(double) * (size_t)n * (m + 1));
    free(basis); free(L); free(b); free(y);
    return ORC_OK;
}

/* ------------------------------------------------------------ Algorithm 3 */

/* Block b of the reordered V holds v_perm(b): [v_0, v_p, v_{p-1}, ..., v_1]. */
static int perm_index(int b, int p) { return b == 0 ? 0 : p + 1 - b; }

/* exp(N) for a nilpotent (p+1)x(p+1) matrix N, by its finite series. */
static void small_expm_nilpotent(const double *N, int P1, double *out)
{
    double *term = (double *)malloc(sizeof(double) * P1 * P1);
    double *tmp = (double *)malloc(sizeof(double) * P1 * P1);
    for (int a = 0; a < P1 * P1; ++a)
        out[a] = term[a] = 0.0;
    for (int a = 0; a < P1; ++a)
        out[a * P1 + a] = term[a * P1 + a] = 1.0;
    for (int d = 1; d <= P1; ++d) {
        for (int a = 0; a < P1; ++a)
            for (int c = 0; c < P1; ++c) {
                double acc = 0.0;
                for (int q = 0; q < P1; ++q)
                    acc += term[a * P1 + q] * N[q * P1 + c];
                tmp[a * P1 + c] = acc / (double)d;
            }
        memcpy(term, tmp, sizeof(double) * P1 * P1);
        for (int a = 0; a < P1 * P1; ++a)
            out[a] += term[a];
    }
    free(term);
    free(tmp);
}

/*
 * Algorithm 3.  form 0: beta-prescaled (general table beta[r][p+1],
 * Delta = I, column (b,i) of V scaled by beta_{i,perm(b)}, the recovery
 * adds beta_i0 v_0).  form 1: the literal alpha-form (Delta = diag(alpha),
 * W = F_1 + F_2 Delta), valid when beta_ij = alpha_i^j.
 *   V   n x (p+1) column-major, natural order v_0..v_p
 *   W   n x r column-major output
 */
int orc_solve(const orc_op *A, int p, int r, const double *t,
              const double *beta, const double *alpha, int form,
              const double *V, double tol, double xi, double s, int kcap,
              double *W, orc_stats_t *st)
{
    const int64_t n = A->n;
    memset(st, 0, sizeof(*st));
    if (n < 1 || p < 0 || r < 1 || !(tol > 0.0) || !isfinite(tol) ||
        !isfinite(xi) || !isfinite(s) || s < 0.0 || kcap < 2 ||
        (form == 1 && !alpha) || (form == 0 && !beta)) {
        st->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    const int P1 = p + 1;
    const int cS = P1 * r;
    const int cR = 2 * r;
    double tmax = 0.0;
    for (int i = 0; i < r; ++i) {
        if (!isfinite(t[i])) {
            st->status = ORC_EINVAL;
            return ORC_EINVAL;
        }
        if (fabs(t[i]) > tmax)
            tmax = fabs(t[i]);
    }
    /* s <- ceil(s max|t_i|) (R7: at least 1) */
    const double sceil = ceil(s * tmax);
    if (!(sceil <= 2147483647.0)) {
        st->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    const int ss = sceil < 1.0 ? 1 : (int)sceil;
    const double ssd = (double)ss;
    st->s_int = ss;

    double *mu = (double *)malloc(sizeof(double) * r);
    double *Dl = (double *)malloc(sizeof(double) * r);
    double *Jt = (double *)malloc(sizeof(double) * r * P1 * P1);    /* exp(Delta_i J/s) */
    double *Js = (double *)malloc(sizeof(double) * r * P1 * P1);    /* (Delta_i J - xi t_i I)/s */
    double *Vb = (double *)malloc(sizeof(double) * (size_t)n * cS);
    double *Vn = (double *)malloc(sizeof(double) * (size_t)n * cS);
    double *S = (double *)malloc(sizeof(double) * (size_t)n * cS);
    double *D = (double *)malloc(sizeof(double) * (size_t)n * cS);
    double *F = (double *)malloc(sizeof(double) * (size_t)n * cR);
    double *E = (double *)malloc(sizeof(double) * (size_t)n * cR);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *Nm = (double *)malloc(sizeof(double) * P1 * P1);
    int status = ORC_OK;
    if (!mu || !Dl || !Jt || !Js || !Vb || !Vn || !S || !D || !F || !E || !y || !Nm) {
        status = ORC_ENOMEM;
        goto done;
    }
    /* T = diag(t), mu = exp((xi/s) T), Delta = diag(alpha) or I */
    for (int i = 0; i < r; ++i) {
        mu[i] = exp(xi * t[i] / ssd);
        Dl[i] = (form == 1) ? alpha[i] : 1.0;
    }
    /* V <- V (I_{p+1} (x) 1_r^T mu / s), reordered, beta-prescaled in form 0 */
    for (int b = 0; b < P1; ++b) {
        const double *vsrc = V + (int64_t)perm_index(b, p) * n;
        for (int i = 0; i < r; ++i) {
            const double wgt = (form == 0) ? beta[i * P1 + perm_index(b, p)] : 1.0;
            const double sc = mu[i] / ssd;
            double *dst = Vb + (int64_t)(b * r + i) * n;
            for (int64_t q = 0; q < n; ++q)
                dst[q] = (vsrc[q] * wgt) * sc;
        }
    }
    /* J = [0] (+) J_p(0): ones at (b, b+1) for 1 <= b < p */
    for (int i = 0; i < r; ++i) {
        double *jt = Jt + i * P1 * P1;
        double *js = Js + i * P1 * P1;
        for (int a = 0; a < P1 * P1; ++a)
            Nm[a] = 0.0;
        for (int bb = 1; bb < p; ++bb)
            Nm[bb * P1 + bb + 1] = Dl[i] / ssd;
        small_expm_nilpotent(Nm, P1, jt);
        for (int a = 0; a < P1 * P1; ++a)
            js[a] = 0.0;
        for (int bb = 0; bb < P1; ++bb)
            js[bb * P1 + bb] = (-xi * t[i]) / ssd;
        for (int bb = 1; bb < p; ++bb)
            js[bb * P1 + bb + 1] = Dl[i] / ssd;
    }
    memcpy(S, Vb, sizeof(double) * (size_t)n * cS);
    memcpy(D, Vb, sizeof(double) * (size_t)n * cS);
    int k = 1;
    double sigma = 1.0;
    double c1 = INFINITY;
    double c2 = norm_inf(D, n, cS);
    while (c1 + c2 > tol * norm_inf(S, n, cS)) {
        if (k >= kcap) {
            status = ORC_ENOCONV;
            goto done;
        }
        k = k + 1;
        c1 = c2;
        sigma = k * sigma;
        /* V <- V J  (per abscissa, block (b,i) couples only within i) */
        for (int i = 0; i < r; ++i) {
            const double *js = Js + i * P1 * P1;
            for (int bc = 0; bc < P1; ++bc) {
                double *dst = Vn + (int64_t)(bc * r + i) * n;
                for (int64_t q = 0; q < n; ++q) {
                    double acc = 0.0;
                    for (int bb = 0; bb < P1; ++bb)
                        acc += Vb[(int64_t)(bb * r + i) * n + q] * js[bb * P1 + bc];
                    dst[q] = acc;
                }
            }
        }
        memcpy(Vb, Vn, sizeof(double) * (size_t)n * cS);
        /* D <- A_1 D (I (x) T/s) + V */
        for (int bb = 0; bb < P1; ++bb)
            for (int i = 0; i < r; ++i) {
                double *dc = D + (int64_t)(bb * r + i) * n;
                const double *vc = Vb + (int64_t)(bb * r + i) * n;
                const double ts = t[i] / ssd;
                apply_A1(A, xi, dc, y);
                for (int64_t q = 0; q < n; ++q)
                    dc[q] = y[q] * ts + vc[q];
            }
        c2 = norm_inf(D, n, cS) / sigma;
        for (int64_t q = 0; q < (int64_t)n * cS; ++q)
            S[q] = S[q] + D[q] / sigma;
        if (isnan(c2)) {
            status = ORC_EINVAL;
            goto done;
        }
    }
    st->terms_S = k;
    /* F = first and last block columns of S */
    for (int i = 0; i < r; ++i) {
        memcpy(F + (int64_t)i * n, S + (int64_t)i * n, sizeof(double) * n);
        if (p >= 1)
            memcpy(F + (int64_t)(r + i) * n, S + (int64_t)(p * r + i) * n, sizeof(double) * n);
        else
            memset(F + (int64_t)(r + i) * n, 0, sizeof(double) * n);
    }
    /* F(:,1:r) <- A F(:,1:r) T + v_0 1^T : recover exp(t_i A/s) v_0 */
    for (int i = 0; i < r; ++i) {
        double *fc = F + (int64_t)i * n;
        const double w0 = (form == 0) ? beta[i * P1 + 0] : 1.0;
        apply_A(A, fc, y);
        for (int64_t q = 0; q < n; ++q)
            fc[q] = y[q] * t[i] + w0 * V[q];
    }
    /* T <- I_2 (x) T/s, mu <- I_2 (x) mu; advance s-1 steps */
    int tot = 0, maxstep = 0;
    for (int j = 1; j <= ss - 1; ++j) {
        memcpy(E, F, sizeof(double) * (size_t)n * cR);
        int kk = 0;
        double d1 = INFINITY;
        double d2 = norm_inf(F, n, cR);
        while (d1 + d2 > tol * norm_inf(E, n, cR)) {
            if (kk >= kcap) {
                status = ORC_ENOCONV;
                goto done;
            }
            kk = kk + 1;
            d1 = d2;
            for (int q = 0; q < cR; ++q) {
                double *fc = F + (int64_t)q * n;
                const double ts = t[q % r] / ssd;
                apply_A1(A, xi, fc, y);
                for (int64_t z = 0; z < n; ++z)
                    fc[z] = y[z] * ts / (double)kk;
            }
            d2 = norm_inf(F, n, cR);
            for (int64_t z = 0; z < (int64_t)n * cR; ++z)
                E[z] = E[z] + F[z];
            if (isnan(d2)) {
                status = ORC_EINVAL;
                goto done;
            }
        }
        tot += kk;
        if (kk > maxstep)
            maxstep = kk;
        /* E <- E mu (undo the shift) */
        for (int q = 0; q < cR; ++q) {
            double *ec = E + (int64_t)q * n;
            const double m_q = mu[q % r];
            for (int64_t z = 0; z < n; ++z)
                ec[z] = ec[z] * m_q;
        }
        /* S <- S exp(J (x) Delta / s) */
        for (int i = 0; i < r; ++i) {
            const double *jt = Jt + i * P1 * P1;
            for (int bc = 0; bc < P1; ++bc) {
                double *dst = Vn + (int64_t)(bc * r + i) * n;
                for (int64_t q = 0; q < n; ++q) {
                    double acc = 0.0;
                    for (int bb = 0; bb < P1; ++bb)
                        acc += S[(int64_t)(bb * r + i) * n + q] * jt[bb * P1 + bc];
                    dst[q] = acc;
                }
            }
        }
        memcpy(S, Vn, sizeof(double) * (size_t)n * cS);
        /* F <- E + S(:, [block 0, block p]);  F(:,1:r) <- E(:,1:r) */
        for (int i = 0; i < r; ++i) {
            memcpy(F + (int64_t)i * n, E + (int64_t)i * n, sizeof(double) * n);
            double *f2 = F + (int64_t)(r + i) * n;
            const double *e2 = E + (int64_t)(r + i) * n;
            const double *sp = S + (int64_t)(p * r + i) * n;
            for (int64_t q = 0; q < n; ++q)
                f2[q] = (p >= 1) ? e2[q] + sp[q] : e2[q];
        }
    }
    st->terms_rec = tot;
    st->max_terms_step = maxstep;
    /* [w_1..w_r] = F(:,1:r) + F(:,r+1:2r) Delta */
    for (int i = 0; i < r; ++i)
        for (int64_t q = 0; q < n; ++q)
            W[(int64_t)i * n + q] = F[(int64_t)i * n + q] + F[(int64_t)(r + i) * n + q] * Dl[i];
done:
    st->status = status;
    free(mu); free(Dl); free(Jt); free(Js); free(Vb); free(Vn);
    free(S); free(D); free(F); free(E); free(y); free(Nm);
    return status;
}

/* ------------------------------------------------------------ Algorithm 2 */

/* One combination w = sum_j alpha^j phi_j(tA) v_j.  V n x (p+1) column-major. */
int orc_solve_single(const orc_op *A, int p, double t, double alpha,
                     const double *V, double tol, double xi, double s, int kcap,
                     double *w, orc_stats_t *st)
{
    const int64_t n = A->n;
    memset(st, 0, sizeof(*st));
    if (n < 1 || p < 0 || !(tol > 0.0) || !isfinite(t) || !isfinite(alpha) ||
        !isfinite(xi) || !isfinite(s) || kcap < 2) {
        st->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    const int P1 = p + 1;
    const double sceil = ceil(fabs(t) * s);
    if (!(sceil <= 2147483647.0)) {
        st->status = ORC_EINVAL;
        return ORC_EINVAL;
    }
    const int ss = sceil < 1.0 ? 1 : (int)sceil;
    const double ssd = (double)ss;
    st->s_int = ss;
    const double mu = exp(t * xi / ssd);
    double *Vr = (double *)malloc(sizeof(double) * (size_t)n * P1);
    double *Vn = (double *)malloc(sizeof(double) * (size_t)n * P1);
    double *S = (double *)malloc(sizeof(double) * (size_t)n * P1);
    double *D = (double *)malloc(sizeof(double) * (size_t)n * P1);
    double *F = (double *)malloc(sizeof(double) * (size_t)n * 2);
    double *E = (double *)malloc(sizeof(double) * (size_t)n * 2);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *Nm = (double *)malloc(sizeof(double) * P1 * P1);
    double *Jt = (double *)malloc(sizeof(double) * P1 * P1);
    double *Js = (double *)malloc(sizeof(double) * P1 * P1);
    int status = ORC_OK;
    if (!Vr || !Vn || !S || !D || !F || !E || !y || !Nm || !Jt || !Js) {
        status = ORC_ENOMEM;
        goto done;
    }
    /* J <- alpha J;  V <- (mu/s)[v_0, v_p, ..., v_1] */
    for (int b = 0; b < P1; ++b) {
        const double *src = V + (int64_t)perm_index(b, p) * n;
        for (int64_t q = 0; q < n; ++q)
            Vr[(int64_t)b * n + q] = (mu / ssd) * src[q];
    }
    for (int a = 0; a < P1 * P1; ++a)
        Nm[a] = 0.0;
    for (int bb = 1; bb < p; ++bb)
        Nm[bb * P1 + bb + 1] = alpha / ssd;
    small_expm_nilpotent(Nm, P1, Jt);               /* Jtilde = exp(J/s) */
    for (int a = 0; a < P1 * P1; ++a)
        Js[a] = 0.0;
    for (int bb = 1; bb < p; ++bb)
        Js[bb * P1 + bb + 1] = alpha / ssd;
    for (int bb = 0; bb < P1; ++bb)
        Js[bb * P1 + bb] = (-t * xi) / ssd;         /* J <- (J - t xi I)/s */
    memcpy(S, Vr, sizeof(double) * (size_t)n * P1);
    memcpy(D, Vr, sizeof(double) * (size_t)n * P1);
    int k = 1;
    double sigma = 1.0, c1 = INFINITY, c2 = norm_inf(D, n, P1);
    while (c1 + c2 > tol * norm_inf(S, n, P1)) {
        if (k >= kcap) {
            status = ORC_ENOCONV;
            goto done;
        }
        k = k + 1;
        c1 = c2;
        sigma = k * sigma;
        for (int bc = 0; bc < P1; ++bc)
            for (int64_t q = 0; q < n; ++q) {
                double acc = 0.0;
                for (int bb = 0; bb < P1; ++bb)
                    acc += Vr[(int64_t)bb * n + q] * Js[bb * P1 + bc];
                Vn[(int64_t)bc * n + q] = acc;
            }
        memcpy(Vr, Vn, sizeof(double) * (size_t)n * P1);
        for (int bb = 0; bb < P1; ++bb) {
            double *dc = D + (int64_t)bb * n;
            apply_A1(A, xi, dc, y);
            for (int64_t q = 0; q < n; ++q)
                dc[q] = t * y[q] / ssd + Vr[(int64_t)bb * n + q];
        }
        c2 = norm_inf(D, n, P1) / sigma;
        for (int64_t q = 0; q < (int64_t)n * P1; ++q)
            S[q] = S[q] + D[q] / sigma;
        if (isnan(c2)) {
            status = ORC_EINVAL;
            goto done;
        }
    }
    st->terms_S = k;
    memcpy(F, S, sizeof(double) * n);
    if (p >= 1)
        memcpy(F + n, S + (int64_t)p * n, sizeof(double) * n);
    else
        memset(F + n, 0, sizeof(double) * n);
    apply_A(A, F, y);
    for (int64_t q = 0; q < n; ++q)
        F[q] = t * y[q] + V[q];                      /* recover exp(tA/s) v_0 */
    int tot = 0, maxstep = 0;
    for (int j = 1; j <= ss - 1; ++j) {
        memcpy(E, F, sizeof(double) * (size_t)n * 2);
        int kk = 0;
        double d1 = INFINITY, d2 = norm_inf(F, n, 2);
        while (d1 + d2 > tol * norm_inf(E, n, 2)) {
            if (kk >= kcap) {
                status = ORC_ENOCONV;
                goto done;
            }
            kk = kk + 1;
            d1 = d2;
            for (int q = 0; q < 2; ++q) {
                double *fc = F + (int64_t)q * n;
                apply_A1(A, xi, fc, y);
                for (int64_t z = 0; z < n; ++z)
                    fc[z] = t * y[z] / (ssd * kk);
            }
            d2 = norm_inf(F, n, 2);
            for (int64_t z = 0; z < (int64_t)n * 2; ++z)
                E[z] = E[z] + F[z];
            if (isnan(d2)) {
                status = ORC_EINVAL;
                goto done;
            }
        }
        tot += kk;
        if (kk > maxstep)
            maxstep = kk;
        for (int64_t z = 0; z < (int64_t)n * 2; ++z)
            E[z] = mu * E[z];                        /* undo the shift */
        for (int bc = 0; bc < P1; ++bc)              /* S <- S Jtilde */
            for (int64_t q = 0; q < n; ++q) {
                double acc = 0.0;
                for (int bb = 0; bb < P1; ++bb)
                    acc += S[(int64_t)bb * n + q] * Jt[bb * P1 + bc];
                Vn[(int64_t)bc * n + q] = acc;
            }
        memcpy(S, Vn, sizeof(double) * (size_t)n * P1);
        memcpy(F, E, sizeof(double) * n);
        for (int64_t q = 0; q < n; ++q)
            F[n + q] = (p >= 1) ? E[n + q] + S[(int64_t)p * n + q] : E[n + q];
    }
    st->terms_rec = tot;
    st->max_terms_step = maxstep;
    for (int64_t q = 0; q < n; ++q)
        w[q] = F[q] + alpha * F[n + q];
done:
    st->status = status;
    free(Vr); free(Vn); free(S); free(D); free(F); free(E); free(y);
    free(Nm); free(Jt); free(Js);
    return status;
}

/* y = A x, exported for tests of the operator expansion. */
void orc_apply(const orc_op *A, const double *x, double *y) { apply_A(A, x, y); }
double orc_binom(int m, int k) { return binom_exact(m, k); }
