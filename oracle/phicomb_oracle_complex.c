/*
 * phicomb_oracle_complex.c -- TEST INFRASTRUCTURE ONLY; not part of the
 * product path.
 *
 * Algorithms 1 and 3 of A. H. Al-Mohy, "Computing Linear Combinations of
 * phi-Function Actions for Exponential Integrators" (arXiv 2509.26475) over
 * the complex numbers, in plain single-threaded C99 complex double.  Sec. 1
 * poses the problem for A in C^{n x n}, V in C^{n x (p+1)} and complex t,
 * alpha; Algorithm 3 takes a shift xi in C; Algorithm 1's listing searches
 * xi on the real line (z = -xi/s0 real, the bracket [-sqrt(n) s0, sqrt(n) s0])
 * from a real unit start vector, so its xi* is real even for complex A.
 *
 *   orz_params: Algorithm 1 (Sec. 3) with complex powers A^k v;
 *   orz_solve:  Algorithm 3 (Sec. 4), alpha-form (J (x) Delta, Delta =
 *               diag(alpha)) or beta-prescaled form (general weight table,
 *               Delta = I), complex t, alpha or beta, xi.
 *
 * The same readings as the real oracle (R1 division of J (x) Delta - xi I (x)
 * T by s, R4 block infinity norm = max row sum of moduli, R5 test every
 * term, R6 term cap, R7 s_int >= 1, R9 short power basis, R13 p = 0), with
 * |t_i| the modulus in s_int = ceil(s max|t_i|).  Brent's minimiser and the
 * exact binomials are the real oracle's (orc_brent_min, orc_binom).
 * Compiled with -O2 -ffp-contract=off.  Blocks are column-major.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORZ_OK 0
#define ORZ_EINVAL (-1)
#define ORZ_ENOMEM (-2)
#define ORZ_ENOCONV (-4)
#define ORZ_EOVERFLOW (-5)

typedef double complex zc;

typedef struct {
    int64_t n;
    int32_t kind;             /* 0: CSR, 1: dense row-major */
    int32_t pad;
    const int32_t *rowptr;    /* CSR: n+1 */
    const int32_t *col;       /* CSR: nnz */
    const zc *val;            /* CSR: nnz */
    const zc *dense;          /* dense: n*n row-major */
} orz_op;

typedef struct {
    double shift;    /* xi* (real: Algorithm 1 searches the real line) */
    double s0;
    double zstar;
    double fstar;
    double s;
    int32_t m;
    int32_t r_acc;
    int32_t n_feval;
    int32_t status;
} orz_params_t;

typedef struct {
    int32_t s_int;
    int32_t terms_S;
    int32_t terms_rec;
    int32_t max_terms_step;
    int32_t status;
    int32_t pad;
} orz_stats_t;

typedef double (*orz_fun)(double x, void *ctx);
double orc_brent_min(orz_fun f, void *ctx, double a, double b, double rel, double abs_tol,
                     int max_iter, double *fmin, int *nfev);
double orc_binom(int m, int k);

/* y = A x, row sums in stored order. */
static void zapply(const orz_op *A, const zc *x, zc *y)
{
    const int64_t n = A->n;
    for (int64_t i = 0; i < n; ++i) {
        zc acc = 0.0;
        if (A->kind == 0) {
            for (int32_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q)
                acc += A->val[q] * x[A->col[q]];
        } else {
            const zc *row = A->dense + i * n;
            for (int64_t j = 0; j < n; ++j)
                acc += row[j] * x[j];
        }
        y[i] = acc;
    }
}

/* y = (A - xi I) x. */
static void zapply1(const orz_op *A, zc xi, const zc *x, zc *y)
{
    zapply(A, x, y);
    for (int64_t i = 0; i < A->n; ++i)
        y[i] = y[i] - xi * x[i];
}

/* Block infinity norm: max_i sum_q |X(i,q)| (moduli). */
static double znorm_inf(const zc *X, int64_t n, int c)
{
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = 0; q < c; ++q)
            s += cabs(X[(int64_t)q * n + i]);
        if (s > best || isnan(s))
            best = s;
        if (isnan(best))
            return best;
    }
    return best;
}

/* Euclidean norm with max-modulus scaling. */
static double znorm_2(const zc *x, int64_t n)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double a = cabs(x[i]);
        if (a > mx || isnan(a))
            mx = a;
    }
    if (mx == 0.0 || isnan(mx) || isinf(mx))
        return mx;
    double ssq = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double q = cabs(x[i]) / mx;
        ssq += q * q;
    }
    return mx * sqrt(ssq);
}

static int zfinite(zc z) { return isfinite(creal(z)) && isfinite(cimag(z)); }

/* ------------------------------------------------------------ Algorithm 1 */

typedef struct {
    const zc *basis;   /* n x (m+1) */
    int64_t n;
    int m;
    const double *b;
    zc *y;
} zobjective_ctx;

/* f(xi) = || V (b .* p(xi)) ||_2^(1/m), z = -xi/s0 real, p = [z^m .. z 1]. */
static double zobjective(double z, void *vctx)
{
    zobjective_ctx *c = (zobjective_ctx *)vctx;
    const int m = c->m;
    double *coef = (double *)malloc(sizeof(double) * (m + 1));
    double pw = 1.0;
    for (int k = m; k >= 0; --k) {
        coef[k] = c->b[k] * pw;
        pw = pw * z;
    }
    for (int64_t i = 0; i < c->n; ++i) {
        zc acc = 0.0;
        for (int k = 0; k <= m; ++k)
            acc += coef[k] * c->basis[(int64_t)k * c->n + i];
        c->y[i] = acc;
    }
    free(coef);
    const double nrm = znorm_2(c->y, c->n);
    if (nrm == 0.0)
        return 0.0;
    return exp(log(nrm) / (double)m);
}

/* Algorithm 1 for a complex operator; v_in real (the listing's v in R^n). */
int orz_params(const orz_op *A, double tol, int m, const double *v_in, double brent_rel,
               double brent_abs, int brent_maxit, orz_params_t *out)
{
    const int64_t n = A->n;
    memset(out, 0, sizeof(*out));
    out->m = m;
    if (n < 1 || m < 1 || m > 120 || !(tol > 0.0) || !isfinite(tol)) {
        out->status = ORZ_EINVAL;
        return ORZ_EINVAL;
    }
    const double gmax = 0.8 * log(DBL_MAX);
    const double gmin = 0.8 * log(DBL_MIN);
    double lmax = -INFINITY;
    for (int j = 0; j <= m; ++j) {
        const double lj = lgamma(m + 1.0) - lgamma(j + 1.0) - lgamma(m - j + 1.0);
        if (lj > lmax)
            lmax = lj;
    }
    zc *basis = (zc *)calloc((size_t)n * (m + 1), sizeof(zc));
    double *L = (double *)calloc((size_t)m + 1, sizeof(double));
    double *b = (double *)malloc(sizeof(double) * (m + 1));
    zc *y = (zc *)malloc(sizeof(zc) * n);
    int status = ORZ_OK;
    if (!basis || !L || !b || !y) {
        status = ORZ_ENOMEM;
        goto done;
    }
    double vn = 0.0;
    {
        double mx = 0.0, ssq = 0.0;
        for (int64_t i = 0; i < n; ++i)
            if (fabs(v_in[i]) > mx)
                mx = fabs(v_in[i]);
        for (int64_t i = 0; mx > 0.0 && i < n; ++i)
            ssq += (v_in[i] / mx) * (v_in[i] / mx);
        vn = mx * sqrt(ssq);
    }
    if (!(vn > 0.0) || !isfinite(vn)) {
        status = ORZ_EINVAL;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i)
        basis[i] = v_in[i] / vn;
    /* guarded powers W_k = A V_{k-1}, L_k = log ||W_k||_2 */
    int r = 0;
    for (int k = 1; k <= m; ++k) {
        zc *Wk = basis + (int64_t)k * n;
        zapply(A, basis + (int64_t)(k - 1) * n, Wk);
        const double Lk = log(znorm_2(Wk, n));
        L[k] = Lk;
        if (isnan(Lk)) {
            status = ORZ_EINVAL;
            goto done;
        }
        if (Lk + 0.5 * log(k + 1.0) + lmax > gmax || Lk < gmin)
            break;
        r = k;
    }
    out->r_acc = r;
    if (r == 0) {
        if (L[1] < gmin) {   /* A v vanishes: A is treated as zero (R9) */
            out->s = 1.0;
            status = ORZ_OK;
        } else {
            status = ORZ_EOVERFLOW;
        }
        goto done;
    }
    double s0;
    if (r >= 3) {
        const int jr = (r - 5 > 2) ? r - 5 : 2;
        double sum = 0.0;
        for (int j = jr; j <= r - 1; ++j)
            sum += L[j + 1] - L[j];
        s0 = exp(sum / (double)(r - jr));
    } else {
        s0 = exp(L[r] / (double)r);
    }
    out->s0 = s0;
    const double ls0 = log(s0);
    for (int j = 1; j <= r; ++j) {
        const double sc = exp(-(double)j * ls0);
        zc *Vj = basis + (int64_t)j * n;
        for (int64_t i = 0; i < n; ++i)
            Vj[i] = Vj[i] * sc;
    }
    for (int k = r + 1; k <= m; ++k) {
        zc *Vk = basis + (int64_t)k * n;
        zapply(A, basis + (int64_t)(k - 1) * n, Vk);
        for (int64_t i = 0; i < n; ++i)
            Vk[i] = Vk[i] / s0;
    }
    for (int k = 0; k <= m; ++k)
        b[k] = orc_binom(m, k);
    zobjective_ctx ctx = {basis, n, m, b, y};
    const double zmax = sqrt((double)n);
    double fz = 0.0;
    int nfev = 0;
    const double zs = orc_brent_min(zobjective, &ctx, -zmax, zmax, brent_rel, brent_abs,
                                    brent_maxit, &fz, &nfev);
    out->zstar = zs;
    out->shift = -zs * s0;
    out->fstar = fz;
    out->n_feval = nfev;
    out->s = s0 * fz / exp((log(tol) + lgamma(m + 1.0)) / (double)m);
done:
    out->status = status;
    free(basis); free(L); free(b); free(y);
    return status;
}

/* ------------------------------------------------------------ Algorithm 3 */

static int zperm(int b, int p) { return b == 0 ? 0 : p + 1 - b; }

/* exp(N) of a nilpotent (p+1) x (p+1) matrix by its finite series. */
static void zexpm_nilpotent(const zc *N, int P1, zc *out)
{
    zc *term = (zc *)malloc(sizeof(zc) * P1 * P1);
    zc *tmp = (zc *)malloc(sizeof(zc) * P1 * P1);
    for (int a = 0; a < P1 * P1; ++a)
        out[a] = term[a] = 0.0;
    for (int a = 0; a < P1; ++a)
        out[a * P1 + a] = term[a * P1 + a] = 1.0;
    for (int d = 1; d <= P1; ++d) {
        for (int a = 0; a < P1; ++a)
            for (int c = 0; c < P1; ++c) {
                zc acc = 0.0;
                for (int q = 0; q < P1; ++q)
                    acc += term[a * P1 + q] * N[q * P1 + c];
                tmp[a * P1 + c] = acc / (double)d;
            }
        memcpy(term, tmp, sizeof(zc) * P1 * P1);
        for (int a = 0; a < P1 * P1; ++a)
            out[a] += term[a];
    }
    free(term);
    free(tmp);
}

/*
 * Algorithm 3 over C.  form 0: beta-prescaled (beta[r][p+1] complex,
 * Delta = I); form 1: the literal alpha-form (Delta = diag(alpha)).
 *   V [p+1][n] column-major, W [r][n] column-major output, *xi_in the shift.
 */
int orz_solve(const orz_op *A, int p, int r, const zc *t, const zc *beta, const zc *alpha,
              int form, const zc *V, double tol, const zc *xi_in, double s, int kcap, zc *W,
              orz_stats_t *st)
{
    const int64_t n = A->n;
    const zc xi = *xi_in;
    memset(st, 0, sizeof(*st));
    if (n < 1 || p < 0 || r < 1 || !(tol > 0.0) || !isfinite(tol) || !zfinite(xi) ||
        !isfinite(s) || s < 0.0 || kcap < 2 || (form == 1 && !alpha) || (form == 0 && !beta)) {
        st->status = ORZ_EINVAL;
        return ORZ_EINVAL;
    }
    const int P1 = p + 1, cS = P1 * r, cR = 2 * r;
    double tmax = 0.0;
    for (int i = 0; i < r; ++i) {
        if (!zfinite(t[i])) {
            st->status = ORZ_EINVAL;
            return ORZ_EINVAL;
        }
        if (cabs(t[i]) > tmax)
            tmax = cabs(t[i]);
    }
    /* s <- ceil(s max|t_i|) (R7: at least 1) */
    const double sceil = ceil(s * tmax);
    if (!(sceil <= 2147483647.0)) {
        st->status = ORZ_EINVAL;
        return ORZ_EINVAL;
    }
    const int ss = sceil < 1.0 ? 1 : (int)sceil;
    const double ssd = (double)ss;
    st->s_int = ss;

    zc *mu = (zc *)malloc(sizeof(zc) * r);
    zc *Dl = (zc *)malloc(sizeof(zc) * r);
    zc *Jt = (zc *)malloc(sizeof(zc) * r * P1 * P1);
    zc *Js = (zc *)malloc(sizeof(zc) * r * P1 * P1);
    zc *Vb = (zc *)malloc(sizeof(zc) * (size_t)n * cS);
    zc *Vn = (zc *)malloc(sizeof(zc) * (size_t)n * cS);
    zc *S = (zc *)malloc(sizeof(zc) * (size_t)n * cS);
    zc *D = (zc *)malloc(sizeof(zc) * (size_t)n * cS);
    zc *F = (zc *)malloc(sizeof(zc) * (size_t)n * cR);
    zc *E = (zc *)malloc(sizeof(zc) * (size_t)n * cR);
    zc *y = (zc *)malloc(sizeof(zc) * (size_t)n);
    zc *Nm = (zc *)malloc(sizeof(zc) * P1 * P1);
    int status = ORZ_OK;
    if (!mu || !Dl || !Jt || !Js || !Vb || !Vn || !S || !D || !F || !E || !y || !Nm) {
        status = ORZ_ENOMEM;
        goto done;
    }
    /* T = diag(t), mu = exp((xi/s) T), Delta = diag(alpha) or I */
    for (int i = 0; i < r; ++i) {
        mu[i] = cexp(xi * t[i] / ssd);
        Dl[i] = (form == 1) ? alpha[i] : 1.0;
    }
    /* V <- [v_0, v_p, .., v_1] (I (x) 1^T mu / s), beta-prescaled in form 0 */
    for (int bl = 0; bl < P1; ++bl) {
        const zc *vsrc = V + (int64_t)zperm(bl, p) * n;
        for (int i = 0; i < r; ++i) {
            const zc wgt = (form == 0) ? beta[i * P1 + zperm(bl, p)] : 1.0;
            const zc sc = mu[i] / ssd;
            zc *dst = Vb + (int64_t)(bl * r + i) * n;
            for (int64_t q = 0; q < n; ++q)
                dst[q] = (vsrc[q] * wgt) * sc;
        }
    }
    /* J~ = exp(J (x) Delta / s), J <- (J (x) Delta - xi I (x) T)/s per abscissa */
    for (int i = 0; i < r; ++i) {
        zc *jt = Jt + i * P1 * P1, *js = Js + i * P1 * P1;
        for (int a = 0; a < P1 * P1; ++a)
            Nm[a] = js[a] = 0.0;
        for (int bb = 1; bb < p; ++bb)
            Nm[bb * P1 + bb + 1] = Dl[i] / ssd;
        zexpm_nilpotent(Nm, P1, jt);
        for (int bb = 0; bb < P1; ++bb)
            js[bb * P1 + bb] = (-xi * t[i]) / ssd;
        for (int bb = 1; bb < p; ++bb)
            js[bb * P1 + bb + 1] = Dl[i] / ssd;
    }
    memcpy(S, Vb, sizeof(zc) * (size_t)n * cS);
    memcpy(D, Vb, sizeof(zc) * (size_t)n * cS);
    int k = 1;
    double sigma = 1.0, c1 = INFINITY, c2 = znorm_inf(D, n, cS);
    while (c1 + c2 > tol * znorm_inf(S, n, cS)) {
        if (k >= kcap) {
            status = ORZ_ENOCONV;
            goto done;
        }
        k = k + 1;
        c1 = c2;
        sigma = k * sigma;
        /* V <- V J */
        for (int i = 0; i < r; ++i) {
            const zc *js = Js + i * P1 * P1;
            for (int bc = 0; bc < P1; ++bc) {
                zc *dst = Vn + (int64_t)(bc * r + i) * n;
                for (int64_t q = 0; q < n; ++q) {
                    zc acc = 0.0;
                    for (int bb = 0; bb < P1; ++bb)
                        acc += Vb[(int64_t)(bb * r + i) * n + q] * js[bb * P1 + bc];
                    dst[q] = acc;
                }
            }
        }
        memcpy(Vb, Vn, sizeof(zc) * (size_t)n * cS);
        /* D <- A_1 D (I (x) T/s) + V */
        for (int bb = 0; bb < P1; ++bb)
            for (int i = 0; i < r; ++i) {
                zc *dc = D + (int64_t)(bb * r + i) * n;
                const zc *vc = Vb + (int64_t)(bb * r + i) * n;
                const zc ts = t[i] / ssd;
                zapply1(A, xi, dc, y);
                for (int64_t q = 0; q < n; ++q)
                    dc[q] = y[q] * ts + vc[q];
            }
        c2 = znorm_inf(D, n, cS) / sigma;
        for (int64_t q = 0; q < (int64_t)n * cS; ++q)
            S[q] = S[q] + D[q] / sigma;
        if (isnan(c2)) {
            status = ORZ_EINVAL;
            goto done;
        }
    }
    st->terms_S = k;
    /* F = first and last block columns of S */
    for (int i = 0; i < r; ++i) {
        memcpy(F + (int64_t)i * n, S + (int64_t)i * n, sizeof(zc) * n);
        for (int64_t q = 0; q < n; ++q)
            F[(int64_t)(r + i) * n + q] = (p >= 1) ? S[(int64_t)(p * r + i) * n + q] : 0.0;
    }
    /* F(:,1:r) <- A F(:,1:r) T + v_0 1^T (weighted by beta_i0 in form 0) */
    for (int i = 0; i < r; ++i) {
        zc *fc = F + (int64_t)i * n;
        const zc w0 = (form == 0) ? beta[i * P1 + 0] : 1.0;
        zapply(A, fc, y);
        for (int64_t q = 0; q < n; ++q)
            fc[q] = y[q] * t[i] + w0 * V[q];
    }
    int tot = 0, maxstep = 0;
    for (int j = 1; j <= ss - 1; ++j) {
        memcpy(E, F, sizeof(zc) * (size_t)n * cR);
        int kk = 0;
        double d1 = INFINITY, d2 = znorm_inf(F, n, cR);
        while (d1 + d2 > tol * znorm_inf(E, n, cR)) {
            if (kk >= kcap) {
                status = ORZ_ENOCONV;
                goto done;
            }
            kk = kk + 1;
            d1 = d2;
            /* F <- A_1 F T / k */
            for (int q = 0; q < cR; ++q) {
                zc *fc = F + (int64_t)q * n;
                const zc ts = t[q % r] / ssd;
                zapply1(A, xi, fc, y);
                for (int64_t z = 0; z < n; ++z)
                    fc[z] = y[z] * ts / (double)kk;
            }
            d2 = znorm_inf(F, n, cR);
            for (int64_t z = 0; z < (int64_t)n * cR; ++z)
                E[z] = E[z] + F[z];
            if (isnan(d2)) {
                status = ORZ_EINVAL;
                goto done;
            }
        }
        tot += kk;
        if (kk > maxstep)
            maxstep = kk;
        /* E <- E mu (undo the shift) */
        for (int q = 0; q < cR; ++q)
            for (int64_t z = 0; z < n; ++z)
                E[(int64_t)q * n + z] = E[(int64_t)q * n + z] * mu[q % r];
        /* S <- S J~ */
        for (int i = 0; i < r; ++i) {
            const zc *jt = Jt + i * P1 * P1;
            for (int bc = 0; bc < P1; ++bc) {
                zc *dst = Vn + (int64_t)(bc * r + i) * n;
                for (int64_t q = 0; q < n; ++q) {
                    zc acc = 0.0;
                    for (int bb = 0; bb < P1; ++bb)
                        acc += S[(int64_t)(bb * r + i) * n + q] * jt[bb * P1 + bc];
                    dst[q] = acc;
                }
            }
        }
        memcpy(S, Vn, sizeof(zc) * (size_t)n * cS);
        /* F <- E + S(:, [block 0, block p]);  F(:,1:r) <- E(:,1:r) */
        for (int i = 0; i < r; ++i) {
            memcpy(F + (int64_t)i * n, E + (int64_t)i * n, sizeof(zc) * n);
            for (int64_t q = 0; q < n; ++q) {
                const zc e2 = E[(int64_t)(r + i) * n + q];
                F[(int64_t)(r + i) * n + q] = (p >= 1) ? e2 + S[(int64_t)(p * r + i) * n + q] : e2;
            }
        }
    }
    st->terms_rec = tot;
    st->max_terms_step = maxstep;
    /* [w_1 .. w_r] = F(:,1:r) + F(:,r+1:2r) Delta */
    for (int i = 0; i < r; ++i)
        for (int64_t q = 0; q < n; ++q)
            W[(int64_t)i * n + q] = F[(int64_t)i * n + q] + F[(int64_t)(r + i) * n + q] * Dl[i];
done:
    st->status = status;
    free(mu); free(Dl); free(Jt); free(Js); free(Vb); free(Vn);
    free(S); free(D); free(F); free(E); free(y); free(Nm);
    return status;
}
