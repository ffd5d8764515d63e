/* Reference action of the augmented exponential in quadruple precision
 * (test infrastructure; shares nothing with the oracle or the HIP library).
 *
 * For one abscissa t and weights beta[0..p], w = sum_j beta_j phi_j(tA) v_j
 * is the first n entries of exp(M) r with the augmented matrix
 *     M = [ tA   B ]      B = [beta_p v_p, ..., beta_1 v_1]   (n x p)
 *         [ 0    J ]      J = ones on the superdiagonal      (p x p)
 * and r = [beta_0 v_0; e_p] (Theorem 1 of the paper and its proof; the same
 * construction as the multiprecision helper in refs.py).  exp(M) is the
 * textbook Taylor series of the scaled matrix M / 2^s (||M / 2^s||_1 <= 1/4,
 * summed until the terms fall below 1e-40 of the sum) squared s times, in
 * __float128 (unit roundoff 1e-34).
 *
 *     gcc -O2 -shared -fPIC exact_q.c -o libexact_q.so -lquadmath
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 q;

static void matmul(int N, const q *X, const q *Y, q *Z) {
    for (int i = 0; i < N; ++i) {
        q *zi = Z + (size_t)i * N;
        for (int j = 0; j < N; ++j)
            zi[j] = 0;
        for (int k = 0; k < N; ++k) {
            const q xik = X[(size_t)i * N + k];
            if (xik == 0)
                continue;
            const q *yk = Y + (size_t)k * N;
            for (int j = 0; j < N; ++j)
                zi[j] += xik * yk[j];
        }
    }
}

static q norm1(int N, const q *X) {
    q best = 0;
    for (int j = 0; j < N; ++j) {
        q s = 0;
        for (int i = 0; i < N; ++i)
            s += fabsq(X[(size_t)i * N + j]);
        if (s > best)
            best = s;
    }
    return best;
}

/* A: row-major n x n; V: row-major n x (p+1); w: n outputs.  0 on success. */
int aug_expm_q(int n, int p, const double *A, double t, const double *beta, const double *V,
               double *w) {
    const int N = n + p;
    q *M = calloc((size_t)N * N, sizeof(q));
    q *T = calloc((size_t)N * N, sizeof(q));
    q *P = calloc((size_t)N * N, sizeof(q));
    q *X = calloc((size_t)N * N, sizeof(q));
    if (!M || !T || !P || !X) {
        free(M), free(T), free(P), free(X);
        return -1;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            M[(size_t)i * N + j] = (q)t * (q)A[(size_t)i * n + j];
    for (int c = 0; c < p; ++c) {
        const int jj = p - c;
        for (int i = 0; i < n; ++i)
            M[(size_t)i * N + n + c] = (q)beta[jj] * (q)V[(size_t)i * (p + 1) + jj];
    }
    for (int c = 0; c + 1 < p; ++c)
        M[(size_t)(n + c) * N + n + c + 1] = 1;
    /* scaling */
    const q nm = norm1(N, M);
    int s = 0;
    while (nm / powq(2, s) > 0.25Q)
        ++s;
    const q sc = powq(2, -s);
    for (size_t k = 0; k < (size_t)N * N; ++k)
        M[k] *= sc;
    /* Taylor: T = sum_k M^k / k! */
    for (int i = 0; i < N; ++i)
        T[(size_t)i * N + i] = 1, P[(size_t)i * N + i] = 1;
    for (int k = 1; k <= 60; ++k) {
        matmul(N, P, M, X);
        for (size_t e = 0; e < (size_t)N * N; ++e)
            P[e] = X[e] / k;
        for (size_t e = 0; e < (size_t)N * N; ++e)
            T[e] += P[e];
        if (norm1(N, P) <= 1e-40Q * norm1(N, T))
            break;
    }
    /* squaring */
    for (int k = 0; k < s; ++k) {
        matmul(N, T, T, X);
        memcpy(T, X, sizeof(q) * (size_t)N * N);
    }
    /* apply to r = [beta_0 v_0; e_p] */
    for (int i = 0; i < n; ++i) {
        q acc = 0;
        for (int j = 0; j < n; ++j)
            acc += T[(size_t)i * N + j] * ((q)beta[0] * (q)V[(size_t)j * (p + 1)]);
        if (p > 0)
            acc += T[(size_t)i * N + N - 1];
        w[i] = (double)acc;
    }
    free(M), free(T), free(P), free(X);
    return 0;
}
