// Complex data (Sec. 1 poses the problem for A in C^{n x n}, V in C^{n x (p+1)}
// and complex t, weights; Algorithm 3 takes a shift xi in C).
//
// Algorithm 3 over C runs in its own persistent kernel, zsolve_kernel: every
// block is column-major complex (interleaved re, im; 16 bytes an entry), one
// row per thread in a grid-stride loop over the workgroup's chunk, the blocks
// as the listing has them (the replicated, beta-prescaled V updated by the J
// step each S-series term; S advanced by exp(J/s) at each recovery step), a
// double-buffered operand for every product, and one grid exchange per
// Taylor term carrying the two block infinity norms (row sums of moduli).
//
// Algorithm 1 needs no kernel of its own: its start vector is real, its
// objective combines the powers with real coefficients and its norms are
// 2-norms, so it gives the same result on the real 2n x 2n representation
// [[Re A, -Im A], [Im A, Re A]] of A from the start vector [v; 0].  The
// operator keeps that representation as an ordinary real operator and runs
// the real parameter kernel on it.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace phc {
namespace {

constexpr int kZNT = 512;
constexpr int kZMaxGrid = 4096;
constexpr int kZCols = 4;   // columns of one product pass

struct ZDevOp {
    int64_t n;
    int kind;   // 0: CSR, 1: dense row-major
    int pad;
    const int32_t *rowptr;
    const int32_t *col;
    const double2 *val;
    const double2 *dense;
};

// Small per-solve tables (device memory, copied to LDS by every workgroup).
struct ZTables {
    double2 ts[kRMax];                      // t_i / s
    double2 t[kRMax];                       // t_i
    double2 mu[kRMax];                      // exp(xi t_i / s): undo factor of the shift
    double2 w0[kRMax];                      // beta_i0
    double2 gam[kRMax][kPMax1];             // beta_{i,perm(b)} mu_i / s
    double2 js[kRMax][kPMax1][kPMax1];      // J step (J - xi t_i I)/s
    double jt[kPMax1][kPMax1];              // exp(J/s)
};

struct ZSolveArgs {
    ZDevOp op;
    int64_t n;
    int p, r, P1, cS, cR, s_int, kcap, pad;
    double tol;
    double2 xi;
    const ZTables *tab;
    const double2 *V;    // [n][p+1] row-major (caller)
    double2 *W;          // [n][r] row-major (caller)
    double2 *Vb, *D0, *D1, *S, *F0, *F1, *E;
    unsigned *bar;
    double *part;        // [2][kZMaxGrid][kRedMax]
    int *info;           // status, terms_S, terms_rec, max_terms_step
};

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 zsc(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double zabs(double2 a) { return hypot(a.x, a.y); }

// y[c] = ((A - xi I) X)[q, c0 + c] for c < nc (<= kZCols), X column-major.
__device__ __forceinline__ void zproduct(const ZDevOp &A, int64_t q, const double2 *X, int64_t n,
                                         int c0, int nc, double2 xi, double2 (&y)[kZCols]) {
#pragma unroll
    for (int c = 0; c < kZCols; ++c)
        y[c] = make_double2(0.0, 0.0);
    const double2 *Xc = X + (int64_t)c0 * n;
    if (A.kind == 0) {
        for (int32_t z = A.rowptr[q]; z < A.rowptr[q + 1]; ++z) {
            const double2 a = A.val[z];
            const int64_t k = A.col[z];
#pragma unroll
            for (int c = 0; c < kZCols; ++c)
                if (c < nc)
                    y[c] = zadd(y[c], zmul(a, Xc[(int64_t)c * n + k]));
        }
    } else {
        const double2 *row = A.dense + q * n;
        for (int64_t k = 0; k < n; ++k) {
            const double2 a = row[k];
#pragma unroll
            for (int c = 0; c < kZCols; ++c)
                if (c < nc)
                    y[c] = zadd(y[c], zmul(a, Xc[(int64_t)c * n + k]));
        }
    }
#pragma unroll
    for (int c = 0; c < kZCols; ++c)
        if (c < nc)
            y[c] = zadd(y[c], zmul(make_double2(-xi.x, -xi.y), Xc[(int64_t)c * n + q]));
}

__global__ void zsync_init(unsigned *bar, int *info) {
    for (int i = threadIdx.x; i < kSyncLines * kLineU; i += blockDim.x)
        bar[i] = 0u;
    if (threadIdx.x < 8)
        info[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kZNT) void zsolve_kernel(ZSolveArgs P) {
    __shared__ ZTables tb;
    __shared__ double red[kZNT / 64][kRedMax];
    __shared__ int ok_lds;
    {
        const double *src = (const double *)P.tab;
        double *dst = (double *)&tb;
        for (int i = threadIdx.x; i < (int)(sizeof(ZTables) / sizeof(double)); i += kZNT)
            dst[i] = src[i];
    }
    const unsigned G = gridDim.x;
    const int lb = xcd_logical_block(blockIdx.x, G);
    const int64_t n = P.n;
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = std::min<int64_t>(n, (int64_t)lb * chunk);
    const int64_t hi = std::min<int64_t>(n, lo + chunk);
    const int tid = threadIdx.x;
    const int p = P.p, r = P.r, P1 = P.P1, cS = P.cS, cR = P.cR;
    const ZDevOp &A = P.op;
    auto finish = [&](int st, int tS, int tR, int mS) {
        if (blockIdx.x == 0 && tid == 0) {
            P.info[0] = st;
            P.info[1] = tS;
            P.info[2] = tR;
            P.info[3] = mS;
        }
    };
    GridSync gs;
    if (G > 1 && !grid_setup(gs, P.bar, &ok_lds, G)) {
        finish(PHICOMB_EDEVICE, 0, 0, 0);
        return;
    }
    __syncthreads();
    unsigned epoch = 0;
    auto exchange = [&](auto &v) __attribute__((always_inline)) -> bool {
        constexpr int NV = std::extent<std::remove_reference_t<decltype(v)>>::value;
        if (G == 1) {
            wait_own_stores();
            workgroup_max<NV, kZNT>(v, red);
            return true;
        }
        double *pt = P.part + (size_t)(epoch & 1) * kRedMax * kZMaxGrid;
        store_partials<NV, kZNT>(v, pt, red, blockIdx.x);
        if (!grid_sync(gs, &ok_lds))
            return false;
        load_partials<NV, kZNT>(pt, G, v, red);
        ++epoch;
        return true;
    };
    auto perm = [&](int b) { return b == 0 ? 0 : p + 1 - b; };
    auto col = [&](double2 *X, int c) { return X + (int64_t)c * n; };

    // ---- V <- [v_0, v_p, .., v_1] (I (x) 1^T mu / s) beta-prescaled;  S = D = V
    double mx[1] = {0.0};
    for (int64_t q = lo + tid; q < hi; q += kZNT) {
        double su = 0.0;
        for (int b = 0; b < P1; ++b) {
            const double2 vv = P.V[q * P1 + perm(b)];
            for (int i = 0; i < r; ++i) {
                const double2 u = zmul(vv, tb.gam[i][b]);
                const int c = b * r + i;
                col(P.Vb, c)[q] = u;
                col(P.D0, c)[q] = u;
                col(P.S, c)[q] = u;
                su += zabs(u);
            }
        }
        mx[0] = nmax(mx[0], su);
    }
    if (!exchange(mx)) {
        finish(PHICOMB_EDEVICE, 0, 0, 0);
        return;
    }
    if (!(mx[0] <= 1.79769313486231570e308)) {   // non-finite V (or weights)
        finish(PHICOMB_EINVAL, 0, 0, 0);
        return;
    }

    // ---- S-series (rec.D): V <- V J,  D <- A_1 D (I (x) T/s) + V,  S += D/k!
    int status = PHICOMB_OK;
    int k = 1;
    double sigma = 1.0, c1 = INFINITY, c2 = mx[0], nS = mx[0];
    int par = 0;
    while (c1 + c2 > P.tol * nS) {
        if (k >= P.kcap) {
            status = PHICOMB_ENOCONV;
            break;
        }
        k = k + 1;
        c1 = c2;
        sigma = (double)k * sigma;
        double2 *Dold = par ? P.D1 : P.D0;
        double2 *Dnew = par ? P.D0 : P.D1;
        double m2[2] = {0.0, 0.0};
        for (int64_t q = lo + tid; q < hi; q += kZNT) {
            // V <- V J (row-local).  The J step is bidiagonal: -xi t_i/s on the
            // diagonal and 1/s at (b, b+1) for 1 <= b < p, so column b takes
            // itself times the diagonal plus column b-1 over s (b >= 2);
            // descending b reads column b-1 before it changes.
            for (int i = 0; i < r; ++i) {
                const double2 dg = tb.js[i][0][0];
                for (int b = P1 - 1; b >= 0; --b) {
                    double2 &vb = col(P.Vb, b * r + i)[q];
                    double2 u = zmul(vb, dg);
                    if (b >= 2)
                        u = zadd(u, zmul(col(P.Vb, (b - 1) * r + i)[q], tb.js[i][b - 1][b]));
                    vb = u;
                }
            }
            double sd = 0.0, ss = 0.0;
            for (int c0 = 0; c0 < cS; c0 += kZCols) {
                const int nc = std::min(kZCols, cS - c0);
                double2 y[kZCols];
                zproduct(A, q, Dold, n, c0, nc, P.xi, y);
#pragma unroll
                for (int c = 0; c < kZCols; ++c) {
                    if (c < nc) {
                        const int cc = c0 + c;
                        const double2 d = zadd(zmul(y[c], tb.ts[cc % r]), col(P.Vb, cc)[q]);
                        col(Dnew, cc)[q] = d;
                        double2 &s = col(P.S, cc)[q];
                        s = zadd(s, zsc(d, 1.0 / sigma));
                        sd += zabs(d);
                        ss += zabs(s);
                    }
                }
            }
            m2[0] = nmax(m2[0], sd);
            m2[1] = nmax(m2[1], ss);
        }
        if (!exchange(m2)) {
            finish(PHICOMB_EDEVICE, k, 0, 0);
            return;
        }
        c2 = m2[0] / sigma;
        nS = m2[1];
        par ^= 1;
        if (!(c2 == c2) || !(nS == nS)) {
            status = PHICOMB_EDEVICE;
            break;
        }
    }
    const int terms_S = k;
    if (status != PHICOMB_OK) {
        finish(status, terms_S, 0, 0);
        return;
    }

    // ---- F = [S_0, S_p];  F(:,1:r) <- A F(:,1:r) T + beta_i0 v_0  (exp(t_i A/s) v_0)
    const bool one_step = (P.s_int == 1);
    {
        double m1[1] = {0.0};
        for (int64_t q = lo + tid; q < hi; q += kZNT) {
            double sf = 0.0;
            for (int c0 = 0; c0 < r; c0 += kZCols) {
                const int nc = std::min(kZCols, r - c0);
                double2 y[kZCols];
                zproduct(A, q, P.S, n, c0, nc, make_double2(0.0, 0.0), y);
#pragma unroll
                for (int c = 0; c < kZCols; ++c) {
                    if (c < nc) {
                        const int i = c0 + c;
                        const double2 f1 =
                            zadd(zmul(y[c], tb.t[i]), zmul(tb.w0[i], P.V[q * P1]));
                        const double2 f2 =
                            (p >= 1) ? col(P.S, p * r + i)[q] : make_double2(0.0, 0.0);
                        if (one_step) {
                            P.W[q * r + i] = zadd(f1, f2);
                        } else {
                            col(P.F0, i)[q] = f1;
                            col(P.E, i)[q] = f1;
                            col(P.F0, r + i)[q] = f2;
                            col(P.E, r + i)[q] = f2;
                            sf += zabs(f1) + zabs(f2);
                        }
                    }
                }
            }
            m1[0] = nmax(m1[0], sf);
        }
        if (one_step) {
            finish(PHICOMB_OK, terms_S, 0, 0);
            return;
        }
        if (!exchange(m1)) {
            finish(PHICOMB_EDEVICE, terms_S, 0, 0);
            return;
        }
        c2 = m1[0];
    }

    // ---- recovery (rec.F.shift): s-1 steps, each ended by E <- E mu,
    //      S <- S exp(J/s), F <- E + [0, S_p], and E <- F for the next step
    int tot = 0, maxstep = 0, parF = 0;
    double nF = c2;
    for (int j = 1; j <= P.s_int - 1; ++j) {
        int kk = 0;
        double d1 = INFINITY, d2 = nF, nE = nF;
        while (d1 + d2 > P.tol * nE) {
            if (kk >= P.kcap) {
                status = PHICOMB_ENOCONV;
                break;
            }
            kk = kk + 1;
            d1 = d2;
            const double rk = 1.0 / (double)kk;
            double2 *Fo = parF ? P.F1 : P.F0;
            double2 *Fn = parF ? P.F0 : P.F1;
            double m2[2] = {0.0, 0.0};
            for (int64_t q = lo + tid; q < hi; q += kZNT) {
                double sf = 0.0, se = 0.0;
                for (int c0 = 0; c0 < cR; c0 += kZCols) {
                    const int nc = std::min(kZCols, cR - c0);
                    double2 y[kZCols];
                    zproduct(A, q, Fo, n, c0, nc, P.xi, y);
#pragma unroll
                    for (int c = 0; c < kZCols; ++c) {
                        if (c < nc) {
                            const int cc = c0 + c;
                            const double2 f = zsc(zmul(y[c], tb.ts[cc % r]), rk);
                            col(Fn, cc)[q] = f;
                            double2 &e = col(P.E, cc)[q];
                            e = zadd(e, f);
                            sf += zabs(f);
                            se += zabs(e);
                        }
                    }
                }
                m2[0] = nmax(m2[0], sf);
                m2[1] = nmax(m2[1], se);
            }
            if (!exchange(m2)) {
                finish(PHICOMB_EDEVICE, terms_S, tot + kk, maxstep);
                return;
            }
            d2 = m2[0];
            nE = m2[1];
            parF ^= 1;
        }
        if (status == PHICOMB_OK && (!(d2 == d2) || !(nE == nE)))
            status = PHICOMB_EDEVICE;
        tot += kk;
        maxstep = std::max(maxstep, kk);
        if (status != PHICOMB_OK) {
            finish(status, terms_S, tot, maxstep);
            return;
        }
        const bool last = (j == P.s_int - 1);
        double2 *Fx = parF ? P.F1 : P.F0;   // the latest term: only E is needed
        double m1[1] = {0.0};
        for (int64_t q = lo + tid; q < hi; q += kZNT) {
            // S <- S exp(J/s), row-local per abscissa: exp(J/s) is upper
            // triangular with (b, b') nonzero for 1 <= b <= b' (and (0, 0) = 1),
            // so descending b' reads only columns not yet advanced
            for (int i = 0; i < r; ++i)
                for (int b = P1 - 1; b >= 1; --b) {
                    double2 acc = make_double2(0.0, 0.0);
                    for (int bb = 1; bb <= b; ++bb)
                        acc = zadd(acc, zsc(col(P.S, bb * r + i)[q], tb.jt[bb][b]));
                    col(P.S, b * r + i)[q] = acc;
                }
            double sf = 0.0;
            for (int i = 0; i < r; ++i) {
                const double2 f1 = zmul(col(P.E, i)[q], tb.mu[i]);
                double2 f2 = zmul(col(P.E, r + i)[q], tb.mu[i]);
                if (p >= 1)
                    f2 = zadd(f2, col(P.S, p * r + i)[q]);
                if (last) {
                    P.W[q * r + i] = zadd(f1, f2);
                } else {
                    col(Fx, i)[q] = f1;
                    col(Fx, r + i)[q] = f2;
                    col(P.E, i)[q] = f1;
                    col(P.E, r + i)[q] = f2;
                    sf += zabs(f1) + zabs(f2);
                }
            }
            m1[0] = nmax(m1[0], sf);
        }
        if (last)
            break;
        if (!exchange(m1)) {
            finish(PHICOMB_EDEVICE, terms_S, tot, maxstep);
            return;
        }
        nF = m1[0];
    }
    finish(status, terms_S, tot, maxstep);
}

// SplitMix64 (Steele, Lea & Flood, 2014) of (seed, i), mapped to [-1, 1): the
// start vector the real parameter kernel draws when none is given.
double splitmix_unit_host(uint64_t seed, int64_t i) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

bool finite_c(const double *a, int64_t count) {
    for (int64_t i = 0; i < 2 * count; ++i)
        if (!std::isfinite(a[i]))
            return false;
    return true;
}

}  // namespace
}  // namespace phc

struct phicomb_zop_s {
    int device = 0;
    int64_t n = 0;
    int kind = 0;
    void *mem = nullptr;              // rowptr, col, val (CSR) or the dense matrix
    phc::ZDevOp dev{};
    phicomb_op emb = nullptr;         // real 2n x 2n representation (Algorithm 1)
    std::mutex mu;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int *pinned = nullptr;
};

namespace {
using namespace phc;

void zop_free(phicomb_zop z) {
    if (!z)
        return;
    if (z->emb)
        phicomb_op_destroy(z->emb);
    if (z->mem)
        (void)hipFree(z->mem);
    if (z->ws)
        (void)hipFree(z->ws);
    if (z->pinned)
        (void)hipHostFree(z->pinned);
    delete z;
}

// The real representation [[Re A, -Im A], [Im A, Re A]] as CSR rows, from
// complex CSR rows (entries with a zero part are left out).
int make_embedding(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                   phicomb_op *out) {
    const int64_t nnz = rowptr[n];
    if (4 * nnz > INT32_MAX)
        return PHICOMB_EINVAL;
    std::vector<int32_t> rp(2 * n + 1, 0), ci;
    std::vector<double> va;
    ci.reserve(2 * nnz);
    va.reserve(2 * nnz);
    for (int half = 0; half < 2; ++half)
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t z = rowptr[i]; z < rowptr[i + 1]; ++z) {
                const double re = val[2 * z], im = val[2 * z + 1];
                // row i (real part): Re A x_re - Im A x_im;  row n+i: Im A x_re + Re A x_im
                const double a0 = half == 0 ? re : im, a1 = half == 0 ? -im : re;
                if (a0 != 0.0) {
                    ci.push_back(col[z]);
                    va.push_back(a0);
                }
                if (a1 != 0.0) {
                    ci.push_back((int32_t)(n + col[z]));
                    va.push_back(a1);
                }
            }
            rp[half * n + i + 1] = (int32_t)ci.size();
        }
    if (va.empty()) {   // the zero operator: keep one explicit zero per row
        ci.assign(2 * n, 0);
        va.assign(2 * n, 0.0);
        for (int64_t i = 0; i < 2 * n; ++i) {
            ci[i] = (int32_t)i;
            rp[i + 1] = (int32_t)(i + 1);
        }
    }
    return phicomb_op_create_csr(2 * n, rp.data(), ci.data(), va.data(), out);
}

}  // namespace

using namespace phc;

extern "C" {

int phicomb_zop_create_csr(int64_t n, const int32_t *rowptr, const int32_t *col,
                           const double *val, phicomb_zop *out) {
    if (!out || n < 1 || 2 * n > kMaxRows || !rowptr || !col || !val)
        return PHICOMB_EINVAL;
    *out = nullptr;
    if (rowptr[0] != 0)
        return PHICOMB_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return PHICOMB_EINVAL;
    const int64_t nnz = rowptr[n];
    for (int64_t z = 0; z < nnz; ++z)
        if (col[z] < 0 || col[z] >= n)
            return PHICOMB_EINVAL;
    if (!finite_c(val, nnz))
        return PHICOMB_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return PHICOMB_EDEVICE;
    phicomb_zop z = new (std::nothrow) phicomb_zop_s();
    if (!z)
        return PHICOMB_ENOMEM;
    z->device = dev;
    z->n = n;
    z->kind = 0;
    int st = make_embedding(n, rowptr, col, val, &z->emb);
    const size_t b_rp = sizeof(int32_t) * (size_t)(n + 1), b_ci = sizeof(int32_t) * (size_t)nnz;
    const size_t o_ci = (b_rp + 15) / 16 * 16, o_va = (o_ci + b_ci + 15) / 16 * 16;
    const size_t bytes = o_va + 16 * (size_t)std::max<int64_t>(nnz, 1);
    if (st == PHICOMB_OK && hipMalloc(&z->mem, bytes) != hipSuccess)
        st = PHICOMB_ENOMEM;
    char *m = (char *)z->mem;
    if (st == PHICOMB_OK &&
        (hipMemcpy(m, rowptr, b_rp, hipMemcpyHostToDevice) != hipSuccess ||
         (nnz > 0 && hipMemcpy(m + o_ci, col, b_ci, hipMemcpyHostToDevice) != hipSuccess) ||
         (nnz > 0 && hipMemcpy(m + o_va, val, 16 * (size_t)nnz, hipMemcpyHostToDevice) !=
                         hipSuccess)))
        st = PHICOMB_EDEVICE;
    if (st != PHICOMB_OK) {
        zop_free(z);
        return st;
    }
    z->dev.n = n;
    z->dev.kind = 0;
    z->dev.rowptr = (const int32_t *)m;
    z->dev.col = (const int32_t *)(m + o_ci);
    z->dev.val = (const double2 *)(m + o_va);
    *out = z;
    return PHICOMB_OK;
}

int phicomb_zop_create_dense(int64_t n, const double *A, phicomb_zop *out) {
    if (!out || n < 1 || n > 16384 || !A)
        return PHICOMB_EINVAL;
    *out = nullptr;
    if (!finite_c(A, n * n))
        return PHICOMB_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return PHICOMB_EDEVICE;
    // CSR rows with every column present serve the real representation
    std::vector<int32_t> rp(n + 1), ci((size_t)n * n);
    for (int64_t i = 0; i <= n; ++i)
        rp[i] = (int32_t)(i * n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            ci[(size_t)i * n + j] = (int32_t)j;
    phicomb_zop z = new (std::nothrow) phicomb_zop_s();
    if (!z)
        return PHICOMB_ENOMEM;
    z->device = dev;
    z->n = n;
    z->kind = 1;
    int st = make_embedding(n, rp.data(), ci.data(), A, &z->emb);
    const size_t bytes = 16 * (size_t)n * (size_t)n;
    if (st == PHICOMB_OK && hipMalloc(&z->mem, bytes) != hipSuccess)
        st = PHICOMB_ENOMEM;
    if (st == PHICOMB_OK && hipMemcpy(z->mem, A, bytes, hipMemcpyHostToDevice) != hipSuccess)
        st = PHICOMB_EDEVICE;
    if (st != PHICOMB_OK) {
        zop_free(z);
        return st;
    }
    z->dev.n = n;
    z->dev.kind = 1;
    z->dev.dense = (const double2 *)z->mem;
    *out = z;
    return PHICOMB_OK;
}

int phicomb_zop_destroy(phicomb_zop op) {
    if (!op)
        return PHICOMB_EINVAL;
    (void)hipDeviceSynchronize();
    zop_free(op);
    return PHICOMB_OK;
}

int phicomb_zparams(phicomb_zop op, double tol, int m, const double *v, uint64_t seed,
                    void *stream, phicomb_params_t *out) {
    if (!op || !out || (v && !std::isfinite(v[0])))
        return PHICOMB_EINVAL;
    const int64_t n = op->n;
    std::vector<double> v2(2 * n, 0.0);   // [v; 0]: the real start vector
    for (int64_t i = 0; i < n; ++i)
        v2[i] = v ? v[i] : splitmix_unit_host(seed, i);
    return phicomb_params(op->emb, tol, m, v2.data(), seed, stream, out);
}

int phicomb_zsolve(phicomb_zop op, const phicomb_params_t *prm, const double *shift, int p,
                   int r, const double *t, const double *beta, const void *V, double tol,
                   void *W, void *stream, phicomb_stats_t *stats) {
    if (!op || !prm || !t || !beta || !V || !W)
        return PHICOMB_EINVAL;
    if (p < 0 || p > PHICOMB_MAX_P || r < 1 || r > PHICOMB_MAX_R)
        return PHICOMB_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol) || prm->status != PHICOMB_OK ||
        !std::isfinite(prm->s) || prm->s < 0.0 || !std::isfinite(prm->shift))
        return PHICOMB_EINVAL;
    if (!finite_c(t, r) || !finite_c(beta, (int64_t)r * (p + 1)) ||
        (shift && !finite_c(shift, 1)))
        return PHICOMB_EINVAL;
    const std::complex<double> xi =
        shift ? std::complex<double>(shift[0], shift[1]) : std::complex<double>(prm->shift, 0.0);
    const int64_t n = op->n;
    const int P1 = p + 1, cS = P1 * r, cR = 2 * r;
    double tmax = 0.0;
    std::complex<double> tc[kRMax];
    for (int i = 0; i < r; ++i) {
        tc[i] = std::complex<double>(t[2 * i], t[2 * i + 1]);
        tmax = std::max(tmax, std::abs(tc[i]));
    }
    const double sceil = std::ceil(prm->s * tmax);
    if (!(sceil <= 2147483647.0))
        return PHICOMB_EINVAL;
    const int ss = sceil < 1.0 ? 1 : (int)sceil;
    const double ssd = (double)ss;
    // tables (Algorithm 3's set-up lines, beta-prescaled form: Delta = I)
    ZTables tb;
    std::memset(&tb, 0, sizeof(tb));
    auto put = [](double2 &d, std::complex<double> z) { d = make_double2(z.real(), z.imag()); };
    for (int i = 0; i < r; ++i) {
        const std::complex<double> mu = std::exp(xi * tc[i] / ssd);
        put(tb.ts[i], tc[i] / ssd);
        put(tb.t[i], tc[i]);
        put(tb.mu[i], mu);
        put(tb.w0[i], std::complex<double>(beta[2 * (i * P1)], beta[2 * (i * P1) + 1]));
        for (int b = 0; b < P1; ++b) {
            const int pb = (b == 0) ? 0 : p + 1 - b;
            const std::complex<double> bt(beta[2 * (i * P1 + pb)], beta[2 * (i * P1 + pb) + 1]);
            put(tb.gam[i][b], bt * mu / ssd);
        }
        for (int b = 0; b < P1; ++b)
            put(tb.js[i][b][b], -xi * tc[i] / ssd);
        for (int b = 1; b < p; ++b)
            put(tb.js[i][b][b + 1], std::complex<double>(1.0 / ssd, 0.0));
    }
    // exp(N/s), N the ones at (b, b+1), 1 <= b < p: (N/s)^d / d! on the d-th superdiagonal
    for (int b = 0; b < P1; ++b)
        tb.jt[b][b] = 1.0;
    for (int b = 1; b < p; ++b) {
        double term = 1.0;
        for (int d = 1; b + d <= p; ++d) {
            term = term / (ssd * (double)d);
            tb.jt[b][b + d] = term;
        }
    }
    std::lock_guard<std::mutex> g(op->mu);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return PHICOMB_EDEVICE;
    if (cur != op->device)
        return PHICOMB_EINVAL;   // the operator lives on another device
    const size_t blocks = 16 * (size_t)n * (size_t)(4 * cS + 3 * cR);
    const size_t o_tab = (blocks + 255) / 256 * 256;
    const size_t o_bar = o_tab + (sizeof(ZTables) + 255) / 256 * 256;
    const size_t o_part = o_bar + kSyncBytes;
    const size_t o_info = o_part + sizeof(double) * 2 * kRedMax * kZMaxGrid;
    const size_t need = o_info + 256;
    if (op->ws_bytes < need) {
        if (op->ws)
            (void)hipFree(op->ws);
        op->ws = nullptr;
        op->ws_bytes = 0;
        if (hipMalloc(&op->ws, need) != hipSuccess)
            return PHICOMB_ENOMEM;
        op->ws_bytes = need;
    }
    if (!op->pinned && hipHostMalloc((void **)&op->pinned, 64) != hipSuccess)
        return PHICOMB_ENOMEM;
    char *w = (char *)op->ws;
    ZSolveArgs a;
    std::memset(&a, 0, sizeof(a));
    a.op = op->dev;
    a.n = n;
    a.p = p;
    a.r = r;
    a.P1 = P1;
    a.cS = cS;
    a.cR = cR;
    a.s_int = ss;
    a.kcap = kTermCap;
    a.tol = tol;
    a.xi = make_double2(xi.real(), xi.imag());
    a.tab = (const ZTables *)(w + o_tab);
    a.V = (const double2 *)V;
    a.W = (double2 *)W;
    double2 *d = (double2 *)w;
    a.Vb = d;
    d += (size_t)n * cS;
    a.D0 = d;
    d += (size_t)n * cS;
    a.D1 = d;
    d += (size_t)n * cS;
    a.S = d;
    d += (size_t)n * cS;
    a.F0 = d;
    d += (size_t)n * cR;
    a.F1 = d;
    d += (size_t)n * cR;
    a.E = d;
    a.bar = (unsigned *)(w + o_bar);
    a.part = (double *)(w + o_part);
    a.info = (int *)(w + o_info);
    hipStream_t s = (hipStream_t)stream;
    const int want = (int)std::min<int64_t>(device_cus(op->device), (n + kZNT - 1) / kZNT);
    const int granted = cu_acquire(op->device, want, 1);
    if (granted < 1)
        return PHICOMB_EDEVICE;
    const int G = std::min(want, granted);
    struct Hold {
        int dev, g;
        ~Hold() { cu_release(dev, g); }
    } hold{op->device, granted};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    int st = PHICOMB_OK;
    if (hipMemcpyAsync(w + o_tab, &tb, sizeof(tb), hipMemcpyHostToDevice, s) != hipSuccess)
        st = PHICOMB_EDEVICE;
    if (st == PHICOMB_OK) {
        zsync_init<<<1, 256, 0, s>>>(a.bar, a.info);
        if (timed)
            (void)hipEventRecord(e0, s);
        void *args[] = {&a};
        if (launch_persistent((const void *)zsolve_kernel, (unsigned)G, kZNT, args, s) !=
            hipSuccess)
            st = PHICOMB_EDEVICE;
        if (timed)
            (void)hipEventRecord(e1, s);
    }
    if (st == PHICOMB_OK &&
        (hipMemcpyAsync(op->pinned, a.info, 8 * sizeof(int), hipMemcpyDeviceToHost, s) !=
             hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        st = PHICOMB_EDEVICE;
    if (st == PHICOMB_OK) {
        st = op->pinned[0];
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->s_int = ss;
            stats->terms_S = op->pinned[1];
            stats->terms_rec = op->pinned[2];
            stats->max_terms_step = op->pinned[3];
            stats->status = st;
            float ms = 0.0f;
            if (timed && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                stats->ms = ms;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    return st;
}

}  // extern "C"
