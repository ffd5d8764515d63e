// Parameter selection (Al-Mohy, Sec. 3, Algorithm 1) on the device, FP64, in
// one persistent kernel.
//
//   V_0 = v/||v||_2;  W_k = A V_{k-1}, L_k = log||W_k||_2, accepted while
//   L_k + log(k+1)/2 + max_j log binom(m,j) <= 0.8 log(realmax) and
//   L_k >= 0.8 log(realmin);  s0 = exp(mean of the last (<= 5) log-growth
//   ratios, excluding the newest);  V_j <- s0^-j V_j;  V_k = A V_{k-1}/s0 up
//   to degree m;  f(xi) = ||V (b .* [z^m .. z 1])||_2^(1/m) with z = -xi/s0,
//   minimised by Brent's method over z in [-sqrt(n), sqrt(n)];
//   s = s0 f(xi*) / (tol m!)^(1/m).
//
// The basis is [m+1][n] (column-major).  Each 2-norm is a scaled sum of
// squares (scale, ssq) merged per thread, per wave in a fixed shuffle tree,
// per workgroup in wave order, and finally over all workgroups in index
// order by every workgroup on its own, so all threads hold the same value,
// take the same guard and Brent decisions, and repeated runs give identical
// parameters.  Brent's iteration runs redundantly in every thread; each
// objective evaluation is one pass over the basis plus one grid exchange.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace phc {

constexpr int kPNT = 512;          // threads per workgroup (register-cached CSR rows)
constexpr int kPNTWide = 1024;     // threads per workgroup (every other operator)
constexpr int kParamRows = 4;      // rows per thread of the register-cached CSR variant
constexpr int kPMaxGrid = 4096;

// (scale, ssq) pair: value = scale * sqrt(ssq), scale = max |x| seen.
struct Ssq {
    double scale, ssq;
};

__device__ __forceinline__ void ssq_add(Ssq &a, double x) {
    const double ax = fabs(x);
    if (ax == 0.0)
        return;
    if (!(ax <= a.scale)) {   // also taken for NaN / first value
        const double q = (a.scale == 0.0) ? 0.0 : a.scale / ax;
        a.ssq = 1.0 + a.ssq * q * q;
        a.scale = ax;
    } else {
        const double q = ax / a.scale;
        a.ssq += q * q;
    }
}

__device__ __forceinline__ Ssq ssq_merge(Ssq a, Ssq b) {
    if (b.scale == 0.0)
        return a;
    if (a.scale == 0.0)
        return b;
    if (a.scale >= b.scale) {
        const double q = b.scale / a.scale;
        a.ssq += b.ssq * q * q;
        return a;
    }
    const double q = a.scale / b.scale;
    b.ssq += a.ssq * q * q;
    return b;
}

__device__ __forceinline__ Ssq wave_ssq(Ssq v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Ssq o;
        o.scale = __shfl_xor(v.scale, off, 64);
        o.ssq = __shfl_xor(v.ssq, off, 64);
        // both partners merge (lower lane, upper lane) in the same order
        const bool lower = (threadIdx.x & off) == 0;
        v = lower ? ssq_merge(v, o) : ssq_merge(o, v);
    }
    return v;
}

__device__ __forceinline__ double ssq_log(Ssq s) {
    return (s.scale == 0.0) ? -INFINITY : log(s.scale) + 0.5 * log(s.ssq);
}

struct ParamsArgs {
    DevOp op;
    int64_t n;
    int m, have_v, brent_maxit, pad;
    uint64_t seed;
    double tol, gmax, gmin, lmax, zmax, brent_rel, brent_abs;
    const double *binom;   // [m+1] exact binomials (device)
    double *basis;      // [m+1][n]
    unsigned *bar;      // sync area
    double *part;       // [2][kPMaxGrid][2]
    double *lrpart;     // low rank: [2][hi, lo][kLrRankMax][kPMaxGrid] partial W^T x
    double *out;        // 16 values, see params_fp64
};

__global__ void params_sync_init(unsigned *bar, double *out) {
    for (int i = threadIdx.x; i < kSyncLines * kLineU; i += blockDim.x)
        bar[i] = 0u;
    if (threadIdx.x < 16)
        out[threadIdx.x] = 0.0;
}

// SplitMix64 (Steele, Lea & Flood, 2014) of (seed, i), mapped to [-1, 1).
__device__ __forceinline__ double splitmix_unit(uint64_t seed, int64_t i) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// One lane's share of a dense row times x, one fused multiply-add a term.
// Whole blocks of 128 kRowPairs entries first: lane l takes the pairs
// (c, c + 1), c = 2 l + 128 u, each with one 16-byte load of A and of x, all
// of a block's loads issued before its multiply-adds; then the rest of the
// row (under 128 kRowPairs entries) in steps of 64 entries, c = lane + 64 u,
// kRowSteps loads at a time (clamped into the row, entries past it skipped).
constexpr int kRowPairs = 4;
constexpr int kRowSteps = 8;
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ double dense_row_dot(const double *__restrict__ arow,
                                                const double *__restrict__ x, int64_t n,
                                                int lane) {
    double sum = 0.0;
    int64_t b = 0;
    for (; b + 128 * kRowPairs <= n; b += 128 * kRowPairs) {
        dbl2u av[kRowPairs], xv[kRowPairs];
#pragma unroll
        for (int u = 0; u < kRowPairs; ++u) {
            const int64_t c = b + 128 * u + 2 * lane;
            av[u] = *(const dbl2u *)(arow + c);
            xv[u] = *(const dbl2u *)(x + c);
        }
#pragma unroll
        for (int u = 0; u < kRowPairs; ++u) {
            sum = __builtin_fma(av[u].x, xv[u].x, sum);
            sum = __builtin_fma(av[u].y, xv[u].y, sum);
        }
    }
    for (; b < n; b += 64 * kRowSteps) {
        double av[kRowSteps], xv[kRowSteps];
#pragma unroll
        for (int u = 0; u < kRowSteps; ++u) {
            const int64_t c = b + 64 * u + lane;
            const int64_t cc = c < n ? c : n - 1;
            av[u] = arow[cc];
            xv[u] = x[cc];
        }
#pragma unroll
        for (int u = 0; u < kRowSteps; ++u)
            if (b + 64 * u + lane < n)
                sum = __builtin_fma(av[u], xv[u], sum);
    }
    return sum;
}

template <int KIND, int NT>
__device__ __forceinline__ void params_body(const ParamsArgs &P) {
    __shared__ double wsc[NT / 64], wsq[NT / 64];
    __shared__ double coef[PHICOMB_MAX_M + 1];
    __shared__ double lrc[kLrRankMax];
    __shared__ int ok_lds;
    const unsigned G = gridDim.x;
    const int lb = xcd_logical_block(blockIdx.x, G);
    const int64_t n = P.n;
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = std::min<int64_t>(n, (int64_t)lb * chunk);
    const int64_t hi = std::min<int64_t>(n, lo + chunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = P.m;
    const DevOp &A = P.op;
    double *basis = P.basis;
    // CSR rows of at most kCacheNnz entries, up to kParamRows per thread, stay
    // in registers for all the powers
    constexpr bool CACHED = (KIND == kCsrCached);
    CachedRow crow[CACHED ? kParamRows : 1];
    if constexpr (CACHED) {
#pragma unroll
        for (int q = 0; q < kParamRows; ++q) {
            const int64_t row = lo + tid + (int64_t)q * NT;
            if (row < hi)
                load_cached_row(A, row, crow[q]);
        }
    }
    auto col = [&](int k) { return basis + (int64_t)k * n; };
    auto finish = [&](double status, double r, double s0, double zs, double fs, double shift,
                      double s, double nfev) {
        if (blockIdx.x == 0 && tid == 0) {
            double *o = P.out;
            o[0] = status; o[1] = r; o[2] = s0; o[3] = zs; o[4] = fs; o[5] = shift;
            o[6] = s; o[7] = nfev;
        }
    };

    GridSync gs;
    if (!grid_setup(gs, P.bar, &ok_lds, gridDim.x)) {
        finish(PHICOMB_EDEVICE, 0, 0, 0, 0, 0, 0, 0);
        return;
    }
    unsigned epoch = 0;
    bool alive = true;
    // Deterministic global 2-norm: every workgroup ends with the same value.
    auto exchange = [&](Ssq v) __attribute__((always_inline)) -> Ssq {
        v = wave_ssq(v);
        __syncthreads();
        if (lane == 0) {
            wsc[wave] = v.scale;
            wsq[wave] = v.ssq;
        }
        __syncthreads();
        double *pt = P.part + (size_t)(epoch & 1) * 2 * kPMaxGrid;
        if (tid == 0) {
            Ssq acc{wsc[0], wsq[0]};
            for (int w = 1; w < NT / 64; ++w)
                acc = ssq_merge(acc, Ssq{wsc[w], wsq[w]});
            pt[blockIdx.x * 2] = acc.scale;
            pt[blockIdx.x * 2 + 1] = acc.ssq;
        }
        if (!grid_sync(gs, &ok_lds))
            alive = false;
        Ssq acc{0.0, 0.0};
        for (unsigned b = tid; b < G; b += NT)
            acc = ssq_merge(acc, Ssq{pt[b * 2], pt[b * 2 + 1]});
        acc = wave_ssq(acc);
        __syncthreads();
        if (lane == 0) {
            wsc[wave] = acc.scale;
            wsq[wave] = acc.ssq;
        }
        __syncthreads();
        Ssq tot{wsc[0], wsq[0]};
        for (int w = 1; w < NT / 64; ++w)
            tot = ssq_merge(tot, Ssq{wsc[w], wsq[w]});
        ++epoch;
        return tot;
    };
    // Low rank (A = U W^T, applied as x -> U (W^T x)): lrc = W^T x, each
    // workgroup's partial over its rows, then the sum over all workgroups in
    // index order, the same in every workgroup.
    unsigned lr_epoch = 0;
    const size_t lr_lo = (size_t)kLrRankMax * kPMaxGrid;   // [2 parities][hi, lo][rank][grid]
    auto lr_dot = [&](const double *x) __attribute__((always_inline)) -> bool {
        __syncthreads();   // this workgroup's rows of x are written
        double *pt = P.lrpart + (size_t)(lr_epoch & 1) * 2 * lr_lo;
        const int rank = A.rank;
        for (int k = wave; k < rank; k += NT / 64) {
            DD acc{0.0, 0.0};
            for (int64_t row = lo + lane; row < hi; row += 64)
                dd_fma(acc, A.lr_w[row * rank + k], x[row]);
            acc = wave_sum_dd(acc);
            if (lane == 0) {
                pt[(size_t)k * kPMaxGrid + blockIdx.x] = acc.hi;
                pt[(size_t)k * kPMaxGrid + blockIdx.x + lr_lo] = acc.lo;
            }
        }
        if (!grid_sync(gs, &ok_lds))
            return false;
        for (int k = wave; k < rank; k += NT / 64) {
            DD acc{0.0, 0.0};
            for (unsigned b = lane; b < G; b += 64)
                acc = dd_add(acc, DD{pt[(size_t)k * kPMaxGrid + b],
                                     pt[(size_t)k * kPMaxGrid + b + lr_lo]});
            acc = wave_sum_dd(acc);
            if (lane == 0)
                lrc[k] = acc.hi + acc.lo;
        }
        __syncthreads();
        ++lr_epoch;
        return true;
    };
    auto lr_row = [&](int64_t row) __attribute__((always_inline)) -> double {
        const double *ur = A.lr_u + row * A.rank;
        double y = 0.0;
        for (int k = 0; k < A.rank; ++k)
            y += ur[k] * lrc[k];
        return y;
    };

    // ---- V_0 = v / ||v||
    if (!P.have_v)
        for (int64_t row = lo + tid; row < hi; row += NT)
            basis[row] = splitmix_unit(P.seed, row);
    Ssq a{0.0, 0.0};
    for (int64_t row = lo + tid; row < hi; row += NT)
        ssq_add(a, basis[row]);
    const Ssq vs = exchange(a);
    const double nv = vs.scale * sqrt(vs.ssq);
    if (!alive) {
        finish(PHICOMB_EDEVICE, 0, 0, 0, 0, 0, 0, 0);
        return;
    }
    if (!(nv > 0.0) || !(nv <= DBL_MAX)) {
        finish(PHICOMB_EINVAL, 0, 0, 0, 0, 0, 0, 0);
        return;
    }

    // ---- guarded powers W_k = A V_{k-1}
    double Lh[7];   // L_{k-6} .. L_k, newest last
#pragma unroll
    for (int j = 0; j < 7; ++j)
        Lh[j] = 0.0;
    int r = 0;
    double L1 = 0.0;
    for (int k = 1; k <= m; ++k) {
        const double *x = col(k - 1);
        double *y = col(k);
        Ssq acc{0.0, 0.0};
        if constexpr (KIND == kLowRank) {
            if (!lr_dot(x)) {
                finish(PHICOMB_EDEVICE, 0, 0, 0, 0, 0, 0, 0);
                return;
            }
            for (int64_t row = lo + tid; row < hi; row += NT) {
                const double w = lr_row(row);
                const double val = (k == 1) ? w / nv : w;   // A (v/||v||)
                y[row] = val;
                ssq_add(acc, val);
            }
        } else if constexpr (KIND == kDense) {
            // dense rows: one wave per row, lanes across the row, wave sum
            for (int64_t row = lo + (tid >> 6); row < hi; row += NT / 64) {
                double sum = dense_row_dot(A.dense + row * n, x, n, tid & 63);
                sum = wave_sum(sum);
                if ((tid & 63) == 0) {
                    const double val = (k == 1) ? sum / nv : sum;   // A (v/||v||)
                    y[row] = val;
                    ssq_add(acc, val);
                }
            }
        } else if constexpr (CACHED) {
#pragma unroll
            for (int q = 0; q < kParamRows; ++q) {
                const int64_t row = lo + tid + (int64_t)q * NT;
                if (row < hi) {
                    double w[1];
                    apply_cached<1>(crow[q], (unsigned)row, x, n, 0, 0.0, w);
                    const double val = (k == 1) ? w[0] / nv : w[0];   // A (v/||v||)
                    y[row] = val;
                    ssq_add(acc, val);
                }
            }
        } else {
            for (int64_t row = lo + tid; row < hi; row += NT) {
                const RowCtx rc = row_ctx<KIND>(A, row);
                double w[1];
                apply_cols<KIND, 1>(A, rc, x, n, 0, 0.0, w);
                const double val = (k == 1) ? w[0] / nv : w[0];   // A (v/||v||)
                y[row] = val;
                ssq_add(acc, val);
            }
        }
        const double Lk = ssq_log(exchange(acc));
        if (!alive) {
            finish(PHICOMB_EDEVICE, 0, 0, 0, 0, 0, 0, 0);
            return;
        }
        if (k == 1) {
            L1 = Lk;
            for (int64_t row = lo + tid; row < hi; row += NT)   // nobody reads V_0 again
                basis[row] = basis[row] / nv;
        }
        if (Lk != Lk) {
            finish(PHICOMB_EINVAL, 0, 0, 0, 0, 0, 0, 0);
            return;
        }
        if (Lk + 0.5 * log(k + 1.0) + P.lmax > P.gmax || Lk < P.gmin)
            break;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            Lh[j] = Lh[j + 1];
        Lh[6] = Lk;
        r = k;
    }
    if (r == 0) {
        if (L1 < P.gmin)   // A v vanishes: A is treated as zero
            finish(PHICOMB_OK, 0, 0, 0, 0, 0, 1.0, 0);
        else
            finish(PHICOMB_EOVERFLOW, 0, 0, 0, 0, 0, 0, 0);
        return;
    }
    // s0 from the last accepted ratios L_{j+1} - L_j, j = jr .. r-1 (Lh[6] = L_r)
    double s0;
    if (r >= 3) {
        const int jr = std::max(2, r - 5);
        const int cnt = r - jr;   // 1..5 ratios L_{j+1} - L_j, j = jr .. r-1
        double sum = 0.0;
#pragma unroll
        for (int d = 5; d >= 1; --d)   // d = r - j, so ascending j
            if (d <= cnt)
                sum += Lh[7 - d] - Lh[6 - d];
        s0 = exp(sum / (double)cnt);
    } else {
        s0 = exp(Lh[6] / (double)r);
    }
    // ---- normalise V_j by s0^-j, then extend to degree m
    const double ls0 = log(s0);
    for (int j = 1; j <= r; ++j) {
        const double sc = exp(-(double)j * ls0);
        double *v = col(j);
        for (int64_t row = lo + tid; row < hi; row += NT)
            v[row] = v[row] * sc;
    }
    for (int k = r + 1; k <= m; ++k) {
        const double *x = col(k - 1);
        double *y = col(k);
        // low rank: only this workgroup's rows of x are read, after lr_dot's barrier
        if (!(KIND == kLowRank ? lr_dot(x) : grid_sync(gs, &ok_lds))) {
            finish(PHICOMB_EDEVICE, r, s0, 0, 0, 0, 0, 0);
            return;
        }
        if constexpr (KIND == kLowRank) {
            for (int64_t row = lo + tid; row < hi; row += NT)
                y[row] = lr_row(row) / s0;
        } else if constexpr (KIND == kDense) {
            for (int64_t row = lo + (tid >> 6); row < hi; row += NT / 64) {
                double sum = dense_row_dot(A.dense + row * n, x, n, tid & 63);
                sum = wave_sum(sum);
                if ((tid & 63) == 0)
                    y[row] = sum / s0;
            }
        } else if constexpr (CACHED) {
#pragma unroll
            for (int q = 0; q < kParamRows; ++q) {
                const int64_t row = lo + tid + (int64_t)q * NT;
                if (row < hi) {
                    double w[1];
                    apply_cached<1>(crow[q], (unsigned)row, x, n, 0, 0.0, w);
                    y[row] = w[0] / s0;
                }
            }
        } else {
            for (int64_t row = lo + tid; row < hi; row += NT) {
                const RowCtx rc = row_ctx<KIND>(A, row);
                double w[1];
                apply_cols<KIND, 1>(A, rc, x, n, 0, 0.0, w);
                y[row] = w[0] / s0;
            }
        }
    }

    // ---- objective f(z) = ||sum_k b_k z^(m-k) V_k||^(1/m); every row of the
    //      basis read here was written inside this workgroup, before the
    //      workgroup barrier that opens each evaluation
    auto objective = [&](double z) __attribute__((always_inline)) -> double {
        __syncthreads();
        if (tid <= m) {
            double pw = 1.0;   // z^(m-k), built by repeated multiplication
            for (int e = 0; e < m - tid; ++e)
                pw = pw * z;
            coef[tid] = P.binom[tid] * pw;
        }
        __syncthreads();
        // eight powers per step in flight: the pass streams (m+1) n doubles,
        // so it is bound by how many loads are outstanding; each row still
        // sums its powers in ascending k
        Ssq acc{0.0, 0.0};
        for (int64_t row = lo + tid; row < hi; row += NT) {
            const double *b = basis + row;
            double y = 0.0;
            int k = 0;
            for (; k + 8 <= m + 1; k += 8) {
                double bk[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    bk[j] = b[(int64_t)(k + j) * n];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    y = fma(coef[k + j], bk[j], y);
            }
            for (; k <= m; ++k)
                y = fma(coef[k], b[(int64_t)k * n], y);
            ssq_add(acc, y);
        }
        const Ssq tot = exchange(acc);
        return (tot.scale == 0.0) ? 0.0 : exp(ssq_log(tot) / (double)m);
    };

    // ---- Brent's minimiser without derivatives (Brent 1973, ch. 5):
    //      golden-section steps accelerated by parabolic interpolation.
    const double gsr = 0.3819660112501051;   // (3 - sqrt 5)/2
    double blo = -P.zmax, bhi = P.zmax;
    double x = blo + gsr * (bhi - blo), w = x, v = x;
    double fx = objective(x);
    double fw = fx, fv = fx, step = 0.0, prev = 0.0;
    int evals = 1;
    for (int it = 0; it < P.brent_maxit && alive; ++it) {
        const double mid = 0.5 * (blo + bhi);
        const double tol1 = P.brent_rel * fabs(x) + P.brent_abs;
        if (fabs(x - mid) <= 2.0 * tol1 - 0.5 * (bhi - blo))
            break;
        bool golden = true;
        if (fabs(prev) > tol1) {
            const double r1 = (x - w) * (fx - fv);
            double q = (x - v) * (fx - fw);
            double pp = (x - v) * q - (x - w) * r1;
            q = 2.0 * (q - r1);
            if (q > 0.0)
                pp = -pp;
            else
                q = -q;
            const double older = prev;
            prev = step;
            if (fabs(pp) < fabs(0.5 * q * older) && pp > q * (blo - x) && pp < q * (bhi - x)) {
                step = pp / q;
                const double u = x + step;
                if (u - blo < 2.0 * tol1 || bhi - u < 2.0 * tol1)
                    step = (x < mid) ? tol1 : -tol1;
                golden = false;
            }
        }
        if (golden) {
            prev = (x < mid) ? bhi - x : blo - x;
            step = gsr * prev;
        }
        const double u = (fabs(step) >= tol1) ? x + step : x + (step > 0.0 ? tol1 : -tol1);
        const double fu = objective(u);
        ++evals;
        if (fu <= fx) {
            if (u < x)
                bhi = x;
            else
                blo = x;
            v = w; fv = fw;
            w = x; fw = fx;
            x = u; fx = fu;
        } else {
            if (u < x)
                blo = u;
            else
                bhi = u;
            if (fu <= fw || w == x) {
                v = w; fv = fw;
                w = u; fw = fu;
            } else if (fu <= fv || v == x || v == w) {
                v = u; fv = fu;
            }
        }
    }
    if (!alive) {
        finish(PHICOMB_EDEVICE, r, s0, 0, 0, 0, 0, 0);
        return;
    }
    // s = s0 f* / (tol m!)^(1/m) is formed on the host
    finish(PHICOMB_OK, r, s0, x, fx, -x * s0, 0.0, evals);
}

// Sixteen waves a workgroup (at most 128 registers a lane) keep enough loads
// of the objective's pass in flight with one workgroup per compute unit; the
// register-cached CSR variant holds its rows instead and runs eight.
template <int KIND>
__global__ __launch_bounds__(kPNTWide) void params_kernel(ParamsArgs P) {
    params_body<KIND, kPNTWide>(P);
}

__global__ __launch_bounds__(kPNT) void params_kernel_cached(ParamsArgs P) {
    params_body<kCsrCached, kPNT>(P);
}

int params_nt(int kind) { return kind == kCsrCached ? kPNT : kPNTWide; }

// ------------------------------------------------------------------ host
namespace {
double binom_double(int m, int k) {
    // exact integer in 128 bits, then one correctly rounded conversion
    unsigned __int128 b = 1;
    if (k > m - k)
        k = m - k;
    for (int j = 1; j <= k; ++j)
        b = b * (unsigned __int128)(m - k + j) / (unsigned __int128)j;
    return (double)b;
}

const void *params_fn(int kind) {
    switch (kind) {
    case kStencil: return (const void *)params_kernel<kStencil>;
    case kDense: return (const void *)params_kernel<kDense>;
    case kLowRank: return (const void *)params_kernel<kLowRank>;
    case kCsrCached: return (const void *)params_kernel_cached;
    default: return (const void *)params_kernel<kCsr>;
    }
}

int max_params_grid(int kind, int device) {
    static std::mutex mu;
    static int cached[5][64] = {};
    std::lock_guard<std::mutex> g(mu);
    int &c = cached[kind == kStencil    ? 0
                    : kind == kDense    ? 2
                    : kind == kLowRank  ? 3
                    : kind == kCsrCached ? 4
                                         : 1][device & 63];
    if (c > 0)
        return c;
    const void *fn = params_fn(kind);
    int per_cu = 0;
    hipDeviceProp_t prop;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, params_nt(kind), 0) != hipSuccess ||
        hipGetDeviceProperties(&prop, device) != hipSuccess || per_cu < 1)
        return 0;
    // one workgroup per CU: the barrier cost grows with the number of workgroups
    c = std::min(prop.multiProcessorCount, kPMaxGrid);
    return c;
}
}  // namespace

// Brent settings of the parameter search (tolerances in z = -xi/s0).
constexpr double kBrentRel = 1.4901161193847656e-08;
constexpr double kBrentAbs = 1e-6;
constexpr int kBrentMaxIt = 100;

size_t params_workspace_bytes(int64_t n, int m) {
    return (size_t)kSyncBytes + sizeof(double) * (4 * kPMaxGrid + 32 + 128) +
           sizeof(double) * (size_t)n * (size_t)(m + 1) +
           sizeof(double) * 4 * kLrRankMax * kPMaxGrid;
}

int params_fp64(phicomb_op op, double tol, int m, const double *v, uint64_t seed,
                hipStream_t stream, phicomb_params_t *out) {
    const int64_t n = op->dev.n;
    std::memset(out, 0, sizeof(*out));
    out->m = m;
    out->tol = tol;
    int st = ensure_workspace(op, params_workspace_bytes(n, m));
    if (st != PHICOMB_OK)
        return st;
    char *base = (char *)op->ws.ptr;
    ParamsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.op = op->dev;
    a.n = n;
    a.m = m;
    a.have_v = v ? 1 : 0;
    a.seed = seed;
    a.tol = tol;
    a.gmax = 0.8 * std::log(DBL_MAX);
    a.gmin = 0.8 * std::log(DBL_MIN);
    double lmax = -INFINITY;
    for (int j = 0; j <= m; ++j)
        lmax = std::max(lmax, std::lgamma(m + 1.0) - std::lgamma(j + 1.0) - std::lgamma(m - j + 1.0));
    a.lmax = lmax;
    a.zmax = std::sqrt((double)n);
    a.brent_rel = kBrentRel;
    a.brent_abs = kBrentAbs;
    a.brent_maxit = kBrentMaxIt;
    a.bar = (unsigned *)base;
    a.part = (double *)(base + kSyncBytes);
    a.out = a.part + 4 * kPMaxGrid;
    double *bin_dev = a.part + 4 * kPMaxGrid + 16;
    a.binom = bin_dev;
    a.basis = (double *)(base + kSyncBytes + sizeof(double) * (4 * kPMaxGrid + 32 + 128));
    a.lrpart = a.basis + (size_t)n * (size_t)(m + 1);
    double bin_host[PHICOMB_MAX_M + 1];
    for (int k = 0; k <= m; ++k)
        bin_host[k] = binom_double(m, k);
    if (hipMemcpyAsync(bin_dev, bin_host, sizeof(double) * (m + 1), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
        return PHICOMB_EDEVICE;
    if (v && hipMemcpyAsync(a.basis, v, sizeof(double) * n, hipMemcpyHostToDevice, stream) !=
                 hipSuccess)
        return PHICOMB_EDEVICE;
    const int maxg = max_params_grid(op->dev.kind, op->device);
    if (maxg < 1)
        return PHICOMB_EDEVICE;
    // dense rows are spread thinly, 8 a workgroup (one a wave for half its
    // waves), so that more CUs read A: at n = 2048 the whole chip, 13 % faster
    // than 16 a workgroup
    const int64_t rows_per_wg = (op->dev.kind == kDense) ? 8 : params_nt(op->dev.kind);
    const int64_t G = std::min<int64_t>(maxg, (n + rows_per_wg - 1) / rows_per_wg);
    const int held = round_xcd(G);   // at most ceil(G/8) of the grid lands on any XCD
    // short CSR rows and a chunk of at most kParamRows rows per thread: rows
    // held in registers (the grid has the same size either way)
    int kind = op->dev.kind;
    if (kind == kCsr && op->dev.max_row_nnz <= kCacheNnz &&
        (n + G - 1) / G <= (int64_t)kParamRows * kPNT && max_params_grid(kCsrCached, op->device) >= G)
        kind = kCsrCached;
    const void *fn = params_fn(kind);
    if (cu_acquire(op->device, held, held) != held)
        return PHICOMB_EDEVICE;
    struct Hold {
        int dev, g;
        ~Hold() { cu_release(dev, g); }
    } hold{op->device, held};
    params_sync_init<<<1, 256, 0, stream>>>(a.bar, a.out);
    void *args[] = {&a};
    if (launch_persistent(fn, (unsigned)G, params_nt(kind), args, stream) != hipSuccess)
        return PHICOMB_EDEVICE;
    if (hipMemcpyAsync(op->pinned, a.out, 8 * sizeof(double), hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return PHICOMB_EDEVICE;
    const double *o = op->pinned;
    const int status = (int)o[0];
    out->r_acc = (int)o[1];
    out->s0 = o[2];
    out->zstar = o[3];
    out->fstar = o[4];
    out->shift = o[5];
    out->s = o[6];
    if (status == PHICOMB_OK && out->r_acc > 0)
        out->s = out->s0 * out->fstar / std::exp((std::log(tol) + std::lgamma(m + 1.0)) / (double)m);
    out->n_feval = (int)o[7];
    out->status = status;
    return status;
}

}  // namespace phc
