// Parameter selection (Al-Mohy, Sec. 3, Algorithm 1) on the device, FP64.
//
//   V_0 = v/||v||_2;  W_k = A V_{k-1}, L_k = log||W_k||_2, accepted while
//   L_k + log(k+1)/2 + max_j log binom(m,j) <= 0.8 log(realmax) and
//   L_k >= 0.8 log(realmin);  s0 = exp(mean of the last (<= 5) log-growth
//   ratios, excluding the newest);  V_j <- s0^-j V_j;  V_k = A V_{k-1}/s0 up
//   to degree m;  f(xi) = ||V (b .* [z^m .. z 1])||_2^(1/m) with z = -xi/s0,
//   minimised by Brent's method over z in [-sqrt(n), sqrt(n)];
//   s = s0 f(xi*) / (tol m!)^(1/m).
//
// The basis lives on the device as [m+1][n] (column-major), each product and
// each objective evaluation is one fused pass that also forms a deterministic
// scaled sum of squares (per thread, per wave in a fixed shuffle tree, per
// workgroup, then over workgroups in index order), so repeated runs give
// identical parameters.  The host keeps only the scalar logic: the guard,
// s0, and Brent's iteration.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace phc {

constexpr int kNormBlocks = 1024;

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
        // combine in a lane-independent order so both partners agree
        const bool lower = (threadIdx.x & off) == 0;
        v = lower ? ssq_merge(v, o) : ssq_merge(o, v);
    }
    return v;
}

__device__ __forceinline__ void block_ssq_store(Ssq v, double2 *part) {
    __shared__ double sc[kWaves], sq[kWaves];
    v = wave_ssq(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sc[wave] = v.scale;
        sq[wave] = v.ssq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Ssq acc{sc[0], sq[0]};
        for (int w = 1; w < kWaves; ++w)
            acc = ssq_merge(acc, Ssq{sc[w], sq[w]});
        part[blockIdx.x] = make_double2(acc.scale, acc.ssq);
    }
}

// Combine the per-workgroup partials in index order; out = {log||x||, ||x||}.
__global__ void ssq_final(const double2 *part, int nparts, double *out) {
    __shared__ double sc[kWG], sq[kWG];
    const int t = threadIdx.x;
    Ssq acc{0.0, 0.0};
    for (int b = t; b < nparts; b += kWG)   // fixed assignment, fixed order
        acc = ssq_merge(acc, Ssq{part[b].x, part[b].y});
    sc[t] = acc.scale;
    sq[t] = acc.ssq;
    __syncthreads();
    if (t == 0) {
        Ssq tot{0.0, 0.0};
        for (int w = 0; w < kWG; ++w)
            tot = ssq_merge(tot, Ssq{sc[w], sq[w]});
        if (tot.scale == 0.0) {
            out[0] = -INFINITY;
            out[1] = 0.0;
        } else {
            out[0] = log(tot.scale) + 0.5 * log(tot.ssq);
            out[1] = tot.scale * sqrt(tot.ssq);
        }
    }
}

// y = (A x) * scale  and its partial 2-norm.
template <int KIND>
__global__ __launch_bounds__(kWG) void spmv_norm(DevOp A, const double *__restrict__ x,
                                                 double *__restrict__ y, double scale,
                                                 double2 *part) {
    const int64_t n = A.n;
    Ssq acc{0.0, 0.0};
    for (int64_t row = (int64_t)blockIdx.x * kWG + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * kWG) {
        const RowCtx rc = row_ctx<KIND>(A, row);
        double v[1];
        apply_cols<KIND, 1>(A, rc, x, n, 0, 0.0, v);
        const double w = (scale == 1.0) ? v[0] : v[0] / scale;
        y[row] = w;
        ssq_add(acc, w);
    }
    block_ssq_store(acc, part);
}

// x <- x * f   or  x <- x / d (only one of the two is used)
__global__ void scale_vec(double *x, int64_t n, double f, double d) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        x[i] = (d != 0.0) ? x[i] / d : x[i] * f;
}

__global__ void norm_only(const double *__restrict__ x, int64_t n, double2 *part) {
    Ssq acc{0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        ssq_add(acc, x[i]);
    block_ssq_store(acc, part);
}

// SplitMix64 (Steele, Lea & Flood, 2014) of (seed, i), mapped to [-1, 1).
__global__ void fill_splitmix(double *x, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

// y_i = sum_k c_k V_k[i] (ascending k) and its partial 2-norm.
struct Coef {
    double c[PHICOMB_MAX_M + 1];
};

__global__ __launch_bounds__(kWG) void objective_norm(const double *__restrict__ basis,
                                                      int64_t n, int m, Coef cf, double2 *part) {
    Ssq acc{0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
        double y = 0.0;
        for (int k = 0; k <= m; ++k)
            y += cf.c[k] * basis[(int64_t)k * n + i];
        ssq_add(acc, y);
    }
    block_ssq_store(acc, part);
}

// ------------------------------------------------------------------ host
namespace {

struct Ctx {
    phicomb_op op;
    hipStream_t st;
    double2 *part;
    double *res;      // device [2]
    double *pinned;   // host [2]
    int nb;
};

int readback(Ctx &c, double *lognorm, double *norm) {
    ssq_final<<<1, kWG, 0, c.st>>>(c.part, c.nb, c.res);
    if (hipMemcpyAsync(c.pinned, c.res, 2 * sizeof(double), hipMemcpyDeviceToHost, c.st) !=
        hipSuccess)
        return PHICOMB_EDEVICE;
    if (hipStreamSynchronize(c.st) != hipSuccess)
        return PHICOMB_EDEVICE;
    if (lognorm)
        *lognorm = c.pinned[0];
    if (norm)
        *norm = c.pinned[1];
    return PHICOMB_OK;
}

void launch_spmv(Ctx &c, const double *x, double *y, double scale) {
    const DevOp &A = c.op->dev;
    if (A.kind == kStencil)
        spmv_norm<kStencil><<<c.nb, kWG, 0, c.st>>>(A, x, y, scale, c.part);
    else
        spmv_norm<kCsr><<<c.nb, kWG, 0, c.st>>>(A, x, y, scale, c.part);
}

double binom_double(int m, int k) {
    // exact integer in 128 bits, then one correctly rounded conversion
    unsigned __int128 b = 1;
    if (k > m - k)
        k = m - k;
    for (int j = 1; j <= k; ++j)
        b = b * (unsigned __int128)(m - k + j) / (unsigned __int128)j;
    return (double)b;
}

// Brent's minimiser without derivatives (Brent 1973, ch. 5): golden-section
// search accelerated by parabolic interpolation through the best three
// points.  Returns false if an evaluation failed.
template <class F>
bool brent_minimise(F &&f, double lo, double hi, double rel, double abs_tol, int max_iter,
                    double *xmin, double *fmin, int *nfev) {
    const double gs = 0.3819660112501051;   // (3 - sqrt 5)/2
    double x = lo + gs * (hi - lo), w = x, v = x;
    double fx;
    if (!f(x, &fx))
        return false;
    double fw = fx, fv = fx, step = 0.0, prev = 0.0;
    int evals = 1;
    for (int it = 0; it < max_iter; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double tol1 = rel * std::fabs(x) + abs_tol;
        if (std::fabs(x - mid) <= 2.0 * tol1 - 0.5 * (hi - lo))
            break;
        bool golden = true;
        if (std::fabs(prev) > tol1) {
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
            if (std::fabs(pp) < std::fabs(0.5 * q * older) && pp > q * (lo - x) &&
                pp < q * (hi - x)) {
                step = pp / q;
                const double u = x + step;
                if (u - lo < 2.0 * tol1 || hi - u < 2.0 * tol1)
                    step = (x < mid) ? tol1 : -tol1;
                golden = false;
            }
        }
        if (golden) {
            prev = (x < mid) ? hi - x : lo - x;
            step = gs * prev;
        }
        const double u = (std::fabs(step) >= tol1) ? x + step : x + (step > 0.0 ? tol1 : -tol1);
        double fu;
        if (!f(u, &fu))
            return false;
        ++evals;
        if (fu <= fx) {
            (u < x ? hi : lo) = x;
            v = w;
            fv = fw;
            w = x;
            fw = fx;
            x = u;
            fx = fu;
        } else {
            (u < x ? lo : hi) = u;
            if (fu <= fw || w == x) {
                v = w;
                fv = fw;
                w = u;
                fw = fu;
            } else if (fu <= fv || v == x || v == w) {
                v = u;
                fv = fu;
            }
        }
    }
    *xmin = x;
    *fmin = fx;
    *nfev = evals;
    return true;
}

}  // namespace

// Brent settings of the parameter search (tolerances in z = -xi/s0).
constexpr double kBrentRel = 1.4901161193847656e-08;
constexpr double kBrentAbs = 1e-6;
constexpr int kBrentMaxIt = 100;

int params_fp64(phicomb_op op, double tol, int m, const double *v, uint64_t seed,
                hipStream_t stream, phicomb_params_t *out) {
    const int64_t n = op->dev.n;
    std::memset(out, 0, sizeof(*out));
    out->m = m;
    out->tol = tol;
    double *basis = nullptr;
    double2 *part = nullptr;
    double *res = nullptr;
    if (hipMalloc(&basis, sizeof(double) * (size_t)n * (m + 1)) != hipSuccess)
        return PHICOMB_ENOMEM;
    if (hipMalloc(&part, sizeof(double2) * kNormBlocks) != hipSuccess ||
        hipMalloc(&res, 4 * sizeof(double)) != hipSuccess) {
        hipFree(basis);
        hipFree(part);
        return PHICOMB_ENOMEM;
    }
    int nb = (int)std::min<int64_t>(kNormBlocks, (n + kWG - 1) / kWG);
    Ctx c{op, stream, part, res, op->pinned, nb};
    int status = PHICOMB_OK;
    auto cleanup = [&]() {
        hipStreamSynchronize(stream);
        hipFree(basis);
        hipFree(part);
        hipFree(res);
    };
    // V_0 = v / ||v||
    if (v) {
        if (hipMemcpyAsync(basis, v, sizeof(double) * n, hipMemcpyHostToDevice, stream) !=
            hipSuccess) {
            cleanup();
            return PHICOMB_EDEVICE;
        }
    } else {
        fill_splitmix<<<nb, kWG, 0, stream>>>(basis, n, seed);
    }
    norm_only<<<nb, kWG, 0, stream>>>(basis, n, part);
    double lv = 0.0, nv = 0.0;
    if ((status = readback(c, &lv, &nv)) != PHICOMB_OK) {
        cleanup();
        return status;
    }
    if (!(nv > 0.0) || !std::isfinite(nv)) {
        cleanup();
        return PHICOMB_EINVAL;
    }
    scale_vec<<<nb, kWG, 0, stream>>>(basis, n, 1.0, nv);

    const double gmax = 0.8 * std::log(DBL_MAX);
    const double gmin = 0.8 * std::log(DBL_MIN);
    double lmax = -INFINITY;
    for (int j = 0; j <= m; ++j)
        lmax = std::max(lmax, std::lgamma(m + 1.0) - std::lgamma(j + 1.0) - std::lgamma(m - j + 1.0));
    std::vector<double> L(m + 2, 0.0);
    int r = 0;
    for (int k = 1; k <= m; ++k) {
        launch_spmv(c, basis + (size_t)(k - 1) * n, basis + (size_t)k * n, 1.0);
        double lk = 0.0;
        if ((status = readback(c, &lk, nullptr)) != PHICOMB_OK) {
            cleanup();
            return status;
        }
        L[k] = lk;
        if (std::isnan(lk)) {
            cleanup();
            return PHICOMB_EINVAL;
        }
        if (lk + 0.5 * std::log(k + 1.0) + lmax > gmax || lk < gmin)
            break;
        r = k;
    }
    out->r_acc = r;
    if (r == 0) {
        cleanup();
        if (L[1] < gmin) {   // A v vanishes: treat A as zero
            out->shift = 0.0;
            out->s = 1.0;
            out->status = PHICOMB_OK;
            return PHICOMB_OK;
        }
        return PHICOMB_EOVERFLOW;
    }
    double s0;
    if (r >= 3) {
        const int jr = std::max(2, r - 5);
        double sum = 0.0;
        for (int j = jr; j <= r - 1; ++j)
            sum += L[j + 1] - L[j];
        s0 = std::exp(sum / (double)(r - jr));
    } else {
        s0 = std::exp(L[r] / (double)r);
    }
    out->s0 = s0;
    const double ls0 = std::log(s0);
    for (int j = 1; j <= r; ++j)
        scale_vec<<<nb, kWG, 0, stream>>>(basis + (size_t)j * n, n, std::exp(-(double)j * ls0), 0.0);
    for (int k = r + 1; k <= m; ++k)
        launch_spmv(c, basis + (size_t)(k - 1) * n, basis + (size_t)k * n, s0);

    std::vector<double> bino(m + 1);
    for (int k = 0; k <= m; ++k)
        bino[k] = binom_double(m, k);
    auto f = [&](double z, double *fz) -> bool {
        Coef cf;
        double pw = 1.0;
        for (int k = m; k >= 0; --k) {
            cf.c[k] = bino[k] * pw;
            pw = pw * z;
        }
        objective_norm<<<nb, kWG, 0, stream>>>(basis, n, m, cf, part);
        double ln = 0.0, nr = 0.0;
        if (readback(c, &ln, &nr) != PHICOMB_OK)
            return false;
        *fz = (nr == 0.0) ? 0.0 : std::exp(ln / (double)m);
        return true;
    };
    const double zmax = std::sqrt((double)n);
    double zs = 0.0, fz = 0.0;
    int nfev = 0;
    if (!brent_minimise(f, -zmax, zmax, kBrentRel, kBrentAbs, kBrentMaxIt, &zs, &fz, &nfev)) {
        cleanup();
        return PHICOMB_EDEVICE;
    }
    out->zstar = zs;
    out->shift = -zs * s0;
    out->fstar = fz;
    out->n_feval = nfev;
    out->s = s0 * fz / std::exp((std::log(tol) + std::lgamma(m + 1.0)) / (double)m);
    out->status = PHICOMB_OK;
    cleanup();
    return PHICOMB_OK;
}

}  // namespace phc
