// The single block series of the Proposition in Sec. 4 (Al-Mohy) with
// g_i = phi_i: column k of
//     G = sum_j A^j V D_j Gamma T^j,   D_j = diag(1/(i+j)!),  i = 0..p,
// is w_k = sum_i beta_ki phi_i(t_k A) v_i (Gamma generalised to any weight
// table).  No shift and no scaling: one Taylor series whose products act on
// the p+1 input columns only, whatever the number r of abscissae, so it is
// the cheap evaluation when |t| ||A|| is small; for large |t| ||A|| it needs
// many terms and loses accuracy to cancellation, and Algorithm 3 is the
// method to use.
//
// With tau = max_k |t_k| the device carries P_j = (tau A)^j V / j! (the p+1
// columns, column-major ping-pong) and adds to output column k the term
//     sum_i beta_ki (t_k/tau)^j  j!/(i+j)!  P_j[:, i],
// one persistent launch, one grid exchange per term (the block norms of the
// new term and of G for the stopping rule (stopTm) of Algorithm 3).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "solve_body.h"

namespace phc {

struct SeriesArgs {
    DevOp op;
    int64_t n;
    int p, r, P1, kcap;
    double tol, tau;
    double rho[kRMax];                  // t_k / tau
    double beta[kRMax][kPMax1];
    const double *V;                    // [n][p+1] row-major (caller)
    double *W;                          // [n][r] row-major (caller)
    double *X0, *X1;                    // [p+1][n] ping-pong
    unsigned *bar;
    double *part;                       // [2][kMaxGrid][2]
    double *lrpart;                     // low rank: [2][hi, lo][rank (p+1)][kMaxGrid] partial W^T P_j
    int *info;                          // status, terms
};

__global__ void series_sync_init(unsigned *bar, int *info) {
    for (int i = threadIdx.x; i < kSyncLines * kLineU; i += blockDim.x)
        bar[i] = 0u;
    if (threadIdx.x < 8)
        info[threadIdx.x] = 0;
}

template <int KIND, int R>
__global__ __launch_bounds__(kNT) void series_kernel(SeriesArgs P) {
    __shared__ double red[kNT / 64][kRedMax];
    __shared__ double wk[kRMax][kPMax1];   // this term's weight of P_j[:, i] in column k
    __shared__ double rpow[kRMax];         // (t_k / tau)^j
    __shared__ double lrc[kLrVals];        // low rank: W^T P_j of the coming product
    __shared__ int ok;
    const unsigned G = gridDim.x, bid = blockIdx.x;
    const int lb = xcd_logical_block(bid, G);
    const int64_t n = P.n;
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = std::min<int64_t>(n, (int64_t)lb * chunk);
    const int64_t hi = std::min<int64_t>(n, lo + chunk);
    const int tid = threadIdx.x, P1 = P.P1;
    const DevOp &A = P.op;
    auto finish = [&](int st, int terms) {
        if (bid == 0 && tid == 0) {
            P.info[0] = st;
            P.info[1] = terms;
        }
    };
    GridSync gs;
    const bool single = (G == 1);
    if (!single && !grid_setup(gs, P.bar, &ok, G)) {
        finish(PHICOMB_EDEVICE, 0);
        return;
    }
    unsigned epoch = 0;
    // low rank (A = U W^T): the pass that writes P_j also leaves this
    // workgroup's partial W^T P_j, summed by every workgroup after the exchange
    const int nlr = (KIND == kLowRank) ? A.rank * P1 : 0;
    const size_t lr_lo = (size_t)nlr * kMaxGrid;
    auto lr_part = [&]() { return P.lrpart + (size_t)(epoch & 1) * 2 * lr_lo; };
    auto exchange = [&](double (&v)[2], const double *Xw) -> bool {
        if constexpr (KIND == kLowRank)
            lr_publish(A, n, lo, hi, Xw, P1, 0, lr_part(), lr_lo, single ? 0u : bid);
        if (single) {
            wait_own_stores();
            workgroup_max<2, kNT>(v, red);
            if constexpr (KIND == kLowRank)
                lr_gather(lr_part(), lr_lo, 1, nlr, lrc);
            ++epoch;
            return true;
        }
        double *pt = P.part + (size_t)(epoch & 1) * kRedMax * kMaxGrid;
        store_partials<2, kNT>(v, pt, red, bid);
        if (!grid_sync(gs, &ok))
            return false;
        load_partials<2, kNT>(pt, G, v, red);
        if constexpr (KIND == kLowRank)
            lr_gather(lr_part(), lr_lo, G, nlr, lrc);
        ++epoch;
        return true;
    };

    // ---- j = 0: P_0 = V, G = sum_i beta_ki v_i / i!
    if (tid < R * P1) {
        const int k = tid / P1, i = tid % P1;
        double f = 1.0;
        for (int l = 2; l <= i; ++l)
            f *= (double)l;
        wk[k][i] = P.beta[k][i] / f;
        if (i == 0)
            rpow[k] = 1.0;
    }
    __syncthreads();
    double nv[2] = {0.0, 0.0};
    for (int64_t row = lo + tid; row < hi; row += kNT) {
        double g[R];
#pragma unroll
        for (int k = 0; k < R; ++k)
            g[k] = 0.0;
        for (int i = 0; i < P1; ++i) {
            const double v = P.V[row * P1 + i];
            P.X0[(int64_t)i * n + row] = v;
#pragma unroll
            for (int k = 0; k < R; ++k)
                g[k] += wk[k][i] * v;
        }
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            P.W[row * R + k] = g[k];
            s += fabs(g[k]);
        }
        nv[0] = nmax(nv[0], s);
    }
    nv[1] = nv[0];
    if (!exchange(nv, P.X0)) {
        finish(PHICOMB_EDEVICE, 1);
        return;
    }
    double c1 = INFINITY, c2 = nv[0], nG = nv[1];
    int j = 0;
    int status = PHICOMB_OK;
    while (c1 + c2 > P.tol * nG && P.tau > 0.0) {
        if (j + 1 >= P.kcap) {
            status = PHICOMB_ENOCONV;
            break;
        }
        j = j + 1;
        c1 = c2;
        // weights of this term: beta_ki (t_k/tau)^j j!/(i+j)!
        __syncthreads();
        if (tid < R * P1) {
            const int k = tid / P1, i = tid % P1;
            double e = 1.0;
            for (int l = 1; l <= i; ++l)
                e /= (double)(j + l);
            wk[k][i] = P.beta[k][i] * (rpow[k] * P.rho[k]) * e;
        }
        __syncthreads();
        if (tid < R)
            rpow[tid] = rpow[tid] * P.rho[tid];
        const double *Xo = (j & 1) ? P.X0 : P.X1;
        double *Xn = (j & 1) ? P.X1 : P.X0;
        const double step = P.tau / (double)j;
        double mx[2] = {0.0, 0.0};
        for (int64_t row = lo + tid; row < hi; row += kNT) {
            RowCtx rc{};
            if constexpr (KIND != kLowRank)
                rc = row_ctx<KIND>(A, row);
            double tk[R];
#pragma unroll
            for (int k = 0; k < R; ++k)
                tk[k] = 0.0;
            for (int i = 0; i < P1; ++i) {
                double y[1];
                if constexpr (KIND == kLowRank) {
                    // U_row (W^T P_{j-1})[:, i]
                    const double *ur = A.lr_u + row * A.rank;
                    y[0] = 0.0;
                    for (int k = 0; k < A.rank; ++k)
                        y[0] += ur[k] * lrc[i * A.rank + k];
                } else {
                    apply_cols<KIND, 1>(A, rc, Xo, n, i, 0.0, y);
                }
                const double x = y[0] * step;
                Xn[(int64_t)i * n + row] = x;
#pragma unroll
                for (int k = 0; k < R; ++k)
                    tk[k] += wk[k][i] * x;
            }
            double st = 0.0, sg = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double gnew = P.W[row * R + k] + tk[k];
                P.W[row * R + k] = gnew;
                st += fabs(tk[k]);
                sg += fabs(gnew);
            }
            mx[0] = nmax(mx[0], st);
            mx[1] = nmax(mx[1], sg);
        }
        if (!exchange(mx, Xn)) {
            finish(PHICOMB_EDEVICE, j + 1);
            return;
        }
        c2 = mx[0];
        nG = mx[1];
    }
    if (!(c2 == c2) || !(nG == nG))
        status = PHICOMB_EDEVICE;
    finish(status, j + 1);
}

using SeriesFn = void (*)(SeriesArgs);

template <int KIND>
static SeriesFn series_r(int r) {
    switch (r) {
    case 1: return series_kernel<KIND, 1>;
    case 2: return series_kernel<KIND, 2>;
    case 3: return series_kernel<KIND, 3>;
    case 4: return series_kernel<KIND, 4>;
    default: return nullptr;
    }
}

}  // namespace phc

using namespace phc;

extern "C" int phicomb_solve_series(phicomb_op op, int p, int r, const double *t,
                                    const double *beta, const void *V, double tol, void *W,
                                    void *stream_, phicomb_stats_t *stats) {
    if (stats)
        std::memset(stats, 0, sizeof(*stats));
    if (!op || !t || !beta || !V || !W)
        return PHICOMB_EINVAL;
    if (p < 0 || p > PHICOMB_MAX_P || r < 1 || r > PHICOMB_MAX_R)
        return PHICOMB_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol))
        return PHICOMB_EINVAL;
    for (int k = 0; k < r; ++k)
        if (!std::isfinite(t[k]))
            return PHICOMB_EINVAL;
    for (int k = 0; k < r * (p + 1); ++k)
        if (!std::isfinite(beta[k]))
            return PHICOMB_EINVAL;
    const int kind = op->dev.kind;
    SeriesFn fn = (kind == kStencil)  ? series_r<kStencil>(r)
                  : (kind == kLowRank) ? series_r<kLowRank>(r)
                                       : series_r<kCsr>(r);
    if (!fn)
        return PHICOMB_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t n = op->dev.n;
    const int P1 = p + 1;

    std::lock_guard<std::mutex> lk(op->mu);
    const size_t sync = (size_t)kSyncBytes + sizeof(double) * 2 * kRedMax * kMaxGrid + 256;
    const int rank = op_lr_rank(op);
    const size_t lr = (rank > 0) ? sizeof(double) * 4 * (size_t)rank * P1 * kMaxGrid + 256 : 0;
    const size_t need = sync + sizeof(double) * 2 * (size_t)P1 * (size_t)n + lr;
    int st = ensure_workspace(op, need);
    if (st != PHICOMB_OK)
        return st;
    SeriesArgs a;
    std::memset(&a, 0, sizeof(a));
    a.op = op->dev;
    a.n = n;
    a.p = p;
    a.r = r;
    a.P1 = P1;
    a.kcap = kTermCap;
    a.tol = tol;
    double tau = 0.0;
    for (int k = 0; k < r; ++k)
        tau = std::max(tau, std::fabs(t[k]));
    a.tau = tau;
    for (int k = 0; k < r; ++k) {
        a.rho[k] = (tau > 0.0) ? t[k] / tau : 0.0;
        for (int i = 0; i < P1; ++i)
            a.beta[k][i] = beta[k * P1 + i];
    }
    char *base = (char *)op->ws.ptr;
    a.bar = (unsigned *)base;
    a.part = (double *)(base + kSyncBytes);
    a.info = (int *)(base + kSyncBytes + sizeof(double) * 2 * kRedMax * kMaxGrid);
    a.X0 = (double *)(base + sync);
    a.X1 = a.X0 + (size_t)P1 * n;
    if (rank > 0)
        a.lrpart = (double *)(((uintptr_t)(a.X1 + (size_t)P1 * n) + 255) & ~(uintptr_t)255);
    a.V = (const double *)V;
    a.W = (double *)W;

    // one workgroup per 512 rows up to one per CU, from the slot ledger
    const int cus = device_cus(op->device);
    const int want = (int)std::min<int64_t>(std::min<int64_t>(cus, kMaxGrid), (n + kNT - 1) / kNT);
    const int granted = cu_acquire(op->device, want, want);
    if (granted < 1)
        return PHICOMB_EDEVICE;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, kNT, 0) !=
            hipSuccess ||
        per_cu < 1) {
        cu_release(op->device, granted);
        return PHICOMB_EDEVICE;
    }
    const int G = granted;
    const int held = std::min(granted, round_xcd(G));
    if (held < granted)
        cu_release(op->device, granted - held);
    struct Hold {
        int dev, g;
        ~Hold() { cu_release(dev, g); }
    } hold{op->device, held};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    series_sync_init<<<1, 256, 0, stream>>>(a.bar, a.info);
    if (timed)
        hipEventRecord(e0, stream);
    void *args[] = {&a};
    if (launch_persistent((const void *)fn, (unsigned)G, kNT, args, stream) != hipSuccess) {
        if (timed) {
            hipEventDestroy(e0);
            hipEventDestroy(e1);
        }
        return PHICOMB_EDEVICE;
    }
    if (timed)
        hipEventRecord(e1, stream);
    hipMemcpyAsync(op->pinned, a.info, 8 * sizeof(int), hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess)
        return PHICOMB_EDEVICE;
    const int *info = (const int *)op->pinned;
    st = info[0];
    if (stats) {
        stats->s_int = 1;
        stats->terms_S = info[1];
        stats->status = st;
        // per term: the p+1 columns read and written, W read and written
        const double opb = (kind == kStencil)   ? 0.0
                           : (kind == kLowRank) ? 16.0 * n * rank / P1   // U and W once per term
                                                : 12.0 * (double)op->nnz + 4.0 * (n + 1);
        stats->bytes_alg = 8.0 * n * (P1 + 2.0 * P1 + r) +
                           (info[1] - 1) * (16.0 * n * P1 + 16.0 * n * r + P1 * opb);
        float ms = 0.0f;
        if (timed && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            stats->ms = ms;
    }
    if (timed) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
    }
    return st;
}
