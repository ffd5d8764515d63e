// Time stepping of u' = A u + g(u) with the fourth-order six-stage exponential
// Runge-Kutta scheme expRK4s6 (Al-Mohy, Sec. 1, eq. (expRK4s6)), every
// phi-combination evaluated by Algorithm 3 with one set of Algorithm 1
// parameters reused for all calls (Sec. 5, fourth experiment).
//
// The stages that the scheme allows to be formed together are one block call
// each, four calls per step:
//   U2              t = c2 h          V = [0, h f]
//   U3, U4          t = (c3, c4) h    V = [0, h f, h D2]
//   U5, U6          t = (c5, c6) h    V = [0, h f, h q2(D3, D4), h q3(D3, D4)]
//   u_{n+1}         t = h             V = [0, h f, h q2(D5, D6), h q3(D5, D6)]
// with f = A u_n + g(u_n), D_i = g(U_i) - g(u_n) and the weight tables the
// scheme's phi_1, phi_2, phi_3 coefficients.  Between the calls, one pointwise
// kernel per stage forms U_i = u_n + w_i, the increments D_i and the next
// input block, so nothing leaves the device.
//
// The host does not wait for each call: the workgroup slots for the solves
// are taken from the ledger once for the whole integration, every solve is
// launched without a host synchronisation, and a one-thread kernel after it
// folds the call's status and term counts into a device accumulator.  The
// update u <- u + w of a step is skipped once any call has failed, so u keeps
// the last completed step; the host reads the accumulator every kCheckEvery
// steps and at the end, and stops at the first failure it sees.
#include <cmath>
#include <cstring>

#include "solve_body.h"

namespace phc {

constexpr int kENT = 256;

struct Cubic {
    double c0, c1, c2, c3;
};

__device__ __forceinline__ double cubic(const Cubic &g, double u) {
    return g.c0 + u * (g.c1 + u * (g.c2 + u * g.c3));
}

// gu = g(u), hf = h (A u + g(u)), V = [0, hf] (row-major n x 2).
template <int KIND>
__global__ __launch_bounds__(kENT) void exprk_rhs(DevOp A, Cubic g, double h,
                                                  const double *__restrict__ u,
                                                  double *__restrict__ gu,
                                                  double *__restrict__ hf,
                                                  double *__restrict__ V) {
    const int64_t row = (int64_t)blockIdx.x * kENT + threadIdx.x;
    if (row >= A.n)
        return;
    const RowCtx rc = row_ctx<KIND>(A, row);
    double y[1];
    apply_cols<KIND, 1>(A, rc, u, A.n, 0, 0.0, y);
    const double g0 = cubic(g, u[row]);
    const double f = h * (y[0] + g0);
    gu[row] = g0;
    hf[row] = f;
    V[row * 2 + 0] = 0.0;
    V[row * 2 + 1] = f;
}

// D2 = g(u + w) - g(u); V = [0, hf, h D2] (n x 3).
__global__ __launch_bounds__(kENT) void exprk_stage2(int64_t n, Cubic g, double h,
                                                     const double *__restrict__ u,
                                                     const double *__restrict__ gu,
                                                     const double *__restrict__ hf,
                                                     const double *__restrict__ W,
                                                     double *__restrict__ V) {
    const int64_t row = (int64_t)blockIdx.x * kENT + threadIdx.x;
    if (row >= n)
        return;
    const double d2 = cubic(g, u[row] + W[row]) - gu[row];
    V[row * 3 + 0] = 0.0;
    V[row * 3 + 1] = hf[row];
    V[row * 3 + 2] = h * d2;
}

// Two stages U_a = u + W[:,0], U_b = u + W[:,1]; D_a, D_b; the next block
// V = [0, hf, h (ka D_a + kb D_b), h (la D_a + lb D_b)] (n x 4).
__global__ __launch_bounds__(kENT) void exprk_stage_pair(int64_t n, Cubic g, double h, double ka,
                                                         double kb, double la, double lb,
                                                         const double *__restrict__ u,
                                                         const double *__restrict__ gu,
                                                         const double *__restrict__ hf,
                                                         const double *__restrict__ W,
                                                         double *__restrict__ V) {
    const int64_t row = (int64_t)blockIdx.x * kENT + threadIdx.x;
    if (row >= n)
        return;
    const double ur = u[row], g0 = gu[row];
    const double da = cubic(g, ur + W[row * 2 + 0]) - g0;
    const double db = cubic(g, ur + W[row * 2 + 1]) - g0;
    V[row * 4 + 0] = 0.0;
    V[row * 4 + 1] = hf[row];
    V[row * 4 + 2] = h * (ka * da + kb * db);
    V[row * 4 + 3] = h * (la * da + lb * db);
}

// u <- u + w, unless a call of the integration has failed.
__global__ __launch_bounds__(kENT) void exprk_update(int64_t n, double *__restrict__ u,
                                                     const double *__restrict__ W,
                                                     const long long *__restrict__ acc) {
    const int64_t row = (int64_t)blockIdx.x * kENT + threadIdx.x;
    if (row < n && acc[0] == 0)
        u[row] = u[row] + W[row];
}

// acc: first non-zero status, Taylor terms, FP32 terms, calls, steps completed.
__global__ void exprk_acc_init(long long *acc) {
    if (threadIdx.x < 8)
        acc[threadIdx.x] = 0;
}

__global__ void exprk_fold(const int *__restrict__ info, long long *acc) {
    if (threadIdx.x == 0) {
        if (acc[0] == 0 && info[0] != 0)
            acc[0] = info[0];
        acc[1] += (long long)info[1] + info[2];
        acc[2] += info[4] + info[5];
        acc[3] += 1;
    }
}

__global__ void exprk_step_done(long long *acc) {
    if (threadIdx.x == 0 && acc[0] == 0)
        acc[4] += 1;
}

constexpr int kCheckEvery = 64;   // steps between host reads of the accumulator

}  // namespace phc

using namespace phc;

extern "C" int phicomb_exprk4s6(phicomb_op op, const phicomb_params_t *prm, const double g[4],
                                double h, int nsteps, double tol, int precision, void *u,
                                void *stream_, phicomb_exprk_stats_t *stats) {
    if (stats)
        std::memset(stats, 0, sizeof(*stats));
    if (!op || !prm || !g || !u || nsteps < 0 || !(h > 0.0) || !std::isfinite(h))
        return PHICOMB_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol) || prm->status != PHICOMB_OK ||
        !std::isfinite(prm->shift) || !std::isfinite(prm->s) || prm->s < 0.0)
        return PHICOMB_EINVAL;
    if (precision != PHICOMB_FP64 && precision != PHICOMB_MIXED)
        return PHICOMB_EINVAL;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(g[k]))
            return PHICOMB_EINVAL;
    // the right-hand side reads the operator row by row: stencil, or the CSR
    // form (which dense operators also keep); a low-rank operator has neither
    const int kind = op->dev.kind;
    if (kind == kLowRank)
        return PHICOMB_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t n = op->dev.n;
    const Cubic gc{g[0], g[1], g[2], g[3]};
    // nodes of the scheme
    const double c2 = 0.5, c3 = 0.5, c4 = 1.0 / 3.0, c5 = 5.0 / 6.0, c6 = 1.0 / 3.0;

    std::lock_guard<std::mutex> lk(op->mu);
    const int rank = op_lr_rank(op);
    size_t need = 0;
    for (int p = 1; p <= 3; ++p)
        for (int r = 1; r <= 2; ++r)
            need = std::max(need, solve_workspace_bytes(n, p, r, precision, rank));
    int st = ensure_workspace(op, need);
    if (st != PHICOMB_OK)
        return st;
    // gu, hf: n each; V: n x 4; W: n x 2; the accumulator
    const size_t aux_bytes = sizeof(double) * ((size_t)n * 8 + 8);
    if (op->aux.bytes < aux_bytes) {
        if (op->aux.ptr)
            hipFree(op->aux.ptr);
        op->aux.ptr = nullptr;
        op->aux.bytes = 0;
        if (hipMalloc(&op->aux.ptr, aux_bytes) != hipSuccess)
            return PHICOMB_ENOMEM;
        op->aux.bytes = aux_bytes;
    }
    double *gu = (double *)op->aux.ptr;
    double *hf = gu + n;
    double *V = hf + n;
    double *W = V + 4 * n;
    long long *accd = (long long *)(W + 2 * n);
    double *ud = (double *)u;
    const unsigned grid = (unsigned)((n + kENT - 1) / kENT);

    // workgroup slots for every solve of the integration, held until the end
    int want = 0, need_g = 0;
    solve_grid_request(op, &want, &need_g);
    const int slots = cu_acquire(op->device, want, want);
    if (slots < 1)
        return PHICOMB_EDEVICE;
    struct Hold {
        int dev, g;
        hipStream_t s;
        ~Hold() {
            hipStreamSynchronize(s);   // every solve has completed before the slots return
            cu_release(dev, g);
        }
    } hold{op->device, slots, stream};

    phicomb_exprk_stats_t acc;
    std::memset(&acc, 0, sizeof(acc));
    auto call = [&](int p, int r, const double *t, const double *beta) -> int {
        const int *info = nullptr;
        int s_int = 0;
        const int rc = solve_launch_held(op, prm, p, r, t, beta, V, tol, precision, W, stream,
                                         op->ws.ptr, op->ws.bytes, slots, &info, &s_int);
        if (rc != PHICOMB_OK)
            return rc;
        exprk_fold<<<1, 64, 0, stream>>>(info, accd);
        acc.max_s_int = std::max(acc.max_s_int, s_int);
        return PHICOMB_OK;
    };
    // device accumulator -> acc; its status
    auto check = [&]() -> int {
        if (hipMemcpyAsync(op->pinned, accd, 8 * sizeof(long long), hipMemcpyDeviceToHost,
                           stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return PHICOMB_EDEVICE;
        const long long *h = (const long long *)op->pinned;
        acc.terms = h[1];
        acc.fp32_terms = h[2];
        acc.calls = (int)h[3];
        acc.steps = (int)h[4];
        return (int)h[0];
    };
    const double t2[1] = {c2 * h};
    const double b2[2] = {0.0, c2};
    const double t34[2] = {c3 * h, c4 * h};
    const double b34[6] = {0.0, c3, c3 * c3 / c2, 0.0, c4, c4 * c4 / c2};
    const double t56[2] = {c5 * h, c6 * h};
    const double b56[8] = {0.0, c5, c5 * c5 / (c3 - c4), 2.0 * c5 * c5 * c5 / (c3 - c4),
                           0.0, c6, c6 * c6 / (c3 - c4), 2.0 * c6 * c6 * c6 / (c3 - c4)};
    const double t1[1] = {h};
    const double b1[4] = {0.0, 1.0, 1.0 / (c5 - c6), 2.0 / (c5 - c6)};

    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    exprk_acc_init<<<1, 64, 0, stream>>>(accd);
    if (timed)
        hipEventRecord(e0, stream);
    st = PHICOMB_OK;
    for (int step = 0; step < nsteps && st == PHICOMB_OK; ++step) {
        if (kind == kStencil)
            exprk_rhs<kStencil><<<grid, kENT, 0, stream>>>(op->dev, gc, h, ud, gu, hf, V);
        else
            exprk_rhs<kCsr><<<grid, kENT, 0, stream>>>(op->dev, gc, h, ud, gu, hf, V);
        if ((st = call(1, 1, t2, b2)) != PHICOMB_OK)
            break;
        exprk_stage2<<<grid, kENT, 0, stream>>>(n, gc, h, ud, gu, hf, W, V);
        if ((st = call(2, 2, t34, b34)) != PHICOMB_OK)
            break;
        exprk_stage_pair<<<grid, kENT, 0, stream>>>(n, gc, h, -c4 / c3, c3 / c4, 1.0 / c3,
                                                    -1.0 / c4, ud, gu, hf, W, V);
        if ((st = call(3, 2, t56, b56)) != PHICOMB_OK)
            break;
        exprk_stage_pair<<<grid, kENT, 0, stream>>>(n, gc, h, -c6 / c5, c5 / c6, 1.0 / c5,
                                                    -1.0 / c6, ud, gu, hf, W, V);
        if ((st = call(3, 1, t1, b1)) != PHICOMB_OK)
            break;
        exprk_update<<<grid, kENT, 0, stream>>>(n, ud, W, accd);
        exprk_step_done<<<1, 64, 0, stream>>>(accd);
        if ((step + 1) % kCheckEvery == 0)
            st = check();
    }
    if (timed)
        hipEventRecord(e1, stream);
    // the accumulator holds the first failing call's status, if any
    const int dev_st = check();
    if (st == PHICOMB_OK)
        st = dev_st;
    if (timed) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            acc.ms = ms;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
    }
    acc.status = st;
    if (stats)
        *stats = acc;
    return st;
}
