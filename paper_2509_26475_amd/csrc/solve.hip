// Single-solve launch of Algorithm 3 (Al-Mohy, Sec. 4; r = 1 is Algorithm 2)
// and its host side: arguments, variant choice, workspace layout, statistics.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <utility>

#include "solve_body.h"

namespace phc {

__global__ void solve_sync_init(unsigned *bar, int *info) {
    for (int i = threadIdx.x; i < kSyncLines * kLineU; i += blockDim.x)
        bar[i] = 0u;
    if (threadIdx.x < 8)
        info[threadIdx.x] = 0;
}

static KernelFn pick_kernel(int kind, int r, int rpt, bool emem, bool mix) {
    if (kind == kLowRank)
        return pick_lowrank(r, rpt, emem, mix);
    if (kind == kStencil)
        return pick_r<kStencil>(r, rpt, emem, mix);
    if (kind == kCsr)
        return pick_r<kCsr>(r, rpt, emem, mix);
    if (kind == kCsrCached && !emem)
        return pick_r<kCsrCached>(r, rpt, false, mix);
    return nullptr;
}

static int max_coresident(KernelFn fn, int device) {
    static std::mutex m;
    static std::vector<std::pair<std::pair<void *, int>, int>> cache;
    std::lock_guard<std::mutex> g(m);
    for (auto &e : cache)
        if (e.first.first == (void *)fn && e.first.second == device)
            return e.second;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, kNT, 0) !=
        hipSuccess)
        return 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return 0;
    const int total = std::min(per_cu * prop.multiProcessorCount, kMaxGrid);
    cache.push_back({{(void *)fn, device}, total});
    return total;
}

static size_t sync_bytes() { return (size_t)kSyncBytes + sizeof(double) * 4 * kMaxGrid + 256; }
size_t solve_sync_bytes() { return sync_bytes(); }

// Entries of W^T X exchanged per term for a low-rank operator: the S-series
// passes carry the term block and S_0, the recovery passes the 2r columns of F.
static int64_t lr_values(int p, int r, int rank) {
    return (int64_t)rank * std::max<int64_t>((int64_t)(p + 1) * r + r, 2LL * r);
}

size_t solve_workspace_bytes(int64_t n, int p, int r, int precision, int rank) {
    const int64_t cS = (int64_t)(p + 1) * r, cR = 2LL * r, cW = std::max(cS, cR);
    const size_t f32 = (precision == PHICOMB_MIXED) ? (size_t)4 * n * 2 * cR + 256 : 0;
    const size_t lr = (rank > 0) ? (size_t)8 * 2 * lr_values(p, r, rank) * kMaxGrid + 256 : 0;
    return sync_bytes() + (size_t)8 * (size_t)n * (size_t)(cS + 2 * cW + cR) + f32 + lr;
}

// Algorithmic bytes of one solve (FP64): every Taylor term reads and writes
// its term block and its partial-sum block; the S-series terms also read V;
// the operator is read once per product (CSR arrays, the dense matrix, or U
// and W of a low-rank operator; stencil weights are in registers).
// Mixed precision: an FP32 term reads and writes its term block in 4-byte
// words (8 n c bytes fewer per term).
static double algorithmic_bytes(const DevOp &op, int64_t nnz, int64_t n, int p, int r,
                                int terms_S, int terms_rec, int s_int, int f32_rec) {
    const double w = 8.0, N = (double)n;
    const double cS = (double)(p + 1) * r, cR = 2.0 * r;
    const double opb = (op.kind == kCsr)       ? (12.0 * (double)nnz + 4.0 * (N + 1))
                       : (op.kind == kDense)   ? 8.0 * N * N
                       : (op.kind == kLowRank) ? 16.0 * N * op.rank
                                               : 0.0;
    double b = w * N * (p + 1) + 2 * w * N * cS;                        // V -> S, D
    b += (terms_S - 1) * (4 * w * N * cS + w * N * (p + 1) + opb);     // S-series terms
    b += 3 * w * N * r + opb;                                           // recover exp(tA/s) v0
    b += terms_rec * (4 * w * N * cR + opb);                            // recovery terms
    b += (s_int - 1) * (w * N * p * r + 2 * w * N * cR);                // step epilogues
    b += 3 * w * N * r;                                                 // combine
    b -= 8.0 * N * f32_rec * cR;                                         // FP32 term blocks
    return b;
}

// Variant choice within a budget of `cap` workgroups (at most one per CU:
// the barrier cost grows with the number of workgroups): the fewest rows per
// thread of {1, 2, 4, 8} that covers n with E in registers and no register
// spills; a shape with no mixed kernel takes the FP64 one; otherwise E moves
// to memory and rows are grid-strided.  Some instantiations carry a small
// private frame with no scratch traffic in their code (up to kFrameOk
// bytes); spilling ones have hundreds.
constexpr size_t kFrameOk = 64;
template <int R>
static KernelFn dense_kernel() { return solve_kernel<kDense, R, 1, true, false>; }

// Dense operators: at most kDenseRows rows per workgroup (one workgroup up to
// n = kDenseRows), else 32 rows per workgroup so that the k range of every
// row tile is split over the waves; FP64 only.
static int64_t dense_grid(int64_t n) { return n <= kDenseRows ? 1 : (n + 31) / 32; }

static KernelFn select_variant(phicomb_op op, int r, bool mix, int64_t wgs_needed1, int cap,
                               int64_t *G) {
    if (op->dev.kind == kDense) {
        KernelFn f = nullptr;
        switch (r) {
        case 1: f = dense_kernel<1>(); break;
        case 2: f = dense_kernel<2>(); break;
        case 3: f = dense_kernel<3>(); break;
        case 4: f = dense_kernel<4>(); break;
        default: return nullptr;
        }
        const int maxg = std::min(max_coresident(f, op->device), cap);
        if (maxg < 1)
            return nullptr;
        // the grid keeps at most kDenseRows rows per workgroup
        const int64_t need = dense_grid(op->dev.n);
        const int64_t gmin = (op->dev.n + kDenseRows - 1) / kDenseRows;
        if (gmin > maxg)
            return nullptr;
        *G = std::min<int64_t>(need, maxg);
        return f;
    }
    const int kind = (op->dev.kind == kCsr && op->dev.max_row_nnz <= kCacheNnz) ? kCsrCached
                                                                                  : op->dev.kind;
    for (int pass = 0; pass < (mix ? 2 : 1); ++pass) {
        const bool m = mix && pass == 0;
        for (int rpt : {1, 2, 4, 8}) {
            KernelFn f = pick_kernel(kind, r, rpt, false, m);
            if (!f)
                continue;
            hipFuncAttributes fa;
            if (hipFuncGetAttributes(&fa, (const void *)f) != hipSuccess ||
                fa.localSizeBytes > kFrameOk)
                continue;
            const int maxg = std::min(max_coresident(f, op->device), cap);
            const int64_t g = (wgs_needed1 + rpt - 1) / rpt;
            if (maxg >= 1 && g <= maxg) {
                *G = g;
                return f;
            }
        }
    }
    KernelFn f = pick_kernel(op->dev.kind, r, 1, true, mix);
    if (!f)
        return nullptr;
    const int maxg = std::min(max_coresident(f, op->device), cap);
    if (maxg < 1)
        return nullptr;
    *G = std::min<int64_t>(maxg, wgs_needed1);
    return f;
}

int build_solve_args(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                     const double *beta, const void *V, double tol, int precision, void *W,
                     void *ws, size_t ws_bytes, SolveArgs &a) {
    const bool mix = (precision == PHICOMB_MIXED);
    const int64_t n = op->dev.n;
    const int P1 = p + 1;
    std::memset(&a, 0, sizeof(a));
    a.op = op->dev;
    a.n = n;
    a.p = p;
    a.r = r;
    a.P1 = P1;
    a.cS = P1 * r;
    a.cR = 2 * r;
    a.kcap = kTermCap;
    if (const char *cap = getenv("PHICOMB_TERM_CAP"))   // failure-path tests only
        a.kcap = std::max(2, std::min(kTermCap, atoi(cap)));
    a.tol = tol;
    a.xi = prm->shift;
    double tmax = 0.0;
    for (int i = 0; i < r; ++i)
        tmax = std::max(tmax, std::fabs(t[i]));
    const double sc = std::ceil(prm->s * tmax);
    if (!(sc <= 2147483647.0))
        return PHICOMB_EINVAL;
    const int s_int = sc < 1.0 ? 1 : (int)sc;
    a.s_int = s_int;
    const double sd = (double)s_int;
    a.nu = 1.0 / sd;
    for (int i = 0; i < r; ++i) {
        a.t[i] = t[i];
        a.ts[i] = t[i] / sd;
        a.mu[i] = std::exp(prm->shift * t[i] / sd);
        a.a[i] = (-prm->shift * t[i]) / sd;
        a.w0[i] = beta[i * P1 + 0];
        for (int b = 0; b < P1; ++b) {
            const int pb = (b == 0) ? 0 : p + 1 - b;
            a.gam[i][b] = beta[i * P1 + pb] * (a.mu[i] / sd);
        }
    }
    const int64_t cW = std::max<int64_t>(a.cS, a.cR);
    char *base = (char *)ws;
    a.bar = (unsigned *)base;
    a.part = (double *)(base + kSyncBytes);
    a.info = (int *)(base + kSyncBytes + sizeof(double) * 4 * kMaxGrid);
    double *d = (double *)(base + sync_bytes());
    a.S = d;
    d += (size_t)n * a.cS;
    a.U0 = d;
    d += (size_t)n * cW;
    a.U1 = d;
    d += (size_t)n * cW;
    a.E = d;
    d += (size_t)n * a.cR;
    if (mix) {
        float *f = (float *)(((uintptr_t)d + 255) & ~(uintptr_t)255);
        a.Uf0 = f;
        a.Uf1 = f + (size_t)n * a.cR;
        d = (double *)(a.Uf1 + (size_t)n * a.cR);
    }
    const int rank = (op->dev.kind == kLowRank) ? op->dev.rank : 0;
    if (rank > 0) {
        const int64_t lv = lr_values(p, r, rank);
        if (lv > kLrVals)
            return PHICOMB_EINVAL;
        a.lrv = (int)lv;
        a.lrpart = (double *)(((uintptr_t)d + 255) & ~(uintptr_t)255);
    }
    a.mix_tau = tol / (10.0 * 5.9604644775390625e-08);   // u_fp32 = 2^-24
    // FP32 terms stay clear of overflow ((A - xi I) x with |x| <= partial sum)
    // and of the subnormal range.
    a.mix_lo = 1e-20;
    a.mix_hi = 1e30 / std::max(1.0, op->norm_inf + std::fabs(prm->shift));
    a.V = (const double *)V;
    a.W = (double *)W;
    if (solve_workspace_bytes(n, p, r, precision, rank) > ws_bytes)
        return PHICOMB_EINVAL;

    return PHICOMB_OK;
}

int solve_launch_held(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                      const double *beta, const void *V, double tol, int precision, void *W,
                      hipStream_t stream, void *ws, size_t ws_bytes, int slots,
                      const int **info_dev, int *s_int) {
    SolveArgs a;
    const int st = build_solve_args(op, prm, p, r, t, beta, V, tol, precision, W, ws, ws_bytes, a);
    if (st != PHICOMB_OK)
        return st;
    const int64_t wgs_needed1 = (op->dev.n + kNT - 1) / kNT;
    int64_t G = 0;
    KernelFn fn = select_variant(op, r, precision == PHICOMB_MIXED, wgs_needed1, slots, &G);
    if (!fn)
        return PHICOMB_EINVAL;
    solve_sync_init<<<1, 256, 0, stream>>>(a.bar, a.info);
    void *args[] = {&a};
    if (launch_persistent((const void *)fn, (unsigned)G, kNT, args, stream) != hipSuccess)
        return PHICOMB_EDEVICE;
    *info_dev = a.info;
    *s_int = a.s_int;
    return PHICOMB_OK;
}

double solve_algorithmic_bytes(phicomb_op op, int p, int r, int s_int, const int *info) {
    return algorithmic_bytes(op->dev, op->nnz, op->dev.n, p, r, info[1], info[2], s_int, info[4]);
}

int solve_run(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
              const double *beta, const void *V, double tol, int precision, void *W,
              hipStream_t stream, phicomb_stats_t *stats, void *ws, size_t ws_bytes,
              double *pinned, int cu_floor) {
    const bool mix = (precision == PHICOMB_MIXED);
    const int64_t n = op->dev.n;
    SolveArgs a;
    {
        const int st = build_solve_args(op, prm, p, r, t, beta, V, tol, precision, W, ws,
                                        ws_bytes, a);
        if (st != PHICOMB_OK)
            return st;
    }
    const int s_int = a.s_int;
    const int64_t wgs_needed1 = (n + kNT - 1) / kNT;
    const int cus = device_cus(op->device);
    // Persistent launches on one device draw workgroup slots from a shared
    // ledger so that concurrent solves never exceed co-residency together.
    const bool dense = (op->dev.kind == kDense);
    const int want = (int)std::min<int64_t>(cus, dense ? dense_grid(n) : wgs_needed1);
    int floor_g = (cu_floor > 0) ? std::min(want, cu_floor) : want;
    if (dense)   // at most kDenseRows rows per workgroup
        floor_g = std::max<int>(floor_g, (int)std::min<int64_t>(want, (n + kDenseRows - 1) / kDenseRows));
    const int granted = cu_acquire(op->device, want, floor_g);
    if (granted < 1)
        return PHICOMB_EDEVICE;
    int64_t G = 0;
    KernelFn fn = select_variant(op, r, mix, wgs_needed1, granted, &G);
    if (!fn) {
        cu_release(op->device, granted);
        return PHICOMB_EINVAL;
    }
    // keep round_xcd(G) slots: at most ceil(G/8) of the grid lands on any XCD
    const int held = std::min(granted, round_xcd(G));
    if (held < granted)
        cu_release(op->device, granted - held);
    struct Hold {
        int dev, g;
        ~Hold() { cu_release(dev, g); }
    } hold{op->device, held};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool timed = (hipEventCreate(&e0) == hipSuccess) && (hipEventCreate(&e1) == hipSuccess);
    solve_sync_init<<<1, 256, 0, stream>>>(a.bar, a.info);
    if (timed)
        hipEventRecord(e0, stream);
    void *args[] = {&a};
    hipError_t le = launch_persistent((const void *)fn, (unsigned)G, kNT, args, stream);
    if (le != hipSuccess) {
        if (timed) {
            hipEventDestroy(e0);
            hipEventDestroy(e1);
        }
        return PHICOMB_EDEVICE;
    }
    if (timed)
        hipEventRecord(e1, stream);
    hipMemcpyAsync(pinned, a.info, 8 * sizeof(int), hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess)
        return PHICOMB_EDEVICE;
    const int *info = (const int *)pinned;
    const int st = info[0];
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->s_int = s_int;
        stats->terms_S = info[1];
        stats->terms_rec = info[2];
        stats->max_terms_step = info[3];
        stats->fp32_terms = info[4];
        stats->status = st;
        stats->bytes_alg = algorithmic_bytes(op->dev, op->nnz, n, p, r, info[1], info[2], s_int,
                                             info[4]);
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

}  // namespace phc
