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
        return pick_stencil(r, rpt, emem, mix);
    if (kind == kCsr)
        return pick_csr(r, rpt, emem, mix);
    if (kind == kCsrCached && !emem)
        return pick_csr_cached(r, rpt, mix);
    return nullptr;
}

// Co-resident workgroups of a kernel on a device (occupancy x CUs), cached in
// a fixed table (no allocation after the first query of a kernel).
static int max_coresident(KernelFn fn, int device, int nt = kNT) {
    struct Entry {
        void *fn;
        int device, total;
    };
    constexpr int kCache = 512;
    static std::mutex m;
    static Entry cache[kCache];
    static int used = 0;
    std::lock_guard<std::mutex> g(m);
    for (int i = 0; i < used; ++i)
        if (cache[i].fn == (void *)fn && cache[i].device == device)
            return cache[i].total;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, nt, 0) !=
        hipSuccess)
        return 0;
    const int total = std::min(per_cu * device_cus(device), kMaxGrid);
    if (used < kCache)
        cache[used++] = Entry{(void *)fn, device, total};
    return total;
}

static size_t sync_bytes() { return (size_t)kSyncBytes + sizeof(double) * 2 * kRedMax * kMaxGrid + 256; }
size_t solve_sync_bytes() { return sync_bytes(); }

// Entries of W^T X exchanged per term for a low-rank operator: the S-series
// passes carry the term block and S_0, the recovery passes the 2r columns of F.
static int64_t lr_values(int p, int r, int rank) {
    return (int64_t)rank * std::max<int64_t>((int64_t)(p + 1) * r + r, 2LL * r);
}

size_t solve_workspace_bytes(int64_t n, int p, int r, int precision, int rank) {
    const int64_t cS = (int64_t)(p + 1) * r, cR = 2LL * r, cW = std::max(cS, cR);
    const size_t f32 = (precision == PHICOMB_MIXED) ? (size_t)4 * n * 2 * cW + 256 : 0;
    const size_t lr = (rank > 0) ? (size_t)8 * 4 * lr_values(p, r, rank) * kMaxGrid + 256 : 0;
    return sync_bytes() + (size_t)8 * (size_t)n * (size_t)(cS + 2 * cW + cR) + f32 + lr;
}

// Algorithmic bytes of one solve (FP64): every Taylor term reads and writes
// its term block and its partial-sum block; the S-series terms also read V;
// the operator is read once per product (CSR arrays, the dense matrix, or U
// and W of a low-rank operator; stencil weights are in registers).
// Mixed precision: an FP32 term reads and writes its term block in 4-byte
// words (8 n c bytes fewer per term).
static double algorithmic_bytes(const DevOp &op, int64_t nnz, int64_t n, int p, int r,
                                int terms_S, int terms_rec, int s_int, int f32_rec,
                                int f32_S) {
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
    b -= 8.0 * N * (f32_rec * cR + f32_S * cS);                          // FP32 term blocks
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

// Dense operators: at most kDenseRows rows per workgroup (one workgroup up to
// n = kDenseRows), else one 16-row tile per workgroup, so that the k range
// of the tile is split over all eight waves and as many CUs as the grid
// allows read A; FP64 only.
static int64_t dense_grid(int64_t n) { return n <= kDenseRows ? 1 : (n + 15) / 16; }

void solve_grid_request(phicomb_op op, int *want, int *floor_g) {
    const int64_t n = op->dev.n;
    const int cus = device_cus(op->device);
    if (op->dev.kind == kDense) {
        *want = (int)std::min<int64_t>(cus, dense_grid(n));
        // at most kDenseRows rows per workgroup
        *floor_g = (int)std::min<int64_t>(*want, (n + kDenseRows - 1) / kDenseRows);
    } else {
        *want = (int)std::min<int64_t>(cus, (n + kNT - 1) / kNT);
        *floor_g = 1;
    }
}

// Dynamic LDS a workgroup may hold on this device (0 if unknown).
static int max_lds_per_block(int device) {
    static std::mutex m;
    static int cache[64] = {};
    std::lock_guard<std::mutex> g(m);
    int &c = cache[device & 63];
    if (c == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
                hipSuccess ||
            v < 0)
            v = 0;
        c = v + 1;   // 0 means not yet queried
    }
    return c - 1;
}

static KernelFn select_variant(phicomb_op op, int r, bool mix, int64_t wgs_needed1, int cap,
                               int64_t *G, int *nt, size_t *lds, int p) {
    *nt = kNT;
    *lds = 0;
    if (op->dev.kind == kDense) {
        if (!mix && cap >= 1 && op->dev.n <= kDenseLdsN) {
            // everything in LDS on one workgroup when it fits
            KernelFn f = pick_dense_lds(r);
            hipFuncAttributes fa;
            const size_t dyn = dense_lds_bytes(op->dev.n, (int64_t)(p + 1) * r, 2LL * r);
            if (f && hipFuncGetAttributes(&fa, (const void *)f) == hipSuccess &&
                fa.localSizeBytes <= kFrameOk &&
                fa.sharedSizeBytes + dyn <= (size_t)max_lds_per_block(op->device) &&
                hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)dyn) == hipSuccess) {
                *G = 1;
                *lds = dyn;
                return f;
            }
        }
        KernelFn f = pick_dense(r);
        if (!f)
            return nullptr;
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
    // E in memory.  Stencils with an even grid line: the 1024-thread kernel
    // (16 waves per CU keep twice the loads in flight of the 512-thread one)
    if (op->dev.kind == kStencil && op->dev.nx % 2 == 0) {
        for (int pass = 0; pass < (mix ? 2 : 1); ++pass) {
            KernelFn f = pick_stencil_wide(r, mix && pass == 0);
            hipFuncAttributes fa;
            if (!f || hipFuncGetAttributes(&fa, (const void *)f) != hipSuccess ||
                fa.localSizeBytes > kFrameOk)
                continue;
            const int maxg = std::min(max_coresident(f, op->device, kWideNT), cap);
            if (maxg < 1)
                continue;
            *G = std::min<int64_t>(maxg, (op->dev.n + kWideNT - 1) / kWideNT);
            *nt = kWideNT;
            return f;
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
    a.info = (int *)(base + kSyncBytes + sizeof(double) * 2 * kRedMax * kMaxGrid);
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
        a.Uf1 = f + (size_t)n * cW;
        d = (double *)(a.Uf1 + (size_t)n * cW);
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
    int nt = kNT;
    size_t lds = 0;
    KernelFn fn =
        select_variant(op, r, precision == PHICOMB_MIXED, wgs_needed1, slots, &G, &nt, &lds, p);
    if (!fn)
        return PHICOMB_EINVAL;
    solve_sync_init<<<1, 256, 0, stream>>>(a.bar, a.info);
    void *args[] = {&a};
    if (launch_persistent((const void *)fn, (unsigned)G, nt, args, stream, lds) != hipSuccess)
        return PHICOMB_EDEVICE;
    *info_dev = a.info;
    *s_int = a.s_int;
    return PHICOMB_OK;
}

double solve_algorithmic_bytes(phicomb_op op, int p, int r, int s_int, const int *info) {
    return algorithmic_bytes(op->dev, op->nnz, op->dev.n, p, r, info[1], info[2], s_int, info[4],
                             info[5]);
}

int solve_run(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
              const double *beta, const void *V, double tol, int precision, void *W,
              hipStream_t stream, phicomb_stats_t *stats, void *ws, size_t ws_bytes,
              double *pinned, int cu_floor, hipEvent_t *events) {
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
    // Persistent launches on one device draw workgroup slots from a shared
    // ledger so that concurrent solves never exceed co-residency together.
    int want = 0, need_g = 0;
    solve_grid_request(op, &want, &need_g);
    const int floor_g = std::max((cu_floor > 0) ? std::min(want, cu_floor) : want, need_g);
    const int granted = cu_acquire(op->device, want, floor_g);
    if (granted < 1)
        return PHICOMB_EDEVICE;
    int64_t G = 0;
    int nt = kNT;
    size_t lds = 0;
    KernelFn fn = select_variant(op, r, mix, wgs_needed1, granted, &G, &nt, &lds, p);
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
    const bool own_events = (events == nullptr);
    bool timed;
    if (own_events) {
        timed = (hipEventCreate(&e0) == hipSuccess) && (hipEventCreate(&e1) == hipSuccess);
    } else {
        e0 = events[0];
        e1 = events[1];
        timed = true;
    }
    auto drop_events = [&]() {
        if (own_events) {
            if (e0)
                hipEventDestroy(e0);
            if (e1)
                hipEventDestroy(e1);
        }
    };
    solve_sync_init<<<1, 256, 0, stream>>>(a.bar, a.info);
    if (timed)
        hipEventRecord(e0, stream);
    void *args[] = {&a};
    hipError_t le = launch_persistent((const void *)fn, (unsigned)G, nt, args, stream, lds);
    if (le != hipSuccess) {
        drop_events();
        return PHICOMB_EDEVICE;
    }
    if (timed)
        hipEventRecord(e1, stream);
    hipMemcpyAsync(pinned, a.info, 8 * sizeof(int), hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess) {
        drop_events();
        return PHICOMB_EDEVICE;
    }
    const int *info = (const int *)pinned;
    const int st = info[0];
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->s_int = s_int;
        stats->terms_S = info[1];
        stats->terms_rec = info[2];
        stats->max_terms_step = info[3];
        stats->fp32_terms = info[4] + info[5];
        stats->status = st;
        stats->bytes_alg = algorithmic_bytes(op->dev, op->nnz, n, p, r, info[1], info[2], s_int,
                                             info[4], info[5]);
        float ms = 0.0f;
        if (timed && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            stats->ms = ms;
    }
    drop_events();
    return st;
}

// ------------------------------------------------ solve without allocation
// The work blocks of phicomb_solve_static live in this file-scope device
// array (one copy per device the library runs on, kept until the process
// ends).  In host code its name is only a stand-in for the device symbol:
// the device address comes from hipGetSymbolAddress, taken once per device
// at the first call with that device current, and only that address is
// ever passed to kernels or copies.  The same first call creates the two
// timing events of the device.  Calls on one device share the array; they
// are serialised here (a call returns when its result is written), so
// calls that would overlap on one device wait for each other.
constexpr size_t kScratchBytes = (size_t)PHICOMB_STATIC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct StaticSlot {
    std::mutex mu;          // serialises the calls on this device
    bool ready = false;
    void *ptr = nullptr;    // device address of this device's scratch
    hipEvent_t ev[2] = {nullptr, nullptr};
};
StaticSlot g_static[kMaxDevices];
}  // namespace

}  // namespace phc

extern "C" int phicomb_solve_static(phicomb_op op, const phicomb_params_t *prm, int p, int r,
                                    const double *t, const double *beta, const void *V,
                                    double tol, int precision, void *W, void *stream,
                                    phicomb_stats_t *stats) {
    using namespace phc;
    if (solve_check_args(op, prm, p, r, t, beta, V, tol, precision, W) != PHICOMB_OK)
        return PHICOMB_EINVAL;
    const size_t need = solve_workspace_bytes(op->dev.n, p, r, precision, op_lr_rank(op));
    if (need > kScratchBytes)
        return PHICOMB_EINVAL;   // the work blocks exceed the static array
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return PHICOMB_EDEVICE;
    if (dev != op->device)
        return PHICOMB_EINVAL;   // the operator lives on another device
    StaticSlot &sl = g_static[dev];
    std::lock_guard<std::mutex> g(sl.mu);
    if (!sl.ready) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return PHICOMB_EDEVICE;
        if (hipEventCreate(&sl.ev[0]) != hipSuccess || hipEventCreate(&sl.ev[1]) != hipSuccess)
            return PHICOMB_EDEVICE;
        sl.ptr = ptr;
        sl.ready = true;
    }
    std::lock_guard<std::mutex> go(op->mu);
    const int st = solve_run(op, prm, p, r, t, beta, V, tol, precision, W, (hipStream_t)stream,
                             stats, sl.ptr, kScratchBytes, op->pinned, 0, sl.ev);
    if (stats)
        stats->status = st;
    return st;
}

namespace phc {

}  // namespace phc
