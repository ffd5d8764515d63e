// C ABI of the phicomb library: operators, Algorithm 1, Algorithm 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <new>

#include "internal.h"

using namespace phc;

namespace {

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess)
        return -1;
    return d;
}

phicomb_op new_op() {
    phicomb_op op = new (std::nothrow) phicomb_op_s();
    if (!op)
        return nullptr;
    std::memset(&op->dev, 0, sizeof(op->dev));
    op->device = current_device();
    if (hipHostMalloc((void **)&op->pinned, 64 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        delete op;
        return nullptr;
    }
    return op;
}

void free_op(phicomb_op op) {
    if (!op)
        return;
    if (op->mem)
        hipFree(op->mem);
    if (op->dense_mem)
        hipFree(op->dense_mem);
    if (op->ws.ptr)
        hipFree(op->ws.ptr);
    if (op->aux.ptr)
        hipFree(op->aux.ptr);
    if (op->pinned)
        hipHostFree(op->pinned);
    delete op;
}

bool finite_array(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i]))
            return false;
    return true;
}

int upload_csr(phicomb_op op, int64_t n, const int32_t *rowptr, const int32_t *col,
               const double *val) {
    const int64_t nnz = rowptr[n];
    const size_t b_rp = sizeof(int32_t) * (size_t)(n + 1);
    const size_t b_ci = sizeof(int32_t) * (size_t)nnz;
    const size_t b_va = sizeof(double) * (size_t)nnz;
    const size_t off_va = 0, off_rp = (b_va + 255) & ~(size_t)255,
                 off_ci = off_rp + ((b_rp + 255) & ~(size_t)255);
    char *mem = nullptr;
    if (hipMalloc(&mem, off_ci + b_ci + 256) != hipSuccess)
        return PHICOMB_ENOMEM;
    if (hipMemcpy(mem + off_va, val, b_va, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mem + off_rp, rowptr, b_rp, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mem + off_ci, col, b_ci, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(mem);
        return PHICOMB_EDEVICE;
    }
    int maxrow = 0;
    double norm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        maxrow = std::max(maxrow, rowptr[i + 1] - rowptr[i]);
        double sr = 0.0;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            sr += std::fabs(val[q]);
        norm = std::max(norm, sr);
    }
    op->dev.max_row_nnz = maxrow;
    op->norm_inf = norm;
    op->mem = mem;
    op->nnz = nnz;
    op->dev.kind = kCsr;
    op->dev.n = n;
    op->dev.val = (const double *)(mem + off_va);
    op->dev.rowptr = (const int32_t *)(mem + off_rp);
    op->dev.col = (const int32_t *)(mem + off_ci);
    return PHICOMB_OK;
}

}  // namespace

namespace phc {
namespace {
struct Ledger {
    std::mutex mu;
    std::condition_variable cv;
    int total = -1, free = 0;
};
constexpr int kMaxDevices = 64;
Ledger g_ledger[kMaxDevices];

Ledger &ledger(int device) { return g_ledger[device & (kMaxDevices - 1)]; }
}  // namespace

int device_cus(int device) {
    static std::mutex mu;
    static int cache[kMaxDevices] = {};
    std::lock_guard<std::mutex> g(mu);
    int &c = cache[device & (kMaxDevices - 1)];
    if (c == 0) {
        hipDeviceProp_t prop;
        c = (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
                ? prop.multiProcessorCount
                : 1;
    }
    return c;
}

int cu_acquire(int device, int want, int min_grant) {
    const int total = device_cus(device) / kXcds * kXcds;
    if (total < kXcds)
        return 0;
    want = std::min(round_xcd(std::max(1, want)), total);
    min_grant = std::min(round_xcd(std::max(1, min_grant)), want);
    Ledger &l = ledger(device);
    std::unique_lock<std::mutex> g(l.mu);
    if (l.total < 0) {
        l.total = total;
        l.free = total;
    }
    l.cv.wait(g, [&]() { return l.free >= min_grant; });
    const int got = std::min(want, l.free / kXcds * kXcds);
    l.free -= got;
    return got;
}

void cu_release(int device, int n) {
    if (n <= 0)
        return;
    Ledger &l = ledger(device);
    {
        std::lock_guard<std::mutex> g(l.mu);
        l.free = std::min(l.total, l.free + n);
    }
    l.cv.notify_all();
}

int solve_check_args(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                     const double *beta, const void *V, double tol, int precision, void *W) {
    if (!op || !prm || !t || !beta || !V || !W)
        return PHICOMB_EINVAL;
    if (p < 0 || p > PHICOMB_MAX_P || r < 1 || r > PHICOMB_MAX_R)
        return PHICOMB_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol) || prm->status != PHICOMB_OK)
        return PHICOMB_EINVAL;
    if (!std::isfinite(prm->shift) || !std::isfinite(prm->s) || prm->s < 0.0)
        return PHICOMB_EINVAL;
    if (!finite_array(t, r) || !finite_array(beta, (int64_t)r * (p + 1)))
        return PHICOMB_EINVAL;
    if (precision != PHICOMB_FP64 && precision != PHICOMB_MIXED)
        return PHICOMB_EINVAL;
    return PHICOMB_OK;
}

int ensure_workspace(phicomb_op op, size_t bytes) {
    if (op->ws.bytes >= bytes)
        return PHICOMB_OK;
    if (op->ws.ptr) {
        hipDeviceSynchronize();
        hipFree(op->ws.ptr);
        op->ws.ptr = nullptr;
        op->ws.bytes = 0;
    }
    if (hipMalloc(&op->ws.ptr, bytes) != hipSuccess)
        return PHICOMB_ENOMEM;
    op->ws.bytes = bytes;
    return PHICOMB_OK;
}
}  // namespace phc

extern "C" {

int phicomb_op_create_csr(int64_t n, const int32_t *rowptr, const int32_t *col,
                          const double *val, phicomb_op *out) {
    if (!out || n < 1 || n > kMaxRows || !rowptr || !col || !val)
        return PHICOMB_EINVAL;
    *out = nullptr;
    if (rowptr[0] != 0)
        return PHICOMB_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return PHICOMB_EINVAL;
    const int64_t nnz = rowptr[n];
    for (int64_t q = 0; q < nnz; ++q)
        if (col[q] < 0 || col[q] >= n)
            return PHICOMB_EINVAL;
    if (!finite_array(val, nnz))
        return PHICOMB_EINVAL;
    if (current_device() < 0)
        return PHICOMB_EDEVICE;
    phicomb_op op = new_op();
    if (!op)
        return PHICOMB_ENOMEM;
    const int st = upload_csr(op, n, rowptr, col, val);
    if (st != PHICOMB_OK) {
        free_op(op);
        return st;
    }
    *out = op;
    return PHICOMB_OK;
}

int phicomb_op_create_stencil(int dim, const int32_t grid[3], const double coef[7],
                              double superdiag, phicomb_op *out) {
    if (!out || !grid || !coef || (dim != 2 && dim != 3))
        return PHICOMB_EINVAL;
    *out = nullptr;
    const int64_t nx = grid[0], ny = grid[1], nz = (dim == 3) ? grid[2] : 1;
    if (nx < 1 || ny < 1 || nz < 1)
        return PHICOMB_EINVAL;
    const int64_t n = nx * ny * nz;
    if (n > kMaxRows)
        return PHICOMB_EINVAL;
    if (!finite_array(coef, 7) || !std::isfinite(superdiag))
        return PHICOMB_EINVAL;
    if (current_device() < 0)
        return PHICOMB_EDEVICE;
    phicomb_op op = new_op();
    if (!op)
        return PHICOMB_ENOMEM;
    op->dev.kind = kStencil;
    op->dev.dim = dim;
    op->dev.nx = (int)nx;
    op->dev.ny = (int)ny;
    op->dev.nz = (int)nz;
    op->dev.n = n;
    for (int j = 0; j < 7; ++j)
        op->dev.c[j] = (dim == 2 && j >= 5) ? 0.0 : coef[j];
    op->dev.superdiag = superdiag;
    op->nnz = 0;
    double norm = std::fabs(superdiag);
    for (int j = 0; j < 7; ++j)
        norm += std::fabs(op->dev.c[j]);
    op->norm_inf = norm;
    *out = op;
    return PHICOMB_OK;
}

int phicomb_op_create_dense(int64_t n, const double *A, phicomb_op *out) {
    if (!out || n < 1 || !A || n > 46340)
        return PHICOMB_EINVAL;
    *out = nullptr;
    if (!finite_array(A, n * n))
        return PHICOMB_EINVAL;
    // Dense rows as CSR rows with every column present.
    std::vector<int32_t> rp(n + 1), ci((size_t)n * n);
    for (int64_t i = 0; i <= n; ++i)
        rp[i] = (int32_t)(i * n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            ci[(size_t)i * n + j] = (int32_t)j;
    if (current_device() < 0)
        return PHICOMB_EDEVICE;
    phicomb_op op = new_op();
    if (!op)
        return PHICOMB_ENOMEM;
    // the CSR form serves Algorithm 1; the solve reads the row-major copy
    int st = upload_csr(op, n, rp.data(), ci.data(), A);
    if (st == PHICOMB_OK) {
        const size_t bytes = sizeof(double) * (size_t)n * (size_t)n;
        if (hipMalloc(&op->dense_mem, bytes) != hipSuccess)
            st = PHICOMB_ENOMEM;
        else if (hipMemcpy(op->dense_mem, A, bytes, hipMemcpyHostToDevice) != hipSuccess)
            st = PHICOMB_EDEVICE;
    }
    if (st != PHICOMB_OK) {
        free_op(op);
        return st;
    }
    op->dev.dense = (const double *)op->dense_mem;
    op->dev.kind = kDense;
    *out = op;
    return PHICOMB_OK;
}

int phicomb_op_create_lowrank(int64_t n, int rank, const double *U, const double *W,
                              phicomb_op *out) {
    if (!out || n < 1 || n > kMaxRows || rank < 1 || rank > kLrRankMax || !U || !W)
        return PHICOMB_EINVAL;
    *out = nullptr;
    if (!finite_array(U, n * rank) || !finite_array(W, n * rank))
        return PHICOMB_EINVAL;
    if (current_device() < 0)
        return PHICOMB_EDEVICE;
    phicomb_op op = new_op();
    if (!op)
        return PHICOMB_ENOMEM;
    const size_t bytes = sizeof(double) * (size_t)n * (size_t)rank;
    const size_t off_w = (bytes + 255) & ~(size_t)255;
    char *mem = nullptr;
    if (hipMalloc(&mem, off_w + bytes) != hipSuccess) {
        free_op(op);
        return PHICOMB_ENOMEM;
    }
    op->mem = mem;
    if (hipMemcpy(mem, U, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mem + off_w, W, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        free_op(op);
        return PHICOMB_EDEVICE;
    }
    // ||U W^T||_inf <= max_i sum_k |U_ik| ||W e_k||_1 (an upper bound is all
    // that the FP32 range guard needs; the exact row sums cost O(n^2 rank))
    std::vector<double> w1(rank, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < rank; ++k)
            w1[k] += std::fabs(W[i * rank + k]);
    double norm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double sr = 0.0;
        for (int k = 0; k < rank; ++k)
            sr += std::fabs(U[i * rank + k]) * w1[k];
        norm = std::max(norm, sr);
    }
    op->norm_inf = norm;
    op->nnz = 2 * n * rank;
    op->dev.kind = kLowRank;
    op->dev.n = n;
    op->dev.rank = rank;
    op->dev.lr_u = (const double *)mem;
    op->dev.lr_w = (const double *)(mem + off_w);
    *out = op;
    return PHICOMB_OK;
}

int phicomb_op_destroy(phicomb_op op) {
    if (!op)
        return PHICOMB_EINVAL;
    free_op(op);
    return PHICOMB_OK;
}

int64_t phicomb_op_n(phicomb_op op) { return op ? op->dev.n : -1; }

int phicomb_params(phicomb_op op, double tol, int m, const double *v, uint64_t seed,
                   void *stream, phicomb_params_t *out) {
    if (!op || !out || !(tol > 0.0) || !std::isfinite(tol) || m < 1 || m > PHICOMB_MAX_M)
        return PHICOMB_EINVAL;
    if (v && !finite_array(v, op->dev.n))
        return PHICOMB_EINVAL;
    std::lock_guard<std::mutex> g(op->mu);
    const int st = params_fp64(op, tol, m, v, seed, (hipStream_t)stream, out);
    out->status = st;
    return st;
}

int phicomb_solve(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                  const double *beta, const void *V, double tol, int precision, void *W,
                  void *stream, phicomb_stats_t *stats) {
    if (solve_check_args(op, prm, p, r, t, beta, V, tol, precision, W) != PHICOMB_OK)
        return PHICOMB_EINVAL;
    std::lock_guard<std::mutex> g(op->mu);
    const size_t need = solve_workspace_bytes(op->dev.n, p, r, precision, op_lr_rank(op));
    int st = ensure_workspace(op, need);
    if (st != PHICOMB_OK)
        return st;
    st = solve_run(op, prm, p, r, t, beta, V, tol, precision, W, (hipStream_t)stream, stats,
                   op->ws.ptr, op->ws.bytes, op->pinned);
    if (stats)
        stats->status = st;
    return st;
}

const char *phicomb_strerror(int status) {
    switch (status) {
    case PHICOMB_OK: return "ok";
    case PHICOMB_PENDING: return "pending";
    case PHICOMB_EINVAL: return "invalid argument";
    case PHICOMB_ENOMEM: return "device out of memory";
    case PHICOMB_EADMIT: return "request exceeds the serving memory budget";
    case PHICOMB_ENOCONV: return "Taylor loop hit the term cap";
    case PHICOMB_EOVERFLOW: return "power basis overflow (no power accepted)";
    case PHICOMB_EDEVICE: return "device error or non-finite result";
    default: return "unknown status";
    }
}

}  // extern "C"
