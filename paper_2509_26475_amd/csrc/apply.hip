// Block product Y = (A - shift I) X on its own: the operation every Taylor
// term of Algorithms 1-3 is built from (the paper accesses A only through
// such products).  Used to measure what the product alone reaches on HBM.
//
// One thread per row, 256-row workgroups mapped so that each XCD gets a
// contiguous range of rows (neighbouring rows of a stencil or banded CSR
// operator then share an L2).  Up to 16 columns are done by a kernel of that
// exact width (CSR rows of at most kCacheNnz entries loaded whole into
// registers first); wider blocks in compile-time chunks of NC, so that a CSR
// row's indices and values are read once per chunk.  Stencils with an even grid
// line run one pair of rows per thread instead (16-byte loads and stores,
// x-neighbours across lanes): 4.9 against 3.6 TB/s at 6 columns on the 128^3
// grid; more than 8 such columns run as chunks of 6 (one launch, grid.y
// over the chunks) and one launch for the remaining columns.  X and Y are
// column-major (column c at X + c n).
#include <cmath>
#include <cstring>
#include <utility>

#include "internal.h"

namespace phc {

constexpr int kANT = 256;
constexpr int kPairChunk = 6;   // columns of a chunk when a row-pair product is split

template <int KIND, int NC>
__global__ __launch_bounds__(kANT) void apply_kernel(DevOp A, const double *__restrict__ X,
                                                     int ncols, double shift,
                                                     double *__restrict__ Y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t row = (int64_t)b * kANT + threadIdx.x;
    const int64_t n = A.n;
    if (row >= n)
        return;
    const RowCtx rc = row_ctx<KIND>(A, row);
    for (int c0 = 0; c0 < ncols; c0 += NC) {
        double y[NC];
        apply_cols<KIND, NC>(A, rc, X, n, c0, shift, y);
#pragma unroll
        for (int j = 0; j < NC; ++j)
            Y[(int64_t)(c0 + j) * n + row] = y[j];
    }
}

// Exactly NC columns: no column loop (a runtime chunk loop costs about a
// third of the bandwidth on the 128^3 stencil).
template <int KIND, int NC>
__global__ __launch_bounds__(kANT) void apply_kernel_exact(DevOp A, const double *__restrict__ X,
                                                           int, double shift,
                                                           double *__restrict__ Y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t row = (int64_t)b * kANT + threadIdx.x;
    const int64_t n = A.n;
    if (row >= n)
        return;
    const RowCtx rc = row_ctx<KIND>(A, row);
    double y[NC];
    apply_cols<KIND, NC>(A, rc, X, n, 0, shift, y);
#pragma unroll
    for (int j = 0; j < NC; ++j)
        Y[(int64_t)j * n + row] = y[j];
}

// CSR rows of at most kCacheNnz entries (as the solve keeps them): the row's
// indices and values are loaded together first, then the gathers of all its
// entries and columns are in flight at once; exactly NC columns.  Sums in the
// same order as apply_cols.
template <int NC>
__global__ __launch_bounds__(kANT) void apply_csr_cached_kernel(DevOp A,
                                                                const double *__restrict__ X,
                                                                int, double shift,
                                                                double *__restrict__ Y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t row = (int64_t)b * kANT + threadIdx.x;
    const int64_t n = A.n;
    if (row >= n)
        return;
    CachedRow cr;
    load_cached_row(A, row, cr);
    double y[NC];
    apply_cached<NC, double, double>(cr, (unsigned)row, X, n, 0, shift, y);
#pragma unroll
    for (int j = 0; j < NC; ++j)
        Y[(int64_t)j * n + row] = y[j];
}

// Stencil operators with nx even: one lane per pair of consecutive rows
// (16-byte loads, x-neighbours across lanes; see apply_pair).  Lanes past the
// end compute a clamped pair and store nothing.
template <int NC>
__global__ __launch_bounds__(kANT) void apply_pairs_kernel(DevOp A, const double *__restrict__ X,
                                                           int, double shift,
                                                           double *__restrict__ Y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t n = A.n;
    const int64_t i0 = 2 * ((int64_t)b * kANT + threadIdx.x);
    const bool act = i0 < n;
    // grid.y selects a chunk of NC columns (wide blocks run as several chunks)
    X += (int64_t)blockIdx.y * NC * n;
    Y += (int64_t)blockIdx.y * NC * n;
    const PairCtx pc = pair_ctx(A, act ? i0 : n - 2);
    double y0[NC], y1[NC];
    apply_pair<NC, double, double>(A, pc, X, n, 0, shift, y0, y1);
    if (act) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            typedef double __attribute__((ext_vector_type(2))) d2;
            d2 v = {y0[j], y1[j]};
            *(d2 *)(Y + (int64_t)j * n + i0) = v;
        }
    }
}

using ApplyFn = void (*)(DevOp, const double *, int, double, double *);

template <int... Q>
static ApplyFn pairs_fn(int ncols, std::integer_sequence<int, Q...>) {
    ApplyFn fn = nullptr;
    ((ncols == Q + 1 ? (fn = apply_pairs_kernel<Q + 1>, 0) : 0), ...);
    return fn;
}

template <int... Q>
static ApplyFn cached_fn(int ncols, std::integer_sequence<int, Q...>) {
    ApplyFn fn = nullptr;
    ((ncols == Q + 1 ? (fn = apply_csr_cached_kernel<Q + 1>, 0) : 0), ...);
    return fn;
}

template <int KIND, int... Q>
static ApplyFn exact_fn(int ncols, std::integer_sequence<int, Q...>) {
    ApplyFn fn = nullptr;
    ((ncols == Q + 1 ? (fn = apply_kernel_exact<KIND, Q + 1>, 0) : 0), ...);
    return fn;
}

template <int KIND>
static ApplyFn apply_fn(int ncols) {
    if (ncols <= 16)
        return exact_fn<KIND>(ncols, std::make_integer_sequence<int, 16>{});
    // wider blocks: the widest chunk that divides the column count
    if (ncols % 12 == 0)
        return apply_kernel<KIND, 12>;
    if (ncols % 8 == 0)
        return apply_kernel<KIND, 8>;
    if (ncols % 6 == 0)
        return apply_kernel<KIND, 6>;
    if (ncols % 4 == 0)
        return apply_kernel<KIND, 4>;
    if (ncols % 3 == 0)
        return apply_kernel<KIND, 3>;
    if (ncols % 2 == 0)
        return apply_kernel<KIND, 2>;
    return apply_kernel<KIND, 1>;
}

}  // namespace phc

using namespace phc;

extern "C" int phicomb_op_apply(phicomb_op op, const void *X, int ncols, double shift, void *Y,
                                void *stream_, double *ms) {
    if (ms)
        *ms = 0.0;
    if (!op || !X || !Y || ncols < 1 || ncols > 64 || !std::isfinite(shift))
        return PHICOMB_EINVAL;
    const int kind = op->dev.kind;
    if (kind == kLowRank)
        return PHICOMB_EINVAL;
    // dense operators through their CSR form
    ApplyFn fn = (kind == kStencil) ? apply_fn<kStencil>(ncols) : apply_fn<kCsr>(ncols);
    hipStream_t stream = (hipStream_t)stream_;
    const int64_t n = op->dev.n;
    int64_t blocks = (n + kANT - 1) / kANT;
    // stencils with an even grid line and at most 16 columns: row pairs;
    // more than 8 columns as chunks of 6 on grid.y plus one launch for the
    // rest (12 columns in one kernel keep too few loads in flight: 3.1 TB/s
    // against 4.9 TB/s at 6 on the 128^3 grid)
    int chunks = 1, rest = 0;
    ApplyFn fn_rest = nullptr;
    // CSR with short rows and at most 16 columns: the row in registers
    if (kind == kCsr && op->dev.max_row_nnz <= kCacheNnz && ncols <= 16)
        fn = cached_fn(ncols, std::make_integer_sequence<int, 16>{});
    if (kind == kStencil && op->dev.nx % 2 == 0 && ncols <= 16) {
        blocks = (n / 2 + kANT - 1) / kANT;
        if (ncols > 8) {
            chunks = ncols / kPairChunk;
            rest = ncols % kPairChunk;
            fn = pairs_fn(kPairChunk, std::make_integer_sequence<int, 16>{});
            if (rest)
                fn_rest = pairs_fn(rest, std::make_integer_sequence<int, 16>{});
        } else {
            fn = pairs_fn(ncols, std::make_integer_sequence<int, 16>{});
        }
    }
    if (blocks > 0x7fffffff)
        return PHICOMB_EINVAL;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = ms && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (!timed && e0)   // the second event could not be made
        (void)hipEventDestroy(e0);
    if (timed)
        (void)hipEventRecord(e0, stream);
    fn<<<dim3((unsigned)blocks, (unsigned)chunks), kANT, 0, stream>>>(
        op->dev, (const double *)X, ncols, shift, (double *)Y);
    if (fn_rest) {
        const int64_t off = (int64_t)(ncols - rest) * n;
        fn_rest<<<(unsigned)blocks, kANT, 0, stream>>>(op->dev, (const double *)X + off, rest,
                                                       shift, (double *)Y + off);
    }
    if (hipGetLastError() != hipSuccess) {
        if (timed) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
        }
        return PHICOMB_EDEVICE;
    }
    int st = PHICOMB_OK;
    if (timed) {
        (void)hipEventRecord(e1, stream);
        float t = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            st = PHICOMB_EDEVICE;
        *ms = t;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return st;
}
