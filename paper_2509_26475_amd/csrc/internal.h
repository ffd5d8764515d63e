// Internal declarations of the phicomb HIP library (gfx950).
//
// Device-side building blocks shared by the kernels: operator row products
// (stencil, CSR), wave64 reductions, the grid barrier of the persistent
// kernels, and the host-side op/workspace structures.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "phicomb.h"

namespace phc {

constexpr int kWG = 256;                      // threads per workgroup (four wave64)
constexpr int kWaves = kWG / 64;
constexpr int kPMax1 = PHICOMB_MAX_P + 1;     // p + 1 <= 8
constexpr int kRMax = PHICOMB_MAX_R;          // r <= 4
constexpr int kTermCap = 150;                 // Taylor terms per loop
constexpr long kSpinLimit = 1L << 27;         // barrier wait bound (~10 s), then EDEVICE

enum OpKind : int { kStencil = 0, kCsr = 1, kDense = 2, kCsrCached = 3, kLowRank = 4 };
// Kernel-template kind only (never an operator's kind): a small dense
// operator held in LDS, with the whole solve on one workgroup.
constexpr int kDenseLds = 5;
__host__ __device__ constexpr bool is_dense(int kind) { return kind == kDense || kind == kDenseLds; }

// Low-rank operators A = U W^T: rank at most kLrRankMax.
constexpr int kLrRankMax = 16;
constexpr int kCacheNnz = 8;   // CSR rows up to this length can live in registers
// Largest operator: work-block columns are addressed with 32-bit byte offsets
// (ld_col), which hold FP64 columns of up to 2^29 rows; one power of two to spare.
constexpr int64_t kMaxRows = PHICOMB_MAX_N;

// Operator as seen by the kernels (passed by value).
struct DevOp {
    int kind;
    int dim;
    int nx, ny, nz;
    int pad;
    int64_t n;
    double c[7];          // stencil: centre, -x, +x, -y, +y, -z, +z
    double superdiag;     // stencil: added on (i, i+1), i < n-1
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *dense;  // row-major n x n
    int max_row_nnz;      // CSR: longest row
    int rank;             // low rank: columns of U and W
    const double *lr_u;   // low rank: U, row-major n x rank
    const double *lr_w;   // low rank: W, row-major n x rank
};

// ------------------------------------------------------------ reductions
// Max of non-negative doubles; a NaN operand wins so that it reaches the
// stopping test and is reported.
__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

// v moved by one DPP step (control CTRL, rows ROWS): the source lane's value
// where the step has one, v itself in the lanes it leaves alone.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_or_self(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false),
                            __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false));
}

// Max over the wave's 64 lanes, returned in every lane: row shifts by 1, 2,
// 4, 8 leave each 16-lane row's max in its last lane, two row broadcasts
// carry them to lane 63, which is read back as a scalar.  (Max is order
// free, so this equals any other reduction order, NaN included.)
__device__ __forceinline__ double wave_max(double v) {
    v = nmax(v, dpp_or_self<0x111, 0xF>(v));   // row_shr:1
    v = nmax(v, dpp_or_self<0x112, 0xF>(v));   // row_shr:2
    v = nmax(v, dpp_or_self<0x114, 0xF>(v));   // row_shr:4
    v = nmax(v, dpp_or_self<0x118, 0xF>(v));   // row_shr:8
    v = nmax(v, dpp_or_self<0x142, 0xA>(v));   // row_bcast:15 into rows 1, 3
    v = nmax(v, dpp_or_self<0x143, 0xC>(v));   // row_bcast:31 into rows 2, 3
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------- compensated inner products
// Inner products over all n rows (W^T x of a low-rank operator) are carried as
// unevaluated pairs hi + lo (Dot2 of Ogita, Rump and Oishi, SIAM J. Sci.
// Comput. 26, 2005): the product's rounding error comes from fma, the sum's
// from Knuth's TwoSum, and both are kept in lo.  The sum is then as accurate
// as if it had been formed in twice the working precision and rounded once,
// independently of the order in which rows, lanes and workgroups are added.
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_add(DD a, DD b) {
    const double s = a.hi + b.hi;
    const double z = s - a.hi;
    const double e = (a.hi - (s - z)) + (b.hi - z);   // s + e = a.hi + b.hi exactly
    return DD{s, e + (a.lo + b.lo)};
}

// acc += a * b
__device__ __forceinline__ void dd_fma(DD &acc, double a, double b) {
    const double p = a * b;
    const double pe = __builtin_fma(a, b, -p);         // p + pe = a b exactly
    const double s = acc.hi + p;
    const double z = s - acc.hi;
    const double e = (acc.hi - (s - z)) + (p - z);
    acc.hi = s;
    acc.lo += e + pe;
}

__device__ __forceinline__ DD wave_sum_dd(DD v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const DD o{__shfl_xor(v.hi, off, 64), __shfl_xor(v.lo, off, 64)};
        v = dd_add(v, o);
    }
    return v;
}

// ------------------------------------------------------------ grid barrier
// Barrier of a cooperative (co-resident) grid, grouped by XCD.
//
// Each XCD has its own L2, and an agent-scope release (L2 write-back) or
// acquire (L2 invalidate) acts on the whole L2 of the XCD that issues it, so
// one release and one acquire per XCD suffice.  Workgroups register in the
// group of the XCD they run on (hardware register XCC_ID) once, in
// grid_setup.  In grid_sync every workgroup waits for its own stores
// (workgroup release) and arrives at its group counter; the last arrival of a
// group (the leader) writes the XCD's L2 back and arrives at the top counter;
// the last leader opens the top generation; each leader then invalidates its
// caches and opens its group's generation; members invalidate theirs (agent
// scope, which includes the CU's L1) and continue.  Members cannot write between their leader's write-back and
// invalidate, so no dirty line is dropped.  Every wait is bounded; a timeout
// returns false and the kernel reports PHICOMB_EDEVICE.
constexpr int kLineU = 64;              // uint32 per 256-byte line
constexpr int kSyncLines = 64;          // size of the sync area in lines
constexpr int kSyncBytes = kSyncLines * kLineU * 4;
enum : int {
    kLnTop = 0, kLnTopGen = 1, kLnSetup = 2, kLnSetupFlag = 3,
    kLnGroup = 4,        // 16 group counters
    kLnGroupGen = 20,    // 16 group generations
    kLnGroupSize = 36,   // 16 group sizes
};

constexpr int kRedMax = 4;   // values one exchange reduces at most (lines of 4 u64)

struct GridSync {
    unsigned *bar;
    unsigned xcc, gsize, ngroups, gen;
};

__device__ __forceinline__ unsigned hw_xcc_id() {
    // HW_REG_XCC_ID (hwreg 20), bits [3:0]
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu;
}

__device__ __forceinline__ bool spin_until_ne(const unsigned *p, unsigned v) {
    long spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == v) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit)
            return false;
    }
    return true;
}

// Agent-scope release and acquire, each waited for in the same asm block:
// the compiler's own fences can emit the write-back without a wait for its
// completion, and a counter update that overtakes the write-back lets
// another XCD read stale lines.  The acquire (buffer_inv at agent scope,
// sc1) also invalidates the CU's vector L1; every workgroup needs it after a
// barrier.  A workgroup-scope invalidate (sc0) leaves the L1 alone: lines of
// a double-buffered block read two barriers earlier then come back stale
// once the per-term traffic is small enough not to evict them.
__device__ __forceinline__ void l2_writeback() {
    __asm__ volatile("buffer_wbl2 sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
}
__device__ __forceinline__ void l2_invalidate() {
    __asm__ volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
}

// Every wave waits until its own global stores are acknowledged by the L2
// before the workgroup arrives (s_barrier alone does not wait for them), so
// the leader's L2 write-back covers them.
__device__ __forceinline__ void wait_own_stores() { __builtin_amdgcn_s_waitcnt(0); }

// One-time flat, fully fenced registration barrier; thread 0 fills gs.
__device__ __forceinline__ bool grid_setup(GridSync &gs, unsigned *bar, int *ok_lds,
                                           unsigned nblocks) {
    wait_own_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned x = hw_xcc_id();
        atomicAdd(bar + kLineU * (kLnGroupSize + x), 1u);
        l2_writeback();
        const unsigned prev = atomicAdd(bar + kLineU * kLnSetup, 1u);
        if (prev == nblocks - 1) {
            l2_writeback();
            __hip_atomic_store(bar + kLineU * kLnSetupFlag, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else if (!spin_until_ne(bar + kLineU * kLnSetupFlag, 0u)) {
            ok = 0;
        }
        l2_invalidate();
        unsigned ng = 0;
        for (int k = 0; k < 16; ++k)
            ng += __hip_atomic_load(bar + kLineU * (kLnGroupSize + k), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        gs.bar = bar;
        gs.xcc = x;
        gs.gsize = __hip_atomic_load(bar + kLineU * (kLnGroupSize + x), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        gs.ngroups = ng;
        gs.gen = 0;
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

__device__ __forceinline__ bool grid_sync(GridSync &gs, int *ok_lds) {
    wait_own_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned g = gs.gen;
        unsigned *bar = gs.bar;
        unsigned *gc = bar + kLineU * (kLnGroup + gs.xcc);
        unsigned *gg = bar + kLineU * (kLnGroupGen + gs.xcc);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        // The counters only ever grow (modulo 2^32): arrival number
        // (g+1)*size - 1 closes generation g.  Nothing is reset, so an early
        // arrival at the next barrier can never be overwritten.
        const unsigned prev = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (prev + 1u == (g + 1u) * gs.gsize) {
            l2_writeback();
            const unsigned top = __hip_atomic_fetch_add(bar + kLineU * kLnTop, 1u,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (top + 1u == (g + 1u) * gs.ngroups)
                __hip_atomic_fetch_add(bar + kLineU * kLnTopGen, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            if (!spin_until_ne(bar + kLineU * kLnTopGen, g))
                ok = 0;
            l2_invalidate();
            __hip_atomic_store(gg, g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (!spin_until_ne(gg, g))
                ok = 0;
            l2_invalidate();   // this CU's L1 (and non-coherent L2 lines)
        }
        gs.gen = g + 1;
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

// Workgroup max of NV values into part[bid*kRedMax + j] (plain stores,
// published by the next grid_sync); bid is the workgroup's index within its
// grid.  (Folding the maxima into the barrier's arrival as agent-scope
// atomics was measured slower: the atomics' round trip lies on the
// barrier's critical path.)
template <int NV, int NT>
__device__ __forceinline__ void store_partials(double (&v)[NV], double *part,
                                               double (*red)[kRedMax], unsigned bid) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        v[j] = wave_max(v[j]);
    __syncthreads();   // every wave has finished reading red from the last exchange
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j)
            red[wave][j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double m = red[0][j];
            for (int w = 1; w < NT / 64; ++w)
                m = nmax(m, red[w][j]);
            part[bid * kRedMax + j] = m;
        }
    }
}

// Max over all workgroups' partials, after grid_sync; every thread gets it.
template <int NV, int NT>
__device__ __forceinline__ void load_partials(const double *part, unsigned nblocks,
                                              double (&out)[NV], double (*red)[kRedMax]) {
    double m[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j)
        m[j] = 0.0;
    for (unsigned b = threadIdx.x; b < nblocks; b += NT) {
#pragma unroll
        for (int j = 0; j < NV; ++j)
            m[j] = nmax(m[j], part[b * kRedMax + j]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        m[j] = wave_max(m[j]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j)
            red[wave][j] = m[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double r = red[0][j];
        for (int w = 1; w < NT / 64; ++w)
            r = nmax(r, red[w][j]);
        out[j] = r;
    }
}

// Max of NV values over one workgroup, left in every thread (a grid of a
// single workgroup needs no exchange through memory).
template <int NV, int NT>
__device__ __forceinline__ void workgroup_max(double (&v)[NV], double (*red)[kRedMax]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        v[j] = wave_max(v[j]);
    __syncthreads();   // every wave has finished reading red from the last exchange
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j)
            red[wave][j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double r = red[0][j];
        for (int w = 1; w < NT / 64; ++w)
            r = nmax(r, red[w][j]);
        v[j] = r;
    }
}

// Launch of a persistent kernel whose grid never exceeds the co-resident
// capacity (occupancy x CUs, computed by the caller).  The default is an
// ordinary launch: the blocking entry points own the device while they run,
// and the barrier's bounded wait turns a grid that is not fully resident
// into PHICOMB_EDEVICE instead of a hang.  PHICOMB_LAUNCH=cooperative asks
// the runtime for the co-residency guarantee instead.
inline hipError_t launch_persistent(const void *fn, unsigned grid, unsigned block, void **args,
                                    hipStream_t stream, size_t shmem = 0) {
    static const bool coop = [] {
        const char *e = getenv("PHICOMB_LAUNCH");
        return e && e[0] == 'c';
    }();
    return coop ? hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)shmem,
                                             stream)
                : hipLaunchKernel(fn, dim3(grid), dim3(block), args, shmem, stream);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical block ids so that neighbouring rows share an
// L2 slice.
__device__ __forceinline__ int xcd_logical_block(int b, int nblocks) {
    if (nblocks % 8 != 0)
        return b;
    return (b % 8) * (nblocks / 8) + b / 8;
}

// ------------------------------------------------------------ operator rows
// Everything about one output row that does not depend on the column block.
struct RowCtx {
    int64_t i;
    int q0, q1;          // CSR range
    unsigned mask;       // stencil neighbours present: bit0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z
    double cxp;          // stencil +x weight including the superdiagonal
};

template <int KIND>
__device__ __forceinline__ RowCtx row_ctx(const DevOp &A, int64_t row) {
    RowCtx rc;
    rc.i = row;
    if constexpr (KIND == kStencil) {
        const int r32 = (int)row;
        const int x = r32 % A.nx;
        const int yz = r32 / A.nx;
        const int y = yz % A.ny;
        const int z = yz / A.ny;
        unsigned m = 0;
        m |= (x > 0) ? 1u : 0u;
        const bool xp = x < A.nx - 1;
        const bool sd = (row < A.n - 1) && (A.superdiag != 0.0);
        m |= (xp || sd) ? 2u : 0u;
        m |= (y > 0) ? 4u : 0u;
        m |= (y < A.ny - 1) ? 8u : 0u;
        if (A.dim == 3) {
            m |= (z > 0) ? 16u : 0u;
            m |= (z < A.nz - 1) ? 32u : 0u;
        }
        rc.mask = m;
        rc.cxp = (xp ? A.c[2] : 0.0) + (sd ? A.superdiag : 0.0);
        rc.q0 = rc.q1 = 0;
    } else {
        rc.q0 = A.rowptr[row];
        rc.q1 = A.rowptr[row + 1];
        rc.mask = 0;
        rc.cxp = 0.0;
    }
    return rc;
}

// Load of element `idx` of a column, addressed as a wave-uniform base plus a
// 32-bit byte offset (columns are shorter than 2^28 elements), so the load
// needs a single offset VGPR instead of a 64-bit address pair.
template <typename T>
__device__ __forceinline__ T ld_col(const T *__restrict__ base, unsigned idx) {
    return *(const T *)((const char *)base + idx * (unsigned)sizeof(T));
}

// a b + c with one rounding, in the accumulation type.  Stencil rows are
// accumulated with explicit fused multiply-adds in a fixed order (centre
// product, then -x, +x, -y, +y, -z, +z) so that a row's value is the same in
// every kernel that computes it (one row per lane or two), whatever the
// compiler would contract on its own.
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// y[j] = (A X)(i, col0+j) - shift * X(i, col0+j), j < NC, with X of element
// type TX and the products accumulated in TA (double, or float for the
// reduced-precision terms).  X is column-major: column c at X + c*ld.
template <int KIND, int NC, typename TX, typename TA>
__device__ __forceinline__ void apply_cols(const DevOp &A, const RowCtx &rc,
                                           const TX *__restrict__ X, int64_t ld, int col0,
                                           double shift, TA (&y)[NC]) {
    const TX *__restrict__ cb[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j)
        cb[j] = X + (int64_t)(col0 + j) * ld;
    const unsigned i = (unsigned)rc.i;
    if constexpr (KIND == kStencil) {
        const TA cc = (TA)(A.c[0] - shift);
#pragma unroll
        for (int j = 0; j < NC; ++j)
            y[j] = cc * (TA)ld_col(cb[j], i);
        if (rc.mask & 1u) {
            const unsigned q = i - 1u;
            const TA w = (TA)A.c[1];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = fmadd(w, (TA)ld_col(cb[j], q), y[j]);
        }
        if (rc.mask & 2u) {
            const unsigned q = i + 1u;
            const TA w = (TA)rc.cxp;
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = fmadd(w, (TA)ld_col(cb[j], q), y[j]);
        }
        const unsigned sy = (unsigned)A.nx;
        if (rc.mask & 4u) {
            const unsigned q = i - sy;
            const TA w = (TA)A.c[3];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = fmadd(w, (TA)ld_col(cb[j], q), y[j]);
        }
        if (rc.mask & 8u) {
            const unsigned q = i + sy;
            const TA w = (TA)A.c[4];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = fmadd(w, (TA)ld_col(cb[j], q), y[j]);
        }
        const unsigned sz = (unsigned)A.nx * (unsigned)A.ny;
        if (rc.mask & 16u) {
            const unsigned q = i - sz;
            const TA w = (TA)A.c[5];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = fmadd(w, (TA)ld_col(cb[j], q), y[j]);
        }
        if (rc.mask & 32u) {
            const unsigned q = i + sz;
            const TA w = (TA)A.c[6];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = fmadd(w, (TA)ld_col(cb[j], q), y[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NC; ++j)
            y[j] = (TA)0;
        for (int q = rc.q0; q < rc.q1; ++q) {
            const TA a = (TA)A.val[q];
            const unsigned c = (unsigned)A.col[q];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] += a * (TA)ld_col(cb[j], c);
        }
        if (shift != 0.0) {
            const TA sh = (TA)shift;
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] -= sh * (TA)ld_col(cb[j], i);
        }
    }
}

// ------------------------------------------------------ stencil row pairs
// Rows i0 and i0 + 1 (i0 even) of a stencil product, NC columns, computed by
// one lane with 8- or 16-byte loads of the pair (float2 / double2).  The
// x-neighbours outside the pair (i0 - 1 and i0 + 2) belong to the adjacent
// lanes, which hold the adjacent pairs, and come over by cross-lane moves;
// only the first and last lane of a wave load theirs.  In linear row order
// the right neighbour i + 1 is also where the superdiagonal entry (i, i + 1)
// sits, so the end of a grid line needs no special case.  Requires nx even (a
// pair never straddles a grid line, n is even and the y and z offsets keep
// the pair's alignment) and every lane of the wave to take part: a lane past
// the end computes a clamped pair and its caller does not store it.
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec2<float> {
    typedef float __attribute__((ext_vector_type(2))) type;
};

template <typename T>
__device__ __forceinline__ typename Vec2<T>::type ld_pair(const T *__restrict__ base, unsigned i) {
    return *(const typename Vec2<T>::type *)((const char *)base + i * (unsigned)sizeof(T));
}

struct PairCtx {
    unsigned i0;          // even row of the pair
    unsigned mask;        // neighbours present: bit0 -y, 1 +y, 2 -z, 3 +z
    double wl0, wr0;      // row i0: weights of i0 - 1 and i0 + 1
    double wr1;           // row i0 + 1: weight of i0 + 2
};

__device__ __forceinline__ PairCtx pair_ctx(const DevOp &A, int64_t i0) {
    PairCtx pc;
    const unsigned i = (unsigned)i0;
    pc.i0 = i;
    const unsigned nx = (unsigned)A.nx, ny = (unsigned)A.ny;
    const unsigned x = i % nx, yz = i / nx;
    const unsigned y = yz % ny, z = yz / ny;
    unsigned m = 0;
    m |= (y > 0) ? 1u : 0u;
    m |= (y + 1 < ny) ? 2u : 0u;
    if (A.dim == 3) {
        m |= (z > 0) ? 4u : 0u;
        m |= (z + 1 < (unsigned)A.nz) ? 8u : 0u;
    }
    pc.mask = m;
    const int64_t n = A.n;
    pc.wl0 = (x > 0) ? A.c[1] : 0.0;
    pc.wr0 = A.c[2] + A.superdiag;   // x + 1 < nx always (x even, nx even); i0 + 1 < n
    pc.wr1 = ((x + 2 < nx) ? A.c[2] : 0.0) + ((i0 + 2 < n) ? A.superdiag : 0.0);
    return pc;
}

template <int NC, typename TX, typename TA>
__device__ __forceinline__ void apply_pair(const DevOp &A, const PairCtx &pc,
                                           const TX *__restrict__ X, int64_t ld, int col0,
                                           double shift, TA (&y0)[NC], TA (&y1)[NC]) {
    const int lane = threadIdx.x & 63;
    const unsigned i = pc.i0;
    const unsigned n = (unsigned)A.n;
    const unsigned sy = (unsigned)A.nx, sz = (unsigned)A.nx * (unsigned)A.ny;
    const TA cc = (TA)(A.c[0] - shift);
    const TA wl0 = (TA)pc.wl0, wr0 = (TA)pc.wr0, wl1 = (TA)A.c[1], wr1 = (TA)pc.wr1;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const TX *__restrict__ b = X + (int64_t)(col0 + j) * ld;
        const auto v = ld_pair(b, i);
        TX l = __shfl_up(v.y, 1, 64);
        TX r = __shfl_down(v.x, 1, 64);
        if (lane == 0)
            l = (i > 0) ? ld_col(b, i - 1u) : (TX)0;
        if (lane == 63)
            r = (i + 2u < n) ? ld_col(b, i + 2u) : (TX)0;
        // the same terms in the same order as apply_cols (centre, -x, +x,
        // -y, +y, -z, +z), so that a row's value does not depend on whether
        // it was computed alone or in a pair
        TA a0 = cc * (TA)v.x;
        a0 = fmadd(wl0, (TA)l, a0);
        a0 = fmadd(wr0, (TA)v.y, a0);
        TA a1 = cc * (TA)v.y;
        a1 = fmadd(wl1, (TA)v.x, a1);
        a1 = fmadd(wr1, (TA)r, a1);
        if (pc.mask & 1u) {
            const auto w = ld_pair(b, i - sy);
            a0 = fmadd((TA)A.c[3], (TA)w.x, a0);
            a1 = fmadd((TA)A.c[3], (TA)w.y, a1);
        }
        if (pc.mask & 2u) {
            const auto w = ld_pair(b, i + sy);
            a0 = fmadd((TA)A.c[4], (TA)w.x, a0);
            a1 = fmadd((TA)A.c[4], (TA)w.y, a1);
        }
        if (pc.mask & 4u) {
            const auto w = ld_pair(b, i - sz);
            a0 = fmadd((TA)A.c[5], (TA)w.x, a0);
            a1 = fmadd((TA)A.c[5], (TA)w.y, a1);
        }
        if (pc.mask & 8u) {
            const auto w = ld_pair(b, i + sz);
            a0 = fmadd((TA)A.c[6], (TA)w.x, a0);
            a1 = fmadd((TA)A.c[6], (TA)w.y, a1);
        }
        y0[j] = a0;
        y1[j] = a1;
    }
}

// A CSR row of at most kCacheNnz entries held in registers for a whole
// solve (the operator never changes between Taylor terms).
struct CachedRow {
    unsigned col[kCacheNnz];
    double val[kCacheNnz];
    int cnt;
};

__device__ __forceinline__ void load_cached_row(const DevOp &A, int64_t row, CachedRow &cr) {
    const int q0 = A.rowptr[row], q1 = A.rowptr[row + 1];
    cr.cnt = q1 - q0;
#pragma unroll
    for (int k = 0; k < kCacheNnz; ++k) {
        const bool in = k < cr.cnt;
        cr.col[k] = in ? (unsigned)A.col[q0 + k] : (unsigned)row;
        cr.val[k] = in ? A.val[q0 + k] : 0.0;
    }
}

template <int NC, typename TX, typename TA>
__device__ __forceinline__ void apply_cached(const CachedRow &cr, unsigned i,
                                             const TX *__restrict__ X, int64_t ld, int col0,
                                             double shift, TA (&y)[NC]) {
    const TX *__restrict__ cb[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        cb[j] = X + (int64_t)(col0 + j) * ld;
        y[j] = (TA)0;
    }
#pragma unroll
    for (int k = 0; k < kCacheNnz; ++k) {
        if (k < cr.cnt) {
            const TA a = (TA)cr.val[k];
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] += a * (TA)ld_col(cb[j], cr.col[k]);
        }
    }
    if (shift != 0.0) {
        const TA sh = (TA)shift;
#pragma unroll
        for (int j = 0; j < NC; ++j)
            y[j] -= sh * (TA)ld_col(cb[j], i);
    }
}

// ------------------------------------------------------------ host side
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace phc

struct phicomb_op_s {
    phc::DevOp dev;
    int device = 0;
    int64_t nnz = 0;
    double norm_inf = 0.0;        // max_i sum_j |a_ij| (bounds FP32 intermediates)
    void *mem = nullptr;          // device storage of the operator
    void *dense_mem = nullptr;    // dense operators: row-major n x n copy
    std::mutex mu;                // serialises solves on this operator
    phc::Workspace ws;            // grow-only workspace of blocking solves
    phc::Workspace aux;           // grow-only stage buffers of the time stepper
    double *pinned = nullptr;     // small pinned host buffer for read-backs
};

namespace phc {
// Workgroup-slot ledger of a device (implemented in api.cpp).  Persistent
// kernels spin at grid barriers, so two of them that are each only partly
// resident would wait on each other for ever; every persistent launch of the
// library therefore first takes its workgroup count from this ledger (one
// slot per CU, each workgroup fits a CU on its own) and returns it when the
// kernel has completed.
// Grants are whole multiples of kXcds: workgroups are dealt to the XCDs in
// turn, so a grid of G workgroups puts at most ceil(G/8) on any XCD; holding
// round_xcd(G) slots makes the ledger's bound hold on each XCD's own CUs.
constexpr int kXcds = 8;
inline int round_xcd(int64_t g) { return (int)((g + kXcds - 1) / kXcds * kXcds); }
int device_cus(int device);
int cu_acquire(int device, int want, int min_grant);   // blocks; returns granted in [min, want]
void cu_release(int device, int n);

// implemented in solve.hip
// cu_floor: fewest workgroups the solve accepts (0: one per CU up to n/512).
// events: two events for the kernel's device time, or nullptr to create and
// destroy a pair for this call.
int solve_run(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
              const double *beta, const void *V, double tol, int precision, void *W,
              hipStream_t stream, phicomb_stats_t *stats, void *ws, size_t ws_bytes,
              double *pinned, int cu_floor = 0, hipEvent_t *events = nullptr);
// Workgroups a solve on op asks the slot ledger for (want: one per CU up to
// one per 512 rows, dense operators one per 16 rows) and the fewest it can
// run with (floor: dense operators need one per kDenseRows rows).
void solve_grid_request(phicomb_op op, int *want, int *floor_g);
// rank > 0: a low-rank operator of that rank (adds the W^T X exchange area)
size_t solve_workspace_bytes(int64_t n, int p, int r, int precision, int rank = 0);
// rank of a low-rank operator, 0 for the other kinds
inline int op_lr_rank(const phicomb_op_s *op) { return op->dev.kind == kLowRank ? op->dev.rank : 0; }
// implemented in params.hip
int params_fp64(phicomb_op op, double tol, int m, const double *v, uint64_t seed,
                hipStream_t stream, phicomb_params_t *out);
// implemented in api.cpp
int ensure_workspace(phicomb_op op, size_t bytes);
// Host-side argument checks of phicomb_solve (sizes, finiteness of t, beta
// and tol, parameters, precision): PHICOMB_OK or PHICOMB_EINVAL.
int solve_check_args(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                     const double *beta, const void *V, double tol, int precision, void *W);
}  // namespace phc
