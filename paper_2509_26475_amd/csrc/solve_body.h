// Device side of the Algorithm 3 solve, shared by the single-solve kernel
// (solve.hip) and the batched kernel (batch.hip).
// Block truncated-Taylor scaling-and-recovering solve (Al-Mohy, Sec. 4,
// Algorithm 3; r = 1 is Algorithm 2), FP64, one persistent cooperative kernel.
//
// Work blocks are column-major ([columns][n]) so that every column access of
// a wave64 is one contiguous 512-byte segment:
//   S  [(p+1) r][n]  scaled block series S of (rec.D); column (b, i) at b*r + i,
//                    block b holding v_perm(b), perm = (0, p, p-1, ..., 1)
//   U0, U1           ping-pong term blocks: D_k/k! in the S-series, then the
//                    Taylor terms F of the recovery loop (2r columns); they are
//                    the only blocks other workgroups read (operator products)
//   E                partial sums of the recovery loop: registers of the
//                    thread that owns the row (rows per thread fixed at compile
//                    time), or [2r][n] in memory for very large n
// The weights beta are folded into the columns of V (Corollary of Theorem 1),
// so the Kronecker factor J (x) Delta reduces to one J per abscissa and
// exp(J (x) Delta / s) to exp(J/s).  The replicated V of the listing is never
// stored: its k-th update V J_step^(k-1) is formed per row from the p+1 input
// vectors with (p+1)^2 coefficients per abscissa kept in LDS.
//
// Every Taylor term ends with one grid-wide exchange: each workgroup writes
// the maxima of its row sums (block infinity norms), crosses the XCD-grouped
// grid barrier, and reduces all workgroups' maxima itself, so every thread
// takes the same stopping decision.
//
// Low-rank operators A = U W^T (Sec. 5, third experiment) are applied
// matrix-free as x -> U (W^T x).  The small matrix W^T X of the block X that
// the next product needs rides on the same exchange: the pass that writes X
// also leaves this workgroup's partial sums over its rows, and after the
// barrier every workgroup adds all workgroups' partials in index order, so
// each holds the same W^T X; row i of the product is then U_i (W^T X) minus
// the shift times X_i, from the row's own data only.
#pragma once

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>

#include "internal.h"

namespace phc {

constexpr int kNT = 512;           // threads per workgroup of the solve kernel (8 waves)
constexpr int kWideNT = 1024;      // the E-in-memory stencil kernel (16 waves, see pick_wide)
constexpr int kMaxNT = 1024;
constexpr int kMaxGrid = 4096;     // partial-maximum slots per parity
constexpr int kLrVals = 256;       // entries of W^T X exchanged per term at most

struct SolveArgs {
    DevOp op;
    int64_t n;
    int p, r, P1, cS, cR, s_int, kcap;
    double tol, xi, nu;                 // nu = 1/s_int (superdiagonal of the J step)
    double ts[kRMax];                   // t_i / s_int
    double t[kRMax];                    // t_i
    double mu[kRMax];                   // exp(xi t_i / s_int): undo factor of the shift
    double w0[kRMax];                   // beta_i0: weight of v_0 in exp(t_i A/s) v_0
    double a[kRMax];                    // -xi t_i / s_int: diagonal of the J step
    double gam[kRMax][kPMax1];          // column (b,i) scale beta_{i,perm(b)} mu_i / s_int
    const double *V;                    // [n][p+1] row-major (caller)
    double *W;                          // [n][r]  row-major (caller)
    double *S, *U0, *U1, *E;
    float *Uf0, *Uf1;                   // FP32 term blocks [max(cS, cR)][n] (mixed precision)
    double mix_tau;                     // tol / (10 u_fp32): FP32 term threshold
    double mix_lo, mix_hi;              // partial-sum norms for which FP32 terms are safe
    unsigned *bar;                      // sync area (kSyncBytes)
    double *part;                       // [2][kMaxGrid][kRedMax] partial maxima
    double *lrpart;                     // low rank: [2][2][lrv][kMaxGrid] partial W^T X (hi, lo)
    int lrv;                            // low rank: rank * max(cS + r, 2r)
    int *info;                          // status, terms_S, terms_rec, max_terms_step
};

template <class F, int... Q>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Q...>) {
    (f(std::integral_constant<int, Q>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Visit the rows this thread owns.  Register-resident layout: RPT rows at
// stride NT inside the workgroup's contiguous chunk, visited with a
// compile-time index q; memory layout: a grid-stride loop over the chunk.
template <int RPT, bool EMEM, int NT, class F>
__device__ __forceinline__ void for_rows(int64_t lo, int64_t hi, F &&f) {
    if constexpr (EMEM) {
        for (int64_t row = lo + threadIdx.x; row < hi; row += NT)
            f(row, std::integral_constant<int, 0>{});
    } else {
        static_for<RPT>([&](auto q) {
            unsigned r32 = (unsigned)(lo + threadIdx.x) + (unsigned)(decltype(q)::value * NT);
            // opaque to the optimiser: addresses derived from the row are
            // rebuilt inside every Taylor term instead of being hoisted out
            // of the term loop and kept live for all RPT rows
            __asm__ volatile("" : "+v"(r32));
            const int64_t row = (int64_t)r32;
            if (row < hi)
                f(row, q);
            // keep the rows apart: their loads would otherwise be interleaved
            // and multiply the register footprint by RPT
            __builtin_amdgcn_sched_barrier(0);
        });
    }
}

// Mixed precision (MIX): in every Taylor loop (the S-series and each
// recovery step) a term is computed and stored in FP32 once the previous
// term is small enough that FP32 rounding of the new one stays below tol/10
// of the loop's result (an FP64 head then an FP32 tail).  The reference for
// "the loop's result" is the smaller of the partial sum and the loop's
// starting block: partial sums of a rough block swell through cancellation
// before they settle, so they alone would let FP32 in too early.  The
// partial sums, the stopping test and everything carried from one loop to
// the next stay FP64.
constexpr double kMixSafety = 8.0;   // allowed growth of a term over its predecessor

// ------------------------------------------------------------ dense operator
// A dense operator (row-major n x n) is applied per Taylor term to every
// column the term needs at once: the workgroup computes the products of its
// (at most kDenseRows) rows with FP64 MFMA 16x16x4 tiles, the k range split
// over the waves when there are fewer tiles than waves, the partial tiles
// summed in LDS; the row owners then read their products from LDS.
// v_mfma_f64_16x16x4f64 lane layout (checked on the device): A operand
// A[l % 16][l / 16], B operand B[l / 16][l % 16], result element v of lane l
// is D[l / 16 + 4 v][l % 16].
constexpr int kDenseRows = 128;   // rows per workgroup at most
constexpr int kDenseCols = 32;    // columns per product at most ((p+1) r)
constexpr int kSolveWaves = kNT / 64;
constexpr int kDenseBlocks = 4;   // blocks of 16 k whose loads are in flight together
constexpr int kDenseTail = 8;     // steps of 4 k a round in the rest of a slice
// two doubles at 8-byte alignment (a row of A starts at 8 n bytes)
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));

struct DenseShared {
    double Y[kDenseRows][kDenseCols + 1];   // products of the workgroup's rows
    double part[2 * kSolveWaves][16][17];        // partial 16 x 16 tiles
};

typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

// Small dense operators (n <= kDenseLdsN) on one workgroup.  A stays in
// registers for the whole solve: lane l of wave w holds row 16 w + l / 4,
// columns k = 4 j + l % 4 (j < kDenseLdsJ, zero past n), so a product needs
// no A traffic at all; the term blocks S, U0, U1 and E live in LDS, so a
// Taylor term touches no global memory.  Products run on the vector ALUs
// (two columns at a time, the four partial sums of a row added across the
// lanes of a quad), which for the few columns of a term beats a 16-column
// MFMA tile that FP64 fills at half rate on this chip.
constexpr int kDenseLdsN = 112;
constexpr int kDenseLdsJ = kDenseLdsN / 4;   // columns of A a lane holds
struct DenseLdsShared {
    double Y[kDenseLdsN][kDenseCols + 1];   // products of all rows
};

// Y[i][c] = sum_k A[lo+i][k] X[c n + k] - shift X[c n + lo + i],
// i < hi - lo, c < ncols.  Every thread of the workgroup calls it.
__device__ __forceinline__ void dense_products(const double *__restrict__ Ad, int64_t n,
                                               int64_t lo, int64_t hi,
                                               const double *__restrict__ X, int ncols,
                                               double shift, DenseShared &ds) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rows = (int)(hi - lo);
    const int RT = (rows + 15) / 16, CT = (ncols + 15) / 16;
    const int tiles = RT * CT;
    const int KS = tiles >= kSolveWaves ? 1 : kSolveWaves / tiles;   // k slices per tile
    const int64_t kchunk = ((n + KS - 1) / KS + 3) / 4 * 4;
    for (int task = wave; task < tiles * KS; task += kSolveWaves) {
        const int tile = task % tiles, ks = task / tiles;
        const int rt = tile % RT, ct = tile / RT;
        const int64_t row = lo + rt * 16 + (lane & 15);
        const int col = ct * 16 + (lane & 15);
        const bool rok = row < hi, cok = col < ncols;
        const double *arow = Ad + (rok ? row : lo) * n;
        const double *xcol = X + (int64_t)(cok ? col : 0) * n;
        const int64_t kb = ks * kchunk, ke = std::min<int64_t>(n, kb + kchunk);
        mfma_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const int kq = lane >> 4;
        // Whole blocks of 16 k, kDenseBlocks of them a round: a lane loads
        // four consecutive k of its row of A and of its column of X (two
        // 16-byte loads each, k0 = 16 j + 4 kq within the block), and MFMA
        // step u of the block takes the u-th of them, so every k of the block
        // is used once; all loads of a round are issued before its MFMAs.
        // Rows and columns outside the operands read row lo or column 0 and
        // contribute zeros.
        int64_t kk = kb;
        for (; kk + 16 * kDenseBlocks <= ke; kk += 16 * kDenseBlocks) {
            dbl2u a[kDenseBlocks][2], b[kDenseBlocks][2];
#pragma unroll
            for (int j = 0; j < kDenseBlocks; ++j) {
                const int64_t k0 = kk + 16 * j + 4 * kq;
                a[j][0] = *(const dbl2u *)(arow + k0);
                a[j][1] = *(const dbl2u *)(arow + k0 + 2);
                b[j][0] = *(const dbl2u *)(xcol + k0);
                b[j][1] = *(const dbl2u *)(xcol + k0 + 2);
            }
#pragma unroll
            for (int j = 0; j < kDenseBlocks; ++j) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double av = (u < 2) ? a[j][0][u] : a[j][1][u - 2];
                    const double bv = (u < 2) ? b[j][0][u] : b[j][1][u - 2];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(rok ? av : 0.0, cok ? bv : 0.0,
                                                               acc, 0, 0, 0);
                }
            }
        }
        // the rest of the slice (under 16 kDenseBlocks values of k): steps of
        // four k in ascending order, k clamped into the slice (whose last
        // element exists) and steps past it multiplying zeros
        for (; kk < ke; kk += 4 * kDenseTail) {
            double a[kDenseTail], b[kDenseTail];
#pragma unroll
            for (int u = 0; u < kDenseTail; ++u) {
                const int64_t k = kk + 4 * u + kq;
                const bool kok = k < ke;
                const int64_t kc = kok ? k : ke - 1;
                const double av = arow[kc], bv = xcol[kc];
                a[u] = (rok && kok) ? av : 0.0;
                b[u] = (cok && kok) ? bv : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kDenseTail; ++u)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            ds.part[task][(lane >> 4) + 4 * v][lane & 15] = acc[v];
    }
    __syncthreads();
    for (int e = tid; e < rows * ncols; e += kNT) {
        const int i = e / ncols, c = e % ncols;
        const int tile = (i >> 4) + RT * (c >> 4);
        double sum = 0.0;
        for (int ks = 0; ks < KS; ++ks)
            sum += ds.part[tile + ks * tiles][i & 15][c & 15];
        ds.Y[i][c] = sum - shift * X[(int64_t)c * n + lo + i];
    }
    __syncthreads();
}

// v summed over the four lanes of each quad (DPP quad permutations, the same
// order in every lane: (v0 + v1) + (v2 + v3)).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double quad_sum(double v) {
    v = v + dpp_f64<0xB1>(v);      // lanes q ^ 1
    return v + dpp_f64<0x4E>(v);   // lanes q ^ 2
}

// Y[i][c] = sum_k A[i][k] X[c n + k] - shift X[c n + i] for i < n, c < ncols,
// A in the registers areg (layout above), X in LDS.  X is read at a clamped
// index past n (A is zero there).  Every thread of the workgroup calls it.
__device__ __forceinline__ void dense_products_lds(const double (&areg)[kDenseLdsJ], int64_t n,
                                                   const double *__restrict__ X, int ncols,
                                                   double shift, DenseLdsShared &ds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = wave * 16 + (lane >> 2), q = lane & 3;
    const int nm1 = (int)n - 1;
    if (wave * 16 < n) {
        for (int c0 = 0; c0 < ncols; c0 += 2) {
            const double *x0 = X + (int64_t)c0 * n;
            const double *x1 = X + (int64_t)min(c0 + 1, ncols - 1) * n;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int j = 0; j < kDenseLdsJ; ++j) {
                const int k = min(4 * j + q, nm1);
                a0 = fma(areg[j], x0[k], a0);
                a1 = fma(areg[j], x1[k], a1);
            }
            a0 = quad_sum(a0);
            a1 = quad_sum(a1);
            if (q == 0 && i < n) {
                ds.Y[i][c0] = a0 - shift * x0[i];
                if (c0 + 1 < ncols)
                    ds.Y[i][c0 + 1] = a1 - shift * x1[i];
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------- low-rank operator
// This workgroup's partial sums of W^T X over its rows [lo, hi) for columns
// c < ncols of X (column-major, leading dimension n), as compensated pairs
// stored value-major: hi at out[(voff + c rank + k) kMaxGrid + bid], lo at
// the same index plus lo_off.  One wave per value, lanes over the rows, a
// fixed shuffle tree.  The block was written by this workgroup.
template <class TX>
__device__ __forceinline__ void lr_publish(const DevOp &A, int64_t n, int64_t lo, int64_t hi,
                                           const TX *__restrict__ X, int ncols, int voff,
                                           double *__restrict__ out, size_t lo_off,
                                           unsigned bid) {
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rank = A.rank;
    for (int v = wave; v < ncols * rank; v += kNT / 64) {
        const int c = v / rank, k = v % rank;
        const TX *xc = X + (int64_t)c * n;
        DD acc{0.0, 0.0};
        for (int64_t row = lo + lane; row < hi; row += 64)
            dd_fma(acc, A.lr_w[row * rank + k], (double)xc[row]);
        acc = wave_sum_dd(acc);
        if (lane == 0) {
            const size_t o = (size_t)(voff + v) * kMaxGrid + bid;
            out[o] = acc.hi;
            out[o + lo_off] = acc.lo;
        }
    }
}

// W^T X = the sum of all G workgroups' partial pairs, in the same order in
// every workgroup: one wave per value, lanes over the workgroups, a fixed
// tree, rounded once at the end.
__device__ __forceinline__ void lr_gather(const double *__restrict__ part, size_t lo_off,
                                          unsigned G, int nv, double *lrc) {
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = wave; v < nv; v += kNT / 64) {
        DD acc{0.0, 0.0};
        for (unsigned g = lane; g < G; g += 64) {
            const size_t o = (size_t)v * kMaxGrid + g;
            acc = dd_add(acc, DD{part[o], part[o + lo_off]});
        }
        acc = wave_sum_dd(acc);
        if (lane == 0)
            lrc[v] = acc.hi + acc.lo;
    }
    __syncthreads();
}

// Visit the row pairs (i0, i0 + 1), i0 even, of the rows [lo, hi) (lo even)
// with a wave-uniform loop: every lane of a wave takes part in each step
// (the pair product exchanges x-neighbours across lanes).  A lane whose pair
// starts at or past hi is inactive (act = false) but still computes with its
// true pair while that lies inside the operator, so that its neighbours
// across lanes are right; past n it computes the last pair.
template <int NT, class F>
__device__ __forceinline__ void for_pairs(int64_t lo, int64_t hi, int64_t n, F &&f) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t pb = lo / 2 + wave * 64; 2 * pb < hi; pb += NT) {
        const int64_t i0 = 2 * (pb + lane);
        f(i0 < n ? i0 : n - 2, i0 < hi);
    }
}

template <typename T>
struct TypeTag {
    using type = T;
};

// Workgroup-shared state of one solve.
struct SolveShared {
    double Mk[kRMax][kPMax1][kPMax1];   // J_step^(k-1) / k!
    double Cj[kRMax][kPMax1][kPMax1];   // gam[i][b] * Mk[i][b][.]
    double red[kMaxNT / 64][kRedMax];
    double lrc[kLrVals];                // low rank: W^T X of the coming product
    int ok;
};

// Algorithm 3 for one solve on a grid of G workgroups; this workgroup is
// number bid of them and owns the rows of logical block lb.
template <int KIND, int R, int RPT, bool EMEM, bool MIX, int NT = kNT>
__device__ __forceinline__ void solve_body(const SolveArgs &P, SolveShared &sh, const unsigned G,
                                           const unsigned bid, const int lb) {
    auto &Mk = sh.Mk;
    auto &Cj = sh.Cj;
    auto &red = sh.red;
    const int64_t n = P.n;
    // term blocks: the caller's global memory, or LDS for a small dense
    // operator on one workgroup (A itself then held in registers, areg)
    double *bS = P.S, *bU0 = P.U0, *bU1 = P.U1, *bE = P.E;
    double areg[KIND == kDenseLds ? kDenseLdsJ : 1];
    if constexpr (KIND == kDenseLds) {
        extern __shared__ double lds_dyn[];
        const int i = (threadIdx.x >> 6) * 16 + ((threadIdx.x & 63) >> 2), q = threadIdx.x & 3;
#pragma unroll
        for (int j = 0; j < kDenseLdsJ; ++j) {
            const int k = 4 * j + q;
            areg[j] = (i < n && k < n) ? P.op.dense[(int64_t)i * n + k] : 0.0;
        }
        const int64_t cW = P.cS > P.cR ? P.cS : P.cR;
        bS = lds_dyn;
        bU0 = bS + P.cS * n;
        bU1 = bU0 + cW * n;
        bE = bU1 + cW * n;
    }
    int64_t lo, hi;
    if constexpr (EMEM) {
        // an even chunk: row pairs never straddle two workgroups
        const int64_t chunk = ((n + G - 1) / G + 1) & ~(int64_t)1;
        lo = std::min<int64_t>(n, (int64_t)lb * chunk);
        hi = std::min<int64_t>(n, lo + chunk);
    } else {
        lo = std::min<int64_t>(n, (int64_t)lb * NT * RPT);
        hi = std::min<int64_t>(n, lo + (int64_t)NT * RPT);
    }
    const int tid = threadIdx.x;
    const int P1 = P.P1, p = P.p;
    const DevOp &A = P.op;
    double Ereg[EMEM ? 1 : RPT][2 * R];
    auto Eref = [&](int64_t row, auto q, int c) -> double & {
        if constexpr (EMEM)
            return bE[(int64_t)c * n + row];
        else
            return Ereg[decltype(q)::value][c];
    };
    int n32 = 0, n32S = 0;   // recovery and S-series terms evaluated in FP32
    auto finish = [&](int st, int tS, int tR, int mS) {
        if (bid == 0 && tid == 0) {
            P.info[0] = st;
            P.info[1] = tS;
            P.info[2] = tR;
            P.info[3] = mS;
            P.info[4] = n32;
            P.info[5] = n32S;
        }
    };

    // Operator rows: CSR rows of at most kCacheNnz entries stay in registers
    // for the whole solve; other kinds rebuild their row context per product.
    constexpr bool CACHED = (KIND == kCsrCached);
    // stencils with E in memory and an even grid line: products by row pairs
    // (the wide 16-wave kernel is launched for such operators only and has
    // no single-row path)
    constexpr bool PAIRS_ONLY = (NT == kWideNT);
    bool pairs = PAIRS_ONLY;
    if constexpr (KIND == kStencil && EMEM && !PAIRS_ONLY)
        pairs = (A.nx % 2 == 0);
    CachedRow crow[CACHED ? RPT : 1];
    if constexpr (CACHED)
        for_rows<RPT, EMEM, NT>(lo, hi, [&](int64_t row, auto q) {
            load_cached_row(A, row, crow[decltype(q)::value]);
        });
    int lr_off = 0;   // low rank: column of W^T X holding the operand's first column
    using DS = std::conditional_t<KIND == kDenseLds, DenseLdsShared, DenseShared>;
    DS *dsp = nullptr;
    if constexpr (is_dense(KIND)) {
        __shared__ DS dense_lds;
        dsp = &dense_lds;
    }
    // dense operator: products of this workgroup's rows for the coming term
    auto dense_pass = [&](const double *X, int ncols, double shift)
                          __attribute__((always_inline)) {
        if constexpr (KIND == kDense)
            dense_products(A.dense, n, lo, hi, X, ncols, shift, *dsp);
        else if constexpr (KIND == kDenseLds)
            dense_products_lds(areg, n, X, ncols, shift, *dsp);
    };
    auto opr = [&](int64_t row, auto q, const auto *X, int col0, double shift,
                   auto &y) __attribute__((always_inline)) {
        using Y = std::remove_reference_t<decltype(y)>;
        constexpr int NC = std::extent<Y>::value;
        using TA = std::remove_extent_t<Y>;
        using TX = std::remove_cv_t<std::remove_pointer_t<decltype(X)>>;
        if constexpr (is_dense(KIND)) {
            // products computed by dense_products for this term
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = (TA)dsp->Y[row - lo][col0 + j];
        } else if constexpr (KIND == kLowRank) {
            // U_row (W^T X) - shift X_row, W^T X gathered at the last exchange
            const int rank = A.rank;
            const double *ur = A.lr_u + row * rank;
            const double *cw = sh.lrc + (lr_off + col0) * rank;
#pragma unroll
            for (int j = 0; j < NC; ++j)
                y[j] = -(TA)shift * (TA)X[(int64_t)(col0 + j) * n + row];
            for (int k = 0; k < rank; ++k) {
                const TA u = (TA)ur[k];
#pragma unroll
                for (int j = 0; j < NC; ++j)
                    y[j] += u * (TA)cw[j * rank + k];
            }
        } else if constexpr (CACHED) {
            apply_cached<NC, TX, TA>(crow[decltype(q)::value], (unsigned)row, X, n, col0, shift,
                                     y);
        } else {
            const RowCtx rc = row_ctx<KIND>(A, row);
            apply_cols<KIND, NC, TX, TA>(A, rc, X, n, col0, shift, y);
        }
    };

    GridSync gs;
    // A single workgroup produces and consumes every row on one CU: its own
    // stores, waited for, and a workgroup barrier are all it needs.
    const bool single = (G == 1);
    if (!single && !grid_setup(gs, P.bar, &sh.ok, G)) {
        finish(PHICOMB_EDEVICE, 0, 0, 0);
        return;
    }
    unsigned epoch = 0;
    // low rank: partial W^T X of a block this workgroup just wrote, for the
    // coming exchange (nlr values in all)
    int nlr = 0;
    // [2 parities][hi, lo][lrv][kMaxGrid]
    const size_t lr_lo = (size_t)P.lrv * kMaxGrid;
    auto lr_part = [&]() { return P.lrpart + (size_t)(epoch & 1) * 2 * lr_lo; };
    auto publish = [&](const auto *X, int ncols, int voff) __attribute__((always_inline)) {
        if constexpr (KIND == kLowRank) {
            lr_publish(A, n, lo, hi, X, ncols, voff, lr_part(), lr_lo, single ? 0u : bid);
            nlr = voff + ncols * A.rank;
        }
    };
    // publish this workgroup's maxima, cross the barrier, reduce all of them
    auto exchange = [&](auto &v) __attribute__((always_inline)) -> bool {
        constexpr int NV = std::extent<std::remove_reference_t<decltype(v)>>::value;
        if (single) {
            wait_own_stores();
            workgroup_max<NV, NT>(v, red);
            if constexpr (KIND == kLowRank)
                lr_gather(lr_part(), lr_lo, 1, nlr, sh.lrc);
            ++epoch;
            return true;
        }
        double *pt = P.part + (size_t)(epoch & 1) * kRedMax * kMaxGrid;
        store_partials<NV, NT>(v, pt, red, bid);
        if (!grid_sync(gs, &sh.ok))
            return false;
        load_partials<NV, NT>(pt, G, v, red);
        if constexpr (KIND == kLowRank)
            lr_gather(lr_part(), lr_lo, G, nlr, sh.lrc);
        ++epoch;
        return true;
    };

    // ---- S = D = V (I (x) 1^T mu/s), beta-prescaled; M_1 = I
    if (tid < R * kPMax1 * kPMax1) {
        const int i = tid / (kPMax1 * kPMax1), b = (tid / kPMax1) % kPMax1, c = tid % kPMax1;
        Mk[i][b][c] = (b == c) ? 1.0 : 0.0;
    }
    double nrm[2] = {0.0, 0.0};
    for_rows<RPT, EMEM, NT>(lo, hi, [&](int64_t row, auto) {
        double su = 0.0;
        for (int b = 0; b < P1; ++b) {
            const int pb = (b == 0) ? 0 : p + 1 - b;
            const double vv = P.V[row * P1 + pb];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const double u = vv * P.gam[i][b];
                const int64_t o = (int64_t)(b * R + i) * n + row;
                bU0[o] = u;
                bS[o] = u;
                su += fabs(u);
            }
        }
        nrm[0] = nmax(nrm[0], su);
    });
    publish(bU0, P.cS, 0);
    publish(bS, R, P.cS * A.rank);   // S_0: operand of the first recovery product
    nrm[1] = nrm[0];
    if (!exchange(nrm)) {
        finish(PHICOMB_EDEVICE, 0, 0, 0);
        return;
    }
    double c2 = nrm[0], nS = nrm[1];
    const double nS0 = nS;   // block norm of the first term (the series' start)
    // a non-finite entry of V (t and the weights are checked on the host)
    if (!(c2 <= 1.79769313486231570e308)) {
        finish(PHICOMB_EINVAL, 0, 0, 0);
        return;
    }

    // ---- S-series (rec.D) with the stopping test (stopTm) after every term
    int status = PHICOMB_OK;
    int k = 1;
    double c1 = INFINITY;
    int par = 0;   // the latest term lives in U0 (par = 0) or U1
    bool inS32 = false;   // the latest term is in Uf0/Uf1
    while (c1 + c2 > P.tol * nS) {
        if (k >= P.kcap) {
            status = PHICOMB_ENOCONV;
            break;
        }
        k = k + 1;
        // mixed precision: the same FP64-head / FP32-tail rule as in the
        // recovery steps, referenced to the smaller of the partial sum and
        // the first term
        const double nrefS = fmin(nS, nS0);
        const bool s32 = MIX && (inS32 || (k >= 3 && c2 * kMixSafety <= P.mix_tau * nrefS &&
                                           nrefS >= P.mix_lo && nS <= P.mix_hi));
        c1 = c2;
        const double rk = 1.0 / (double)k;
        // M_k = M_{k-1} J_step / k with J_step = a_i I + nu J  (J: ones on
        // (b, b+1) for 1 <= b < p); C = gam * M_k.
        {
            const bool act = tid < R * P1 * P1;
            int i = 0, b = 0, c = 0;
            double nv = 0.0;
            if (act) {
                i = tid / (P1 * P1);
                b = (tid / P1) % P1;
                c = tid % P1;
                nv = (Mk[i][b][c] * P.a[i] + (c >= 2 ? Mk[i][b][c - 1] * P.nu : 0.0)) * rk;
            }
            __syncthreads();
            if (act) {
                Mk[i][b][c] = nv;
                Cj[i][b][c] = P.gam[i][b] * nv;
            }
            __syncthreads();
        }
        const double *Uo = par ? bU1 : bU0;
        double *Un = par ? bU0 : bU1;
        const float *Uo32 = par ? P.Uf1 : P.Uf0;
        float *Un32 = par ? P.Uf0 : P.Uf1;
        double mx[2] = {0.0, 0.0};
        dense_pass(Uo, P.cS, P.xi);
        // one pass of the term, with the operand of type TX and the new term
        // stored as TS (mixed precision: FP32 tail); the precision is uniform
        // over the grid, so the branch stays outside the row loops
        auto s_pass = [&](auto tx, auto ts_) __attribute__((always_inline)) {
            using TX = typename decltype(tx)::type;
            using TS = typename decltype(ts_)::type;
            const TX *Uo_;
            TS *Un_;
            if constexpr (std::is_same<TX, float>::value)
                Uo_ = Uo32;
            else
                Uo_ = Uo;
            if constexpr (std::is_same<TS, float>::value)
                Un_ = Un32;
            else
                Un_ = Un;
            // the J-coupling of block b for abscissa i from the reordered v
            auto jterm = [&](int i, int b, const double *vr) -> double {
                if (b == 0)
                    return Cj[i][0][0] * vr[0];   // block 0 couples to itself only
                double jt = 0.0;
#pragma unroll
                for (int bb = 1; bb < kPMax1; ++bb)
                    if (bb <= b)
                        jt = fmadd(Cj[i][bb][b], vr[bb], jt);
                return jt;
            };
            if (pairs) {
                // columns two at a time (a runtime loop keeps the registers of
                // one chunk live, so that the wide 16-wave kernel fits)
                for_pairs<NT>(lo, hi, n, [&](int64_t i0, bool act) {
                    const PairCtx pc = pair_ctx(A, i0);
                    double su0 = 0.0, ss0 = 0.0, su1 = 0.0, ss1 = 0.0;
#pragma unroll 1
                    for (int c0 = 0; c0 < P.cS; c0 += 2) {
                        const int nc = (P.cS - c0 >= 2) ? 2 : 1;
                        TX y0[2], y1[2];
                        if (nc == 2) {
                            apply_pair<2, TX, TX>(A, pc, Uo_, n, c0, P.xi, y0, y1);
                        } else {
                            TX z0[1], z1[1];
                            apply_pair<1, TX, TX>(A, pc, Uo_, n, c0, P.xi, z0, z1);
                            y0[0] = z0[0];
                            y1[0] = z1[0];
                            y0[1] = y1[1] = (TX)0;
                        }
                        if (!act)
                            continue;
                        for (int cc = 0; cc < nc; ++cc) {
                            const int c = c0 + cc, b = c / R, i = c % R;
                            const int pb = (b == 0) ? 0 : p + 1 - b;
                            // J-coupling from the reordered v of both rows
                            double j0 = 0.0, j1 = 0.0;
                            if (b == 0) {
                                j0 = Cj[i][0][0] * P.V[i0 * P1];
                                j1 = Cj[i][0][0] * P.V[(i0 + 1) * P1];
                            } else {
                                for (int bb = 1; bb <= b; ++bb) {
                                    const int pbb = p + 1 - bb;
                                    j0 = fmadd(Cj[i][bb][b], P.V[i0 * P1 + pbb], j0);
                                    j1 = fmadd(Cj[i][bb][b], P.V[(i0 + 1) * P1 + pbb], j1);
                                }
                            }
                            (void)pb;
                            double u0 = fmadd((double)y0[cc] * P.ts[i], rk, j0);
                            double u1 = fmadd((double)y1[cc] * P.ts[i], rk, j1);
                            const int64_t o = (int64_t)c * n + i0;
                            typename Vec2<TS>::type uv = {(TS)u0, (TS)u1};
                            *(typename Vec2<TS>::type *)(Un_ + o) = uv;
                            u0 = (double)uv.x;
                            u1 = (double)uv.y;
                            auto sv = ld_pair(bS + (int64_t)c * n, (unsigned)i0);
                            sv.x += u0;
                            sv.y += u1;
                            *(typename Vec2<double>::type *)(bS + o) = sv;
                            su0 += fabs(u0);
                            su1 += fabs(u1);
                            ss0 += fabs(sv.x);
                            ss1 += fabs(sv.y);
                        }
                    }
                    if (act) {
                        mx[0] = nmax(mx[0], nmax(su0, su1));
                        mx[1] = nmax(mx[1], nmax(ss0, ss1));
                    }
                });
                return;
            }
            if constexpr (!PAIRS_ONLY) {
            for_rows<RPT, EMEM, NT>(lo, hi, [&](int64_t row, auto q) {
                double vr[kPMax1];   // reordered v: vr[b] = v_perm(b)(row)
#pragma unroll
                for (int b = 0; b < kPMax1; ++b)
                    vr[b] = (b < P1) ? P.V[row * P1 + ((b == 0) ? 0 : p + 1 - b)] : 0.0;
                double su = 0.0, ss = 0.0;
#pragma unroll 1
                for (int b = 0; b < P1; ++b) {
                    TX y[R];
                    opr(row, q, Uo_, b * R, P.xi, y);
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        double u = fmadd((double)y[i] * P.ts[i], rk, jterm(i, b, vr));
                        const int64_t o = (int64_t)(b * R + i) * n + row;
                        const TS us = (TS)u;
                        Un_[o] = us;
                        u = (double)us;
                        const double sn = bS[o] + u;
                        bS[o] = sn;
                        su += fabs(u);
                        ss += fabs(sn);
                    }
                }
                mx[0] = nmax(mx[0], su);
                mx[1] = nmax(mx[1], ss);
            });
            }
        };
        if constexpr (MIX) {
            if (inS32)
                s_pass(TypeTag<float>{}, TypeTag<float>{});
            else if (s32)
                s_pass(TypeTag<double>{}, TypeTag<float>{});
            else
                s_pass(TypeTag<double>{}, TypeTag<double>{});
        } else {
            s_pass(TypeTag<double>{}, TypeTag<double>{});
        }
        if (MIX && s32)
            publish(Un32, P.cS, 0);
        else
            publish(Un, P.cS, 0);
        publish(bS, R, P.cS * A.rank);
        if (!exchange(mx)) {
            finish(PHICOMB_EDEVICE, k, 0, 0);
            return;
        }
        c2 = mx[0];
        nS = mx[1];
        par ^= 1;
        inS32 = s32;
        n32S += s32 ? 1 : 0;
    }
    if (!(c2 == c2) || !(nS == nS))
        status = PHICOMB_EDEVICE;
    const int terms_S = k;
    if (status != PHICOMB_OK) {
        finish(status, terms_S, 0, 0);
        return;
    }

    // ---- F = [S_0, S_p];  F_1 <- A F_1 T + beta_0 v_0  (recovers exp(t_i A/s) v_0)
    const bool one_step = (P.s_int == 1);
    double nF = 0.0;
    {
        double mx[1] = {0.0};
        dense_pass(bS, R, 0.0);
        lr_off = P.cS;
        for_rows<RPT, EMEM, NT>(lo, hi, [&](int64_t row, auto q) {
            double y[R];
            opr(row, q, bS, 0, 0.0, y);
            const double v0 = P.V[row * P1];
            double f1[R], f2[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                f1[i] = y[i] * P.t[i] + P.w0[i] * v0;
                f2[i] = (p >= 1) ? bS[(int64_t)(p * R + i) * n + row] : 0.0;
            }
            if (one_step) {
#pragma unroll
                for (int i = 0; i < R; ++i)
                    P.W[row * R + i] = f1[i] + f2[i];
            } else {
                double sf = 0.0;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    bU0[(int64_t)i * n + row] = f1[i];
                    Eref(row, q, i) = f1[i];
                    sf += fabs(f1[i]);
                }
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    bU0[(int64_t)(R + i) * n + row] = f2[i];
                    Eref(row, q, R + i) = f2[i];
                    sf += fabs(f2[i]);
                }
                mx[0] = nmax(mx[0], sf);
            }
        });
        if (one_step) {
            finish(PHICOMB_OK, terms_S, 0, 0);
            return;
        }
        lr_off = 0;
        publish(bU0, 2 * R, 0);
        if (!exchange(mx)) {
            finish(PHICOMB_EDEVICE, terms_S, 0, 0);
            return;
        }
        nF = mx[0];
    }

    // ---- recovery (rec.F.shift): s-1 steps of exp(t(A - xi I)/s), each ended by
    //      E <- E mu, F_2 <- E_2 + (S exp(jJ/s))_p, F_1 <- E_1
    int tot = 0, maxstep = 0;
    par = 0;   // current F in U0
    for (int j = 1; j <= P.s_int - 1; ++j) {
        int kk = 0;
        double d1 = INFINITY, d2 = nF, nE = nF;
        const double nF0 = nF;
        bool in32 = false;   // the latest term is in Uf0/Uf1 (every step starts in FP64)
        while (d1 + d2 > P.tol * nE) {
            if (kk >= P.kcap) {
                status = PHICOMB_ENOCONV;
                break;
            }
            kk = kk + 1;
            const double nref = fmin(nE, nF0);
            const bool t32 =
                MIX && (in32 || (kk >= 2 && d2 * kMixSafety <= P.mix_tau * nref &&
                                 nref >= P.mix_lo && nE <= P.mix_hi));
            d1 = d2;
            const double rk = 1.0 / (double)kk;
            const double *Fo = par ? bU1 : bU0;
            double *Fn = par ? bU0 : bU1;
            const float *Fo32 = par ? P.Uf1 : P.Uf0;
            float *Fn32 = par ? P.Uf0 : P.Uf1;
            double mx[2] = {0.0, 0.0};
            dense_pass(Fo, 2 * R, P.xi);
            // one Taylor term with the operand of type TX and the new term
            // stored as TS; FP32 operands are multiplied in FP32
            auto r_pass = [&](auto tx, auto ts_) __attribute__((always_inline)) {
                using TX = typename decltype(tx)::type;
                using TS = typename decltype(ts_)::type;
                const TX *Fo_;
                TS *Fn_;
                if constexpr (std::is_same<TX, float>::value)
                    Fo_ = Fo32;
                else
                    Fo_ = Fo;
                if constexpr (std::is_same<TS, float>::value)
                    Fn_ = Fn32;
                else
                    Fn_ = Fn;
                // the new term's entry from the product y of the operand
                auto term = [&](TX y, int c) -> double {
                    if constexpr (std::is_same<TX, float>::value)
                        return (double)((y * (float)P.ts[c % R]) * (float)rk);
                    else
                        return (double)(TS)(((double)y * P.ts[c % R]) * rk);
                };
                if (pairs) {
                    // columns two at a time (2r is even), as in the S-series
                    for_pairs<NT>(lo, hi, n, [&](int64_t i0, bool act) {
                        const PairCtx pc = pair_ctx(A, i0);
                        double sf0 = 0.0, sf1 = 0.0, se0 = 0.0, se1 = 0.0;
#pragma unroll 1
                        for (int c0 = 0; c0 < 2 * R; c0 += 2) {
                            TX y0[2], y1[2];
                            apply_pair<2, TX, TX>(A, pc, Fo_, n, c0, P.xi, y0, y1);
                            if (!act)
                                continue;
#pragma unroll
                            for (int cc = 0; cc < 2; ++cc) {
                                const int c = c0 + cc;
                                const double f0 = term(y0[cc], c), f1 = term(y1[cc], c);
                                const int64_t o = (int64_t)c * n + i0;
                                typename Vec2<TS>::type fv = {(TS)f0, (TS)f1};
                                *(typename Vec2<TS>::type *)(Fn_ + o) = fv;
                                auto ev = ld_pair(bE + (int64_t)c * n, (unsigned)i0);
                                ev.x += f0;
                                ev.y += f1;
                                *(typename Vec2<double>::type *)(bE + o) = ev;
                                sf0 += fabs(f0);
                                sf1 += fabs(f1);
                                se0 += fabs(ev.x);
                                se1 += fabs(ev.y);
                            }
                        }
                        if (act) {
                            mx[0] = nmax(mx[0], nmax(sf0, sf1));
                            mx[1] = nmax(mx[1], nmax(se0, se1));
                        }
                    });
                    return;
                }
                if constexpr (!PAIRS_ONLY) {
                for_rows<RPT, EMEM, NT>(lo, hi, [&](int64_t row, auto q) {
                    TX y[2 * R];
                    opr(row, q, Fo_, 0, P.xi, y);
                    double sf = 0.0, se = 0.0;
#pragma unroll
                    for (int c = 0; c < 2 * R; ++c) {
                        const double f = term(y[c], c);
                        Fn_[(int64_t)c * n + row] = (TS)f;
                        double &e = Eref(row, q, c);
                        e = e + f;
                        sf += fabs(f);
                        se += fabs(e);
                    }
                    mx[0] = nmax(mx[0], sf);
                    mx[1] = nmax(mx[1], se);
                });
                }
            };
            if constexpr (MIX) {
                if (in32)
                    r_pass(TypeTag<float>{}, TypeTag<float>{});
                else if (t32)
                    r_pass(TypeTag<double>{}, TypeTag<float>{});
                else
                    r_pass(TypeTag<double>{}, TypeTag<double>{});
            } else {
                r_pass(TypeTag<double>{}, TypeTag<double>{});
            }
            if (MIX && t32)
                publish(Fn32, 2 * R, 0);
            else
                publish(Fn, 2 * R, 0);
            if (!exchange(mx)) {
                finish(PHICOMB_EDEVICE, terms_S, tot + kk, maxstep);
                return;
            }
            d2 = mx[0];
            nE = mx[1];
            par ^= 1;
            in32 = t32;
            n32 += t32 ? 1 : 0;
        }
        if (!(d2 == d2) || !(nE == nE))
            status = PHICOMB_EDEVICE;
        tot += kk;
        maxstep = std::max(maxstep, kk);
        if (status != PHICOMB_OK) {
            finish(status, terms_S, tot, maxstep);
            return;
        }
        // (exp(jJ/s))_{b,p} = (j/s)^(p-b)/(p-b)!, b >= 1
        double cd[kPMax1];
        cd[0] = 1.0;
#pragma unroll
        for (int d = 1; d < kPMax1; ++d)
            cd[d] = cd[d - 1] * ((double)j * P.nu) / (double)d;
        const bool last = (j == P.s_int - 1);
        double *Fx = par ? bU1 : bU0;   // overwrite the latest term: only E is needed
        double mx[1] = {0.0};
        for_rows<RPT, EMEM, NT>(lo, hi, [&](int64_t row, auto q) {
            double f1[R], f2[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                f1[i] = Eref(row, q, i) * P.mu[i];
                double acc = Eref(row, q, R + i) * P.mu[i];
                for (int b = 1; b <= p; ++b)
                    acc += bS[(int64_t)(b * R + i) * n + row] * cd[p - b];
                f2[i] = acc;
            }
            if (last) {
#pragma unroll
                for (int i = 0; i < R; ++i)
                    P.W[row * R + i] = f1[i] + f2[i];
            } else {
                double sf = 0.0;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    Fx[(int64_t)i * n + row] = f1[i];
                    Eref(row, q, i) = f1[i];
                    sf += fabs(f1[i]);
                }
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    Fx[(int64_t)(R + i) * n + row] = f2[i];
                    Eref(row, q, R + i) = f2[i];
                    sf += fabs(f2[i]);
                }
                mx[0] = nmax(mx[0], sf);
            }
        });
        if (last)
            break;
        publish(Fx, 2 * R, 0);
        if (!exchange(mx)) {
            finish(PHICOMB_EDEVICE, terms_S, tot, maxstep);
            return;
        }
        nF = mx[0];
    }
    finish(status, terms_S, tot, maxstep);
}

// ------------------------------------------------------------ single solve
template <int KIND, int R, int RPT, bool EMEM, bool MIX, int NT = kNT>
__global__ __launch_bounds__(NT) void solve_kernel(SolveArgs P) {
    __shared__ SolveShared sh;
    solve_body<KIND, R, RPT, EMEM, MIX, NT>(P, sh, gridDim.x, blockIdx.x,
                                            xcd_logical_block(blockIdx.x, gridDim.x));
}

// A small dense operator on one workgroup, A in registers and the term
// blocks in LDS (dynamic shared memory of dense_lds_bytes).  The caller's blocks in global
// memory are not used; V is read and W written as in the other variants.
template <int R>
__global__ __launch_bounds__(kNT) void solve_kernel_dense_lds(SolveArgs P) {
    __shared__ SolveShared sh;
    solve_body<kDenseLds, R, 1, true, false, kNT>(P, sh, 1u, 0u, 0);
}

__host__ __device__ constexpr size_t dense_lds_bytes(int64_t n, int64_t cS, int64_t cR) {
    return sizeof(double) * (size_t)(n * (cS + 2 * (cS > cR ? cS : cR) + cR));
}

using KernelFn = void (*)(SolveArgs);

// Instantiated variants: rows per thread 1..8 (register-cached CSR rows:
// 1..4); larger counts spill and are served by the E-in-memory variant.
// Mixed-precision variants exist for E in registers with 1..4 rows per
// thread and for E in memory; other shapes run the FP64 kernel.
template <int KIND, int R>
KernelFn pick_rpt(int rpt, bool emem, bool mix) {
    if constexpr (KIND != kCsrCached) {
        if (emem)
            return mix ? solve_kernel<KIND, R, 1, true, true> : solve_kernel<KIND, R, 1, true, false>;
    }
    switch (rpt) {
    case 1: return mix ? solve_kernel<KIND, R, 1, false, true> : solve_kernel<KIND, R, 1, false, false>;
    case 2: return mix ? solve_kernel<KIND, R, 2, false, true> : solve_kernel<KIND, R, 2, false, false>;
    case 4: return mix ? solve_kernel<KIND, R, 4, false, true> : solve_kernel<KIND, R, 4, false, false>;
    case 8:
        if constexpr (KIND != kCsrCached)
            return mix ? nullptr : solve_kernel<KIND, R, 8, false, false>;
        return nullptr;
    default: return nullptr;
    }
}

template <int KIND>
KernelFn pick_r(int r, int rpt, bool emem, bool mix) {
    switch (r) {
    case 1: return pick_rpt<KIND, 1>(rpt, emem, mix);
    case 2: return pick_rpt<KIND, 2>(rpt, emem, mix);
    case 3: return pick_rpt<KIND, 3>(rpt, emem, mix);
    case 4: return pick_rpt<KIND, 4>(rpt, emem, mix);
    default: return nullptr;
    }
}

// Variants per operator kind, each instantiated in a translation unit of its
// own so that they compile in parallel (solve_<kind>.hip).
KernelFn pick_lowrank(int r, int rpt, bool emem, bool mix);
KernelFn pick_stencil(int r, int rpt, bool emem, bool mix);
// E in memory, 1024 threads (16 waves) per workgroup, row pairs only: stencil
// operators with an even grid line and r <= 2 (nullptr otherwise)
KernelFn pick_stencil_wide(int r, bool mix);
KernelFn pick_csr(int r, int rpt, bool emem, bool mix);
KernelFn pick_csr_cached(int r, int rpt, bool mix);   // E in registers only
KernelFn pick_dense(int r);                            // E in memory, FP64
KernelFn pick_dense_lds(int r);                        // n <= kDenseLdsN, all in LDS, FP64

// ---------------------------------------------------------------- host side
// (implemented in solve.hip)
size_t solve_sync_bytes();
// Fills every field of a for one solve; the workspace ws (solve_workspace_bytes
// for this shape and precision) receives the sync area and the work blocks.
// Returns PHICOMB_OK, or PHICOMB_EINVAL when ceil(s max|t|) exceeds INT_MAX or
// the workspace is too small.
int build_solve_args(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                     const double *beta, const void *V, double tol, int precision, void *W,
                     void *ws, size_t ws_bytes, SolveArgs &a);
// Launches one solve on stream within `slots` workgroup slots that the
// caller already holds from the ledger (kept until the kernel has completed)
// and returns without waiting: *info_dev points at the kernel's status and
// term counts (status, terms_S, terms_rec, max_terms_step, fp32_terms), valid
// once the kernel has run and until the next launch on this workspace.
int solve_launch_held(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                      const double *beta, const void *V, double tol, int precision, void *W,
                      hipStream_t stream, void *ws, size_t ws_bytes, int slots,
                      const int **info_dev, int *s_int);
// Algorithmic bytes of a finished solve (info as written by the kernel).
double solve_algorithmic_bytes(phicomb_op op, int p, int r, int s_int, const int *info);

}  // namespace phc
