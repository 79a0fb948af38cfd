// Conditioning a realisation on observations by kriging its residuals (the paper names
// conditioning on data as future work, Sec. 6):
//   alpha = (C(X, X) + nugget sigma^2 I)^-1 (d - Y(X)),   Y_c(x) = Y(x) + sum_i alpha_i C(x - x_i),
// with the model covariance C(dx) = sigma^2 rho(|M^T dx|), M = R diag(1/ell) (the same
// anisotropy as the field's wavevectors k = M z; App. A correlations).
//
// The M x M system is factorised in FP64 by a right-looking blocked Cholesky with 64-wide
// panels, one launch per panel: the panel's rows are solved against the stored inverse of its
// diagonal factor and the trailing matrix updated on the FP64 matrix cores, the forward
// substitution rides along as an extra row, and the workgroup that updates the next diagonal
// block factors and inverts it.  The backward substitution takes one launch per block (the
// block solve is a product with the stored inverse).  The correction is summed in FP32 with
// observation chunks staged in LDS.
#include <hip/hip_runtime.h>

#include <cmath>

#include "grf_internal.h"

namespace grf {

namespace {

constexpr int kB = 64;        // Cholesky block and panel width
constexpr int kLd = kB + 2;   // LDS row stride in doubles: matrix-core operand reads hit distinct banks

// rho(r^2) of the standardised covariance (App. A): Gaussian exp(-r^2), exponential exp(-r),
// Matern 3/2 (1 + sqrt3 r) exp(-sqrt3 r), Matern 5/2 (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r).
template <class T>
__device__ __forceinline__ T corr_r2(int kind, T r2)
{
    if (kind == KR_GAUSS) return exp(-r2);
    const T r = sqrt(r2);
    if (kind == KR_EXP) return exp(-r);
    if (kind == KR_M32) {
        const T a = T(1.7320508075688772935) * r;
        return (T(1) + a) * exp(-a);
    }
    const T a = T(2.2360679774997896964) * r;
    return (T(1) + a + a * a * T(1.0 / 3.0)) * exp(-a);
}

// The correction sum works on lags scaled by kappa, chosen so that the base-2 exponential takes
// the scaled distance as it is: Gaussian exp(-r^2) = 2^-(kappa r)^2 with kappa^2 = log2(e);
// exponential exp(-r) = 2^-(kappa r) with kappa = log2(e); Matern nu = 3/2, 5/2:
// exp(-c r) = 2^-(kappa r) with kappa = c log2(e), c = sqrt3, sqrt5, and c r = (kappa r) ln 2.
__device__ __forceinline__ double lag_scale(int kind)
{
    constexpr double kLog2e = 1.4426950408889634074;
    if (kind == KR_GAUSS) return 1.2011224087864498;  // sqrt(log2(e))
    if (kind == KR_EXP) return kLog2e;
    if (kind == KR_M32) return 1.7320508075688772935 * kLog2e;
    return 2.2360679774997896964 * kLog2e;
}

// FP32 correlation of the scaled squared lag q = (kappa r)^2, on the hardware square root and
// base-2 exponential (about 1 ulp each; the sum is FP32 anyway).
template <int KIND>
__device__ __forceinline__ float corr_scaled(float q)
{
    if constexpr (KIND == KR_GAUSS) return __builtin_amdgcn_exp2f(-q);
    const float s = __builtin_amdgcn_sqrtf(q);
    const float e = __builtin_amdgcn_exp2f(-s);
    if constexpr (KIND == KR_EXP) return e;
    const float a = s * 0.69314718f;  // c r
    if constexpr (KIND == KR_M32) return fmaf(a, e, e);
    return fmaf(fmaf(a, 1.f / 3.f, 1.f), a, 1.f) * e;
}

// Standardised lag u = M^T dx (M^T given row-major 3 x 3 in `mt`).
template <class T>
__device__ __forceinline__ T lag_r2(const KrigeModel& km, T d0, T d1, T d2)
{
    const T u0 = T(km.mt[0]) * d0 + T(km.mt[1]) * d1 + T(km.mt[2]) * d2;
    const T u1 = T(km.mt[3]) * d0 + T(km.mt[4]) * d1 + T(km.mt[5]) * d2;
    const T u2 = T(km.mt[6]) * d0 + T(km.mt[7]) * d1 + T(km.mt[8]) * d2;
    return u0 * u0 + u1 * u1 + u2 * u2;
}

// C[i][j] (lower triangle and diagonal; row-major, leading dimension lda).
__global__ __launch_bounds__(256) void k_cov_matrix(const double* __restrict__ x, int64_t m, int dim, KrigeModel km,
                                                   double* __restrict__ C, int64_t lda)
{
    const int64_t i = static_cast<int64_t>(blockIdx.y) * 16 + (threadIdx.x >> 4);
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 16 + (threadIdx.x & 15);
    if (i >= m || j >= m || j > i) return;
    const double* xi = x + i * dim;
    const double* xj = x + j * dim;
    const double d0 = xi[0] - xj[0], d1 = xi[1] - xj[1], d2 = dim == 3 ? xi[2] - xj[2] : 0.0;
    double c = km.s2 * corr_r2<double>(km.kind, lag_r2<double>(km, d0, d1, d2));
    if (i == j) c += km.nugget_abs;
    C[i * lda + j] = c;
}

// Value of lane `src` (wave-uniform) of a double, broadcast through scalar registers.
__device__ __forceinline__ double lane_bcast(double v, int src)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffu), src));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), src));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// One FP64 matrix-core step D = A B + C on 16 x 16 x 4: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 e + l / 16][l % 16] in element e (the FP64 form interleaves
// its output rows across the four lane groups, unlike the 16-bit forms).
__device__ __forceinline__ v4d mfma64(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

using Blk = double[kB][kLd];

// acc += s X Y^T over the 64 columns of the LDS blocks X and Y (s = -1 when `neg`), for the
// 32 x 32 quadrant of the 64 x 64 product that wave w owns (rows 32 (w / 2), columns 32 (w % 2)),
// as 2 x 2 tiles of 16 x 16.
__device__ __forceinline__ void gemm_nt(const Blk& X, const Blk& Y, v4d (&acc)[2][2], bool neg)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int rb = 32 * (w >> 1), cb = 32 * (w & 1);
#pragma unroll 4
    for (int k = 0; k < kB; k += 4) {
        double a0 = X[rb + r][k + q], a1 = X[rb + 16 + r][k + q];
        const double b0 = Y[cb + r][k + q], b1 = Y[cb + 16 + r][k + q];
        if (neg) {
            a0 = -a0;
            a1 = -a1;
        }
        acc[0][0] = mfma64(a0, b0, acc[0][0]);
        acc[0][1] = mfma64(a0, b1, acc[0][1]);
        acc[1][0] = mfma64(a1, b0, acc[1][0]);
        acc[1][1] = mfma64(a1, b1, acc[1][1]);
    }
}

// P = X D^T for the LDS block X and the lower-triangular LDS block D (zero above its diagonal):
// wave w makes the 16-row strip 16 w of P, column tile bj in acc[bj], whose sum over k stops at
// D's diagonal (k < 16 (bj + 1)), so every wave takes 40 of the 64 products of a full strip.
__device__ __forceinline__ void gemm_lower(const Blk& X, const Blk& D, v4d (&acc)[4])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4, rb = 16 * w;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kB; k += 4) {
        const double a = X[rb + r][k + q];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
            if (k < 16 * (bj + 1)) acc[bj] = mfma64(a, D[16 * bj + r][k + q], acc[bj]);
    }
}

// The strip layout of gemm_lower into LDS.
__device__ __forceinline__ void strip_to_lds(const v4d (&acc)[4], Blk& S)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int e = 0; e < 4; ++e) S[16 * w + 4 * e + q][16 * bj + r] = acc[bj][e];
}

// Row and column, within the 64 x 64 block, of element e of accumulator tile (bi, bj).
__device__ __forceinline__ int acc_row(int bi, int e)
{
    return 32 * (static_cast<int>(threadIdx.x) >> 7) + 16 * bi + 4 * e + ((threadIdx.x & 63) >> 4);
}
__device__ __forceinline__ int acc_col(int bj)
{
    return 32 * ((threadIdx.x >> 6) & 1) + 16 * bj + (threadIdx.x & 15);
}

// A 64 x 64 block moves between global memory and LDS in two halves: every thread first loads
// its sixteen entries (rows t / 64 + 4 i, column t % 64; each wave reads whole 512-byte rows)
// into registers, with all loads in flight together, and stores them to LDS afterwards.
using Rows = double[16];

// v = A[r0 + r][c0 + c] for rows r0 + r < rows (else 0).
__device__ __forceinline__ void fetch_rows(Rows& v, const double* __restrict__ A, int64_t lda, int64_t r0, int64_t c0,
                                           int64_t rows)
{
    const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t gr = r0 + rb + 4 * i;
        v[i] = gr < rows ? A[gr * lda + c0 + c] : 0.0;
    }
}

// v = D[r][c] of a dense 64 x 64 row-major block.
__device__ __forceinline__ void fetch_dense(Rows& v, const double* __restrict__ D)
{
    const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = D[(rb + 4 * i) * kB + c];
}

__device__ __forceinline__ void store_rows(Blk& S, const Rows& v)
{
    const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 16; ++i) S[rb + 4 * i][c] = v[i];
}

// 1 / sqrt(d): the hardware estimate refined by two Newton steps, y += y (1/2 - d y^2 / 2), to about
// an ulp.  A pivot d <= 0 or NaN gives NaN (the estimate is NaN below zero and infinite at zero,
// where the first step makes 0 * inf).
__device__ __forceinline__ double rsqrt_nan(double d)
{
    double y = __builtin_amdgcn_rsq(d);
    const double h = 0.5 * d;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// Columns [j0, j0 + 16) of the diagonal block in S, factored by one wave in registers (lane r
// holds row r's 16 entries).  Software-pipelined over the columns: column j's pivot reciprocal
// is made in the previous step, in the pivot's own lane; the entries of column j that the next
// two columns need come by lane broadcasts, the rest through LDS, read one step early and
// applied in the next step (in the shadow of the next pivot's chain).  Entries above the diagonal (c > r in lane r) take part
// in the arithmetic and end up holding values that are never read.  Updated entries are pinned:
// otherwise the compiler defers every update to the entry's first use, lengthening the pivot
// chain.  The pivot reciprocals go to rdiag[j0 ..].
__device__ __forceinline__ void factor_subpanel(Blk& S, int j0, double* __restrict__ rdiag, double* colb)
{
    const int t = threadIdx.x;
    double pv[16], cb[16], isv[16], lprev = 0.0;
    // a zero the compiler cannot see through, so that the broadcast reads below use one base
    // register with immediate offsets instead of materialising every address
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    const double* cbase = colb + zero;
#pragma unroll
    for (int c = 0; c < 16; ++c) pv[c] = S[t][j0 + c];
    double is = rsqrt_nan(lane_bcast(pv[0], j0));
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double lj = pv[j] * is;  // the pivot's own lane: d / sqrt(d)
        pv[j] = lj;
        isv[j] = is;
        // the next pivot, made in its own lane: its entry of this column is its own lj
        if (j + 1 < 16) is = rsqrt_nan(lane_bcast(fma(-lj, lj, pv[j + 1]), j0 + j + 1));
#pragma unroll
        for (int c = j + 1; c < j + 3 && c < 16; ++c) {
            pv[c] -= lj * lane_bcast(lj, j0 + c);
            asm volatile("" : "+v"(pv[c]));
        }
        if (j >= 1 && j <= 13) {
#pragma unroll
            for (int c = j + 2; c < 16; ++c) {
                pv[c] -= lprev * cb[c];
                asm volatile("" : "+v"(pv[c]));
            }
        }
        // the scheduler may overlap what follows with the next column's pivot chain, but moves
        // nothing of this column's chain below this point
        __builtin_amdgcn_sched_barrier(0);
        if (j + 3 < 16) {
            colb[t] = lj;
            // one wave, whose LDS accesses complete in program order: compiler barriers order
            // the store before the reads and the reads before the next column's store
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = j + 3; c < 16; ++c) cb[c] = cbase[j0 + c];
            __builtin_amdgcn_wave_barrier();
            lprev = lj;
        }
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) S[t][j0 + c] = pv[c];
    if (t == 0) {
#pragma unroll
        for (int j = 0; j < 16; ++j) rdiag[j0 + j] = isv[j];
    }
}

// S[r0 ..][c0 ..] (a 16 x 16 tile) -= L[r0 ..][j0 ..] L[c0 ..][j0 ..]^T over the 16 columns of
// the sub-panel at j0, by one wave on the matrix cores.
__device__ __forceinline__ void trail_tile(Blk& S, int j0, int r0, int c0)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    v4d acc;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] = S[r0 + 4 * e + q][c0 + r];
#pragma unroll
    for (int k = 0; k < 16; k += 4) acc = mfma64(-S[r0 + r][j0 + k + q], S[c0 + r][j0 + k + q], acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) S[r0 + 4 * e + q][c0 + r] = acc[e];
}

// Inverse of the 16 x 16 diagonal factor at o = 16 b (one wave): lane c (of each group of 16;
// the first group stores) makes column c by forward substitution, row by row.
__device__ __forceinline__ void leaf_inverse(const Blk& S, Blk& T, const double* __restrict__ rdiag, int o,
                                             double* __restrict__ dout)
{
    const int lane = threadIdx.x & 63, c = lane & 15;
    double x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        double a0 = j == c ? 1.0 : 0.0, a1 = 0.0;
#pragma unroll
        for (int l = 0; l < j; l += 2) {
            a0 -= S[o + j][o + l] * x[l];
            if (l + 1 < j) a1 -= S[o + j][o + l + 1] * x[l + 1];
        }
        x[j] = (a0 + a1) * rdiag[o + j];
        if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    if (lane < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            T[o + j][o + c] = x[j];
            dout[(o + j) * kB + o + c] = x[j];
        }
    }
}

// Lower-left 16 x 16 block of the inverse of the 32 x 32 half at o (one wave), from the
// diagonal blocks' inverses A^-1 (at o) and C^-1 (at o + 16) and the factor's block B:
// -C^-1 (B A^-1), with B A^-1 staged in S's unused upper triangle.  Two accumulators halve the
// dependent chain of products.
__device__ __forceinline__ void half_inverse(Blk& S, Blk& T, int o, double* __restrict__ dout)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0;
    a0 = mfma64(S[o + 16 + r][o + q], T[o + q][o + r], a0);
    a1 = mfma64(S[o + 16 + r][o + 8 + q], T[o + 8 + q][o + r], a1);
    a0 = mfma64(S[o + 16 + r][o + 4 + q], T[o + 4 + q][o + r], a0);
    a1 = mfma64(S[o + 16 + r][o + 12 + q], T[o + 12 + q][o + r], a1);
#pragma unroll
    for (int e = 0; e < 4; ++e) S[o + 4 * e + q][o + 16 + r] = a0[e] + a1[e];
    __builtin_amdgcn_wave_barrier();
    a0 = v4d{0.0, 0.0, 0.0, 0.0};
    a1 = a0;
    a0 = mfma64(T[o + 16 + r][o + 16 + q], S[o + q][o + 16 + r], a0);
    a1 = mfma64(T[o + 16 + r][o + 24 + q], S[o + 8 + q][o + 16 + r], a1);
    a0 = mfma64(T[o + 16 + r][o + 20 + q], S[o + 4 + q][o + 16 + r], a0);
    a1 = mfma64(T[o + 16 + r][o + 28 + q], S[o + 12 + q][o + 16 + r], a1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double v = -(a0[e] + a1[e]);
        T[o + 16 + 4 * e + q][o + r] = v;
        dout[(o + 16 + 4 * e + q) * kB + o + r] = v;
    }
}

// Factor and invert one diagonal block.  On entry S holds the block's lower triangle (rows and
// columns from nb on padded with the identity); on exit S's lower triangle holds the factor L
// (its upper triangle holds values that are never read) and `dout` the inverse L^-1 (64 x 64
// row-major, zeros above the diagonal).  The first non-positive pivot, counted 1-based from the
// matrix's first row via g0, goes to `info` if none was reported before.  T is LDS scratch.
//
// The factorisation runs in four 16-column sub-panels, each factored by wave 0 in registers and
// then applied to the trailing rows and columns (rank-16 updates) on the matrix cores.  Only the
// tiles of the next sub-panel's columns are updated before wave 0 moves on; the other waves
// apply the rest, invert the finished 16 x 16 diagonal factors and form the first-level
// off-diagonal blocks of the inverse while wave 0 factors the next sub-panel.  The inverse
// follows from inv([[A, 0], [B, C]]) = [[A^-1, 0], [-C^-1 B A^-1, C^-1]], within each 32 x 32
// half and then for the whole block.
__device__ __forceinline__ void factor_invert(Blk& S, Blk& T, int nb, int64_t g0, double* __restrict__ dout,
                                              int32_t* __restrict__ info)
{
    __shared__ double rdiag[kB];
    __shared__ double colb[kB];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, r = lane & 15, q = lane >> 4;
    // the inverse's zero blocks above its diagonal 16 x 16 blocks
    for (int e = t; e < kB * kB; e += blockDim.x) {
        const int rr = e >> 6, cc = e & 63;
        if ((cc >> 4) > (rr >> 4)) dout[e] = 0.0;
    }
    // the upper-right 16 x 16 block of each 32 x 32 half of the inverse, in T
    if (w == 3) {
#pragma unroll
        for (int j = 0; j < 16; j += 4) {
            T[j + q][16 + r] = 0.0;
            T[32 + j + q][48 + r] = 0.0;
        }
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const int j0 = 16 * sp;
        if (w == 0) {
            factor_subpanel(S, j0, rdiag, colb);
        } else {
            // work that the previous sub-panel left, in the shadow of this factorisation
            if (w == 1 && sp >= 1) leaf_inverse(S, T, rdiag, j0 - 16, dout);
            if (sp == 1) {
                // the previous update's tiles right of this sub-panel's columns
                if (w == 2) {
                    trail_tile(S, 0, 32, 32);
                    trail_tile(S, 0, 48, 48);
                }
                if (w == 3) trail_tile(S, 0, 48, 32);
            }
            if (sp == 2 && w == 2) trail_tile(S, 16, 48, 48);
            if (sp == 3 && w == 2) {
                half_inverse(S, T, 0, dout);
                __builtin_amdgcn_wave_barrier();
                // W = L21 L11^-1 (the first product of the whole block's off-diagonal block)
                // into T's free upper-right quadrant; L11^-1 is now complete
#pragma unroll
                for (int tile = 0; tile < 4; ++tile) {
                    const int wi = 16 * (tile >> 1), wj = 16 * (tile & 1);
                    v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
                    for (int k = 0; k < 32; k += 8) {
                        a0 = mfma64(S[32 + wi + r][k + q], T[k + q][wj + r], a0);
                        a1 = mfma64(S[32 + wi + r][k + 4 + q], T[k + 4 + q][wj + r], a1);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) T[wi + 4 * e + q][32 + wj + r] = a0[e] + a1[e];
                }
            }
        }
        __syncthreads();
        // the update of the next sub-panel's columns by this one
        if (w < 3 - sp) trail_tile(S, j0, j0 + 16 + 16 * w, j0 + 16);
        if (sp < 3) __syncthreads();
    }
    if (w == 0) {
        // a non-positive pivot leaves NaN on its diagonal and on every later one: the first
        // row of the block whose diagonal is not positive is the one to report
        const uint64_t badm = __ballot(t < nb && !(S[t][t] > 0.0));
        if (t == 0 && badm && info && *info == 0) *info = static_cast<int>(g0 + __builtin_ctzll(badm) + 1);
    }
    if (w == 1) {
        leaf_inverse(S, T, rdiag, 48, dout);
        __builtin_amdgcn_wave_barrier();
        half_inverse(S, T, 32, dout);
    }
    __syncthreads();
    // the whole block's lower-left quadrant of the inverse, -L22^-1 W (W made above)
    const int wi = 16 * (w >> 1), wj = 16 * (w & 1);
    v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        a0 = mfma64(T[32 + wi + r][32 + k + q], T[k + q][32 + wj + r], a0);
        a1 = mfma64(T[32 + wi + r][32 + k + 4 + q], T[k + 4 + q][32 + wj + r], a1);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) dout[(32 + wi + 4 * e + q) * kB + wj + r] = -(a0[e] + a1[e]);
}

// Lower triangle of the diagonal block of A at row/column g0 into S, padded with the identity
// past the matrix's last row.
__device__ __forceinline__ void stage_diag_block(Blk& S, const double* __restrict__ A, int64_t m, int64_t lda,
                                                 int64_t g0)
{
    const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
    Rows v;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = rb + 4 * i;
        v[i] = g0 + r < m ? (c <= r ? A[(g0 + r) * lda + g0 + c] : 0.0) : (c == r ? 1.0 : 0.0);
    }
    store_rows(S, v);
}

// First diagonal block: factor and invert (one workgroup).
__global__ __launch_bounds__(256) void k_chol_first(const double* __restrict__ A, int64_t m, int64_t lda,
                                                   double* __restrict__ dinv, int32_t* __restrict__ info)
{
    __shared__ Blk S, T;
    stage_diag_block(S, A, m, lda, 0);
    __syncthreads();
    factor_invert(S, T, static_cast<int>(min<int64_t>(kB, m)), 0, dinv, info);
}

// One panel step p of the right-looking blocked Cholesky factorisation A = L L^T, with the
// forward substitution L z = r carried along as an extra row.  Workgroup (a, b), b <= a, owns
// the trailing tile of row block i = p + 1 + a and column block j = p + 1 + b (workgroup 0 the
// next diagonal block, so that the step's longest chain starts first).  With the inverse
// D = L_pp^-1 of the panel's diagonal factor (made by the preceding step):
//   panel rows:   L_ip = A_ip D^T (and L_jp), on the matrix cores;
//   update:       A_ij -= L_ip L_jp^T (lower triangle on the diagonal);
//   column b = 0: stores L_ip transposed in A's unused upper triangle, U[k0 + n][i0 + r] =
//                 L_ip[r][n], the layout the backward substitution reads;
//   diagonal:     r_i -= L_ip z_p with z_p = D r_p (workgroup 0 also stores z_p);
//   workgroup 0:  factors and inverts the updated diagonal block p + 1.
// Every workgroup reads only panel p and its own tile, and writes its own tile, its own rows of
// r and of U: no two workgroups touch the same entry.
__global__ __launch_bounds__(256) void k_chol_step(double* __restrict__ A, int64_t m, int64_t lda, int64_t p,
                                                  double* __restrict__ dinv, double* __restrict__ r,
                                                  double* __restrict__ z, int32_t* __restrict__ info)
{
    __shared__ Blk X, Y, D;
    __shared__ double zp[kB], rp[kB];
    const int t = threadIdx.x;
    const int64_t k0 = p * kB;
    const int64_t tid = blockIdx.x;
    int64_t a = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(tid) + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > tid) --a;
    while ((a + 1) * (a + 2) / 2 <= tid) ++a;
    const int64_t b = tid - a * (a + 1) / 2;
    const int64_t i0 = (p + 1 + a) * kB, j0 = (p + 1 + b) * kB;
    const bool diag = a == b;

    Rows vd, vx, vy;
    const double rv = diag && t < kB ? r[k0 + t] : 0.0;
    fetch_dense(vd, dinv + p * kB * kB);
    fetch_rows(vx, A, lda, i0, k0, m);
    if (!diag) fetch_rows(vy, A, lda, j0, k0, m);
    v4d c[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gi = i0 + acc_row(bi, e), gj = j0 + acc_col(bj);
                c[bi][bj][e] = gi < m && gj <= gi ? A[gi * lda + gj] : 0.0;
            }
    store_rows(D, vd);
    store_rows(X, vx);
    if (!diag) store_rows(Y, vy);
    if (diag && t < kB) rp[t] = rv;
    __syncthreads();
    v4d pi[4], pj[4];
    gemm_lower(X, D, pi);
    if (!diag) gemm_lower(Y, D, pj);
    if (diag && t < kB) {
        // z_p = D r_p (D's zeros above the diagonal make the full-length sum exact)
        double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kB; ++k) v[k & 3] += D[t][k] * rp[k];
        zp[t] = (v[0] + v[1]) + (v[2] + v[3]);
    }
    __syncthreads();
    strip_to_lds(pi, X);
    if (!diag) strip_to_lds(pj, Y);
    __syncthreads();
    if (b == 0) {
        // U rows k0 + n, columns i0 .. i0 + 63: consecutive lanes take consecutive columns
        const int rr = t & 63;
        if (i0 + rr < m)
            for (int n = t >> 6; n < kB; n += 4) A[(k0 + n) * lda + i0 + rr] = X[rr][n];
    }
    if (diag && t < kB) {
        if (i0 + t < m) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int n = 0; n < kB; ++n) v[n & 3] += X[t][n] * zp[n];
            r[i0 + t] -= (v[0] + v[1]) + (v[2] + v[3]);
        }
        if (a == 0) z[k0 + t] = zp[t];
    }
    gemm_nt(X, diag ? X : Y, c, true);
    if (tid != 0) {
        // (the next diagonal block is factored below and never read from A again)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t gi = i0 + acc_row(bi, e), gj = j0 + acc_col(bj);
                    if (gi < m && gj <= gi) A[gi * lda + gj] = c[bi][bj][e];
                }
    }
    if (tid == 0) {
        // the next diagonal block, from the updated values still in registers
        const int nbn = static_cast<int>(min<int64_t>(kB, m - i0));
        __syncthreads();
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rr = acc_row(bi, e), cc = acc_col(bj);
                    double v = 0.0;
                    if (rr < nbn) {
                        if (cc <= rr) v = c[bi][bj][e];
                    } else if (cc == rr) {
                        v = 1.0;
                    }
                    D[rr][cc] = v;
                }
        __syncthreads();
        factor_invert(D, Y, nbn, i0, dinv + (p + 1) * kB * kB, info);
    }
}

// y_o = sum_k M[k][o] v_k (trans) or sum_k M[o][k] v_k over all 64 k (v is zero where M's block
// ends), for the 64 x 64 LDS block M: four lanes per output o = t / 4, each summing every fourth
// term, the partial sums meeting by lane exchanges; outputs from no on are 0.
__device__ __forceinline__ double matvec64(const Blk& M, const double* v, int no, bool trans)
{
    const int t = threadIdx.x, o = t >> 2, g = t & 3;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int k = 0; k < kB; k += 8) {
        a0 += (trans ? M[k + g][o] : M[o][k + g]) * v[k + g];
        a1 += (trans ? M[k + 4 + g][o] : M[o][k + 4 + g]) * v[k + 4 + g];
    }
    double acc = a0 + a1;
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    return o < no ? acc : 0.0;
}

// Backward substitution L^T x = z, two blocks per launch (from the last block to the first): for
// the upper block h and the lower block l = h - 1,
//   x_h = D_h^T z_h,   x_l = D_l^T (z_l - L_hl^T x_h),   z_q -= L_lq^T x_l + L_hq^T x_h (q < l),
// with D_b = L_bb^-1 and L below the diagonal read from U (row q0 + n of U holds column n of L
// below block q).  With `two` = 0 the launch takes block h alone.  For the last block z_h is
// made here from the forward-updated right-hand side, z_h = D_h r_h.  Every workgroup forms the
// blocks' solution itself (three 64 x 64 matrix-vector products) and updates 32 rows of z, whose
// U entries it loads first; workgroup 0 stores the solution.
__global__ __launch_bounds__(256) void k_chol_back(const double* __restrict__ A, int64_t m, int64_t lda, int64_t bh,
                                                  int two, const double* __restrict__ dinv,
                                                  const double* __restrict__ r, double* __restrict__ z,
                                                  double* __restrict__ x, int last)
{
    __shared__ Blk Dh, Dl, Uhl;
    __shared__ double zs[kB], xs[2 * kB];
    const int t = threadIdx.x;
    const int64_t h0 = bh * kB, l0 = two ? h0 - kB : h0;
    const int nh = static_cast<int>(min<int64_t>(kB, m - h0));
    // this workgroup's 32 rows of z: eight lanes per row, sixteen consecutive U entries per lane
    // over the columns of the launch's blocks (issued before anything waits)
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 32 + (t >> 3);
    const int q = 16 * (t & 7);
    const int ncols = two ? kB + nh : nh;
    double u[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) u[e] = i < l0 && q + e < ncols ? A[i * lda + l0 + q + e] : 0.0;
    Rows vh, vl, vu;
    fetch_dense(vh, dinv + bh * kB * kB);
    if (two) {
        fetch_dense(vl, dinv + (bh - 1) * kB * kB);
        // U rows of block l, columns of block h (zero past the matrix's last column)
        const int c = t & 63, rb = t >> 6;
#pragma unroll
        for (int e = 0; e < 16; ++e) vu[e] = c < nh ? A[(l0 + rb + 4 * e) * lda + h0 + c] : 0.0;
        store_rows(Dl, vl);
        store_rows(Uhl, vu);
    }
    store_rows(Dh, vh);
    if (t < kB) zs[t] = t < nh ? (last ? r[h0 + t] : z[h0 + t]) : 0.0;
    if (t < 2 * kB) xs[t] = 0.0;
    __syncthreads();
    if (last) {
        const double v = matvec64(Dh, zs, nh, false);
        __syncthreads();
        if ((t & 3) == 0) zs[t >> 2] = v;
        __syncthreads();
    }
    {
        const double v = matvec64(Dh, zs, nh, true);
        if ((t & 3) == 0) xs[(two ? kB : 0) + (t >> 2)] = v;
    }
    __syncthreads();
    if (two) {
        // z_l - L_hl^T x_h, then x_l
        const double v = matvec64(Uhl, xs + kB, kB, false);
        if ((t & 3) == 0) zs[t >> 2] = z[l0 + (t >> 2)] - v;
        __syncthreads();
        const double xl = matvec64(Dl, zs, kB, true);
        if ((t & 3) == 0) xs[t >> 2] = xl;
        __syncthreads();
    }
    if (blockIdx.x == 0 && t < ncols) x[l0 + t] = xs[t];
    double v = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) v += u[e] * xs[(q + e) & (2 * kB - 1)];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (i < l0 && (t & 7) == 0) z[i] -= v;
}

// r = d - y (FP64 residuals).
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ d, const float* __restrict__ y, int64_t m,
                                                 double* __restrict__ r)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) r[i] = static_cast<double>(d[i]) - static_cast<double>(y[i]);
}

// Observation staging for the correction: (u = kappa M^T (x_i - x_0) as FP32, w_i = sigma^2
// alpha_i); lags are taken from the first observation so that the FP32 differences stay small.
__global__ __launch_bounds__(256) void k_krige_stage(const double* __restrict__ x, const double* __restrict__ alpha,
                                                    int64_t m, int dim, KrigeModel km, float4* __restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double* xi = x + i * dim;
    const double d0 = xi[0] - x[0], d1 = xi[1] - x[1], d2 = dim == 3 ? xi[2] - x[2] : 0.0;
    const double ks = lag_scale(km.kind);
    const double u0 = ks * (km.mt[0] * d0 + km.mt[1] * d1 + km.mt[2] * d2);
    const double u1 = ks * (km.mt[3] * d0 + km.mt[4] * d1 + km.mt[5] * d2);
    const double u2 = ks * (km.mt[6] * d0 + km.mt[7] * d1 + km.mt[8] * d2);
    out[i] = make_float4(static_cast<float>(u0), static_cast<float>(u1), static_cast<float>(u2),
                         static_cast<float>(km.s2 * alpha[i]));
}

constexpr int kKc = 256;  // observations per LDS chunk
constexpr int kKr = 4;    // cells per lane (general form)
constexpr int kKx = 8;    // cells per lane along a grid row (row form)

// y[c] += sum_i w_i rho(|u(c) - u_i|) for cells of a grid (grid != nullptr) or points.
template <bool GRID, int KIND>
__global__ __launch_bounds__(256) void k_krige_apply(const float4* __restrict__ obs, const double* __restrict__ ref,
                                                    int64_t m, KrigeModel km, KrigeTarget tg, float* __restrict__ y)
{
    __shared__ float4 so[kKc];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (256 * kKr) + threadIdx.x;
    const double ks = lag_scale(KIND);
    float v0[kKr], v1[kKr], v2[kKr], acc[kKr];
#pragma unroll
    for (int r = 0; r < kKr; ++r) {
        const int64_t c = min(base + 256 * r, tg.count - 1);
        double x0, x1, x2 = 0.0;
        if constexpr (GRID) {
            const int64_t i = c % tg.n[0], q = c / tg.n[0];
            const int64_t j = q % tg.n[1], k = q / tg.n[1];
            x0 = tg.o[0] + (static_cast<double>(i) + 0.5) * tg.h[0];
            x1 = tg.o[1] + (static_cast<double>(j) + 0.5) * tg.h[1];
            if (tg.dim == 3) x2 = tg.o[2] + (static_cast<double>(k) + 0.5) * tg.h[2];
        } else {
            x0 = tg.xyz[c * tg.dim];
            x1 = tg.xyz[c * tg.dim + 1];
            if (tg.dim == 3) x2 = tg.xyz[c * tg.dim + 2];
        }
        const double d0 = x0 - ref[0], d1 = x1 - ref[1], d2 = tg.dim == 3 ? x2 - ref[2] : 0.0;
        v0[r] = static_cast<float>(ks * (km.mt[0] * d0 + km.mt[1] * d1 + km.mt[2] * d2));
        v1[r] = static_cast<float>(ks * (km.mt[3] * d0 + km.mt[4] * d1 + km.mt[5] * d2));
        v2[r] = static_cast<float>(ks * (km.mt[6] * d0 + km.mt[7] * d1 + km.mt[8] * d2));
        acc[r] = 0.f;
    }
    for (int64_t i0 = 0; i0 < m; i0 += kKc) {
        const int nc = static_cast<int>(min<int64_t>(kKc, m - i0));
        __syncthreads();
        if (threadIdx.x < nc) so[threadIdx.x] = obs[i0 + threadIdx.x];
        __syncthreads();
        for (int q = 0; q < nc; ++q) {
            const float4 o = so[q];
#pragma unroll
            for (int r = 0; r < kKr; ++r) {
                const float a = v0[r] - o.x, b = v1[r] - o.y, e = v2[r] - o.z;
                acc[r] = fmaf(o.w, corr_scaled<KIND>(a * a + b * b + e * e), acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kKr; ++r) {
        const int64_t c = base + 256 * r;
        if (c < tg.count) y[c] += acc[r];
    }
}

// Row form of the grid correction, for maps whose second and third lag components do not
// depend on the x index (M^T entries (1, 0) and (2, 0) zero: no rotation that mixes x into
// them).  Each lane takes kKx consecutive cells of one grid row; they share u1 and u2, so the
// part (u1 - u_i1)^2 + (u2 - u_i2)^2 of the squared lag is formed once per observation and row.
template <int KIND>
__global__ __launch_bounds__(256) void k_krige_apply_rows(const float4* __restrict__ obs,
                                                         const double* __restrict__ ref, int64_t m, KrigeModel km,
                                                         KrigeTarget tg, float* __restrict__ y)
{
    __shared__ float4 so[kKc];
    const int64_t n0 = tg.n[0];
    const int64_t nq = (n0 + kKx - 1) / kKx;  // lanes per row
    const int64_t units = tg.count / n0 * nq;
    const int64_t u = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t uc = min(u, units - 1);
    const int64_t row = uc / nq, xs = (uc % nq) * kKx;
    const int64_t j = row % tg.n[1], k = row / tg.n[1];
    const double ks = lag_scale(KIND);
    const double d1 = tg.o[1] + (static_cast<double>(j) + 0.5) * tg.h[1] - ref[1];
    const double d2 = tg.dim == 3 ? tg.o[2] + (static_cast<double>(k) + 0.5) * tg.h[2] - ref[2] : 0.0;
    const float w1 = static_cast<float>(ks * (km.mt[4] * d1 + km.mt[5] * d2));
    const float w2 = static_cast<float>(ks * (km.mt[7] * d1 + km.mt[8] * d2));
    float v0[kKx], acc[kKx];
#pragma unroll
    for (int r = 0; r < kKx; ++r) {
        const double d0 = tg.o[0] + (static_cast<double>(min(xs + r, n0 - 1)) + 0.5) * tg.h[0] - ref[0];
        v0[r] = static_cast<float>(ks * (km.mt[0] * d0 + km.mt[1] * d1 + km.mt[2] * d2));
        acc[r] = 0.f;
    }
    for (int64_t i0 = 0; i0 < m; i0 += kKc) {
        const int nc = static_cast<int>(min<int64_t>(kKc, m - i0));
        __syncthreads();
        if (threadIdx.x < nc) so[threadIdx.x] = obs[i0 + threadIdx.x];
        __syncthreads();
        for (int q = 0; q < nc; ++q) {
            const float4 o = so[q];
            const float b = w1 - o.y, e = w2 - o.z;
            const float be = fmaf(b, b, e * e);
#pragma unroll
            for (int r = 0; r < kKx; ++r) {
                const float a = v0[r] - o.x;
                acc[r] = fmaf(o.w, corr_scaled<KIND>(fmaf(a, a, be)), acc[r]);
            }
        }
    }
    if (u >= units) return;
    float* yr = y + row * n0;
#pragma unroll
    for (int r = 0; r < kKx; ++r)
        if (xs + r < n0) yr[xs + r] += acc[r];
}

}  // namespace

hipError_t launch_cov_matrix(const double* x, int64_t m, int dim, const KrigeModel& km, double* C, int64_t lda,
                             hipStream_t s)
{
    const int64_t t = (m + 15) / 16;
    if (t > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cov_matrix, dim3(static_cast<unsigned>(t), static_cast<unsigned>(t)), dim3(256), 0, s, x, m,
                       dim, km, C, lda);
    return hipGetLastError();
}

hipError_t launch_cholesky(double* A, int64_t m, int64_t lda, double* dinv, double* r, double* z, int32_t* info,
                           hipStream_t s)
{
    const int64_t nblk = (m + kB - 1) / kB;
    if ((nblk - 1) * nblk / 2 > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol_first, dim3(1), dim3(256), 0, s, A, m, lda, dinv, info);
    for (int64_t p = 0; p + 1 < nblk; ++p) {
        const int64_t n = nblk - 1 - p;
        hipLaunchKernelGGL(k_chol_step, dim3(static_cast<unsigned>(n * (n + 1) / 2)), dim3(256), 0, s, A, m, lda, p,
                           dinv, r, z, info);
    }
    return hipGetLastError();
}

hipError_t launch_chol_back(const double* A, int64_t m, int64_t lda, const double* dinv, const double* r, double* z,
                            double* x, hipStream_t s)
{
    const int64_t nblk = (m + kB - 1) / kB;
    for (int64_t bh = nblk - 1; bh >= 0; bh -= 2) {
        const int two = bh >= 1 ? 1 : 0;
        const int64_t rows = (bh - two) * kB;  // rows above the launch's blocks
        const unsigned blocks = static_cast<unsigned>(rows > 0 ? (rows + 31) / 32 : 1);
        hipLaunchKernelGGL(k_chol_back, dim3(blocks), dim3(256), 0, s, A, m, lda, bh, two, dinv, r, z, x,
                           bh == nblk - 1 ? 1 : 0);
    }
    return hipGetLastError();
}

hipError_t launch_residual(const float* d, const float* y, int64_t m, double* r, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256), 0, s, d, y, m, r);
    return hipGetLastError();
}

hipError_t launch_krige_stage(const double* x, const double* alpha, int64_t m, int dim, const KrigeModel& km,
                              float4* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_krige_stage, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256), 0, s, x, alpha, m, dim,
                       km, out);
    return hipGetLastError();
}

hipError_t launch_krige_apply(const float4* obs, const double* xobs, int64_t m, const KrigeModel& km,
                              const KrigeTarget& tg, float* y, hipStream_t s)
{
    if (tg.count <= 0) return hipSuccess;
    if (tg.grid && km.mt[3] == 0.0 && km.mt[6] == 0.0) {
        const int64_t n0 = tg.n[0];
        const int64_t units = tg.count / n0 * ((n0 + kKx - 1) / kKx);
        const int64_t rb = (units + 255) / 256;
        if (rb > 0x7fffffff) return hipErrorInvalidValue;
        const dim3 gr(static_cast<unsigned>(rb));
        switch (km.kind) {
        case KR_GAUSS: hipLaunchKernelGGL((k_krige_apply_rows<KR_GAUSS>), gr, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
        case KR_EXP: hipLaunchKernelGGL((k_krige_apply_rows<KR_EXP>), gr, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
        case KR_M32: hipLaunchKernelGGL((k_krige_apply_rows<KR_M32>), gr, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
        default: hipLaunchKernelGGL((k_krige_apply_rows<KR_M52>), gr, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
        }
        return hipGetLastError();
    }
    const int64_t blocks = (tg.count + 256 * kKr - 1) / (256 * kKr);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g(static_cast<unsigned>(blocks));
    switch (km.kind * 2 + (tg.grid ? 1 : 0)) {
    case KR_GAUSS * 2 + 1: hipLaunchKernelGGL((k_krige_apply<true, KR_GAUSS>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    case KR_GAUSS * 2: hipLaunchKernelGGL((k_krige_apply<false, KR_GAUSS>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    case KR_EXP * 2 + 1: hipLaunchKernelGGL((k_krige_apply<true, KR_EXP>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    case KR_EXP * 2: hipLaunchKernelGGL((k_krige_apply<false, KR_EXP>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    case KR_M32 * 2 + 1: hipLaunchKernelGGL((k_krige_apply<true, KR_M32>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    case KR_M32 * 2: hipLaunchKernelGGL((k_krige_apply<false, KR_M32>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    case KR_M52 * 2 + 1: hipLaunchKernelGGL((k_krige_apply<true, KR_M52>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    default: hipLaunchKernelGGL((k_krige_apply<false, KR_M52>), g, dim3(256), 0, s, obs, xobs, m, km, tg, y); break;
    }
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace grf
