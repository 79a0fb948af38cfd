// Conditioning a realisation on observations by kriging its residuals (the paper names
// conditioning on data as future work, Sec. 6):
//   alpha = (C(X, X) + nugget sigma^2 I)^-1 (d - Y(X)),   Y_c(x) = Y(x) + sum_i alpha_i C(x - x_i),
// with the model covariance C(dx) = sigma^2 rho(|M^T dx|), M = R diag(1/ell) (the same
// anisotropy as the field's wavevectors k = M z; App. A correlations).
//
// The M x M system is factorised in FP64 by a blocked right-looking Cholesky (diagonal block
// factored by every panel workgroup, panel triangular solve, trailing update), solved by
// blocked substitution (one launch
// per block and direction, the right-hand side updated by many workgroups), and the
// correction is summed in FP32 with observation chunks staged in LDS.
#include <hip/hip_runtime.h>

#include <cmath>

#include "grf_internal.h"

namespace grf {

namespace {

constexpr int kNb = 32;  // Cholesky block

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

// FP32 correlation for the correction sum, on the hardware square root and base-2 exponential
// (about 1 ulp each; the sum is FP32 anyway).
template <int KIND>
__device__ __forceinline__ float corr_r2f(float r2)
{
    constexpr float kLog2e = 1.4426950408889634f;
    if constexpr (KIND == KR_GAUSS) return __builtin_amdgcn_exp2f(-r2 * kLog2e);
    const float r = __builtin_amdgcn_sqrtf(r2);
    if constexpr (KIND == KR_EXP) return __builtin_amdgcn_exp2f(-r * kLog2e);
    if constexpr (KIND == KR_M32) {
        const float a = 1.7320508f * r;
        return (1.f + a) * __builtin_amdgcn_exp2f(-a * kLog2e);
    }
    const float a = 2.2360680f * r;
    return (1.f + a + a * a * (1.f / 3.f)) * __builtin_amdgcn_exp2f(-a * kLog2e);
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

// Unblocked factorisation of an nb x nb diagonal block by one wave: lane r holds row r
// (entries c <= r) in `row` on entry and the factor's row on exit; column j goes through the
// LDS scratch `col` for the rank-1 update.  Returns the first non-positive pivot (1-based,
// counted from the matrix's first row via k0) or 0; the factor then carries NaN.
__device__ __forceinline__ int factor_block(double (&row)[kNb], int nb, int64_t k0, double* col)
{
    const int r = threadIdx.x;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < kNb; ++j) {
        if (j < nb) {
            // pivot of column j, from lane j
            const double d = lane_bcast(row[j], j);
            const double sd = d > 0.0 ? sqrt(d) : __builtin_nan("");
            if (!(d > 0.0) && bad == 0) bad = static_cast<int>(k0 + j + 1);
            if (r == j) row[j] = sd;
            if (r > j && r < nb) row[j] /= sd;
            if (r < kNb) col[r] = row[j];
            // one wave, whose LDS accesses complete in program order: a compiler barrier
            // orders the column's stores before the reads and the reads before the next
            // column's stores
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = j + 1; c < kNb; ++c)
                if (c <= r && r < nb) row[c] -= row[j] * col[c];
            __builtin_amdgcn_wave_barrier();
        }
    }
    return bad;
}

// One panel step of the Cholesky factorisation, one wave per workgroup: the factor L_kk of
// the diagonal block [k0, k0 + nb) is either made here (first panel: every workgroup factors
// the block itself, workgroup 0 stores it in `dk` (32 x 32, row-major) and the first
// non-positive pivot in `info`) or read from `dk`, where the preceding trailing update left
// it; then each workgroup solves its panel rows i >= k0 + nb: L[i][k0 ..] = A[i][k0 ..]
// L_kk^-T.  A's diagonal block is only read, so the redundant factorisations never race.
__global__ __launch_bounds__(64) void k_potrf_trsm(double* __restrict__ A, int64_t m, int64_t lda, int64_t k0,
                                                  double* __restrict__ dk, int32_t* __restrict__ info,
                                                  int prefactored)
{
    __shared__ double col[kNb];
    __shared__ double L[kNb][kNb + 1];
    __shared__ double dinv[kNb];
    const int nb = static_cast<int>(min<int64_t>(kNb, m - k0));
    const int r = threadIdx.x;
    if (prefactored) {
        if (r < kNb) {
#pragma unroll
            for (int c = 0; c < kNb; ++c) L[r][c] = dk[r * kNb + c];
        }
    } else {
        double row[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c) row[c] = (r < nb && c <= r) ? A[(k0 + r) * lda + k0 + c] : 0.0;
        const int bad = factor_block(row, nb, k0, col);
        if (r < kNb) {
#pragma unroll
            for (int c = 0; c < kNb; ++c) L[r][c] = c <= r ? row[c] : 0.0;
        }
        if (blockIdx.x == 0) {
            if (r == 0 && bad && info && *info == 0) *info = bad;
            if (r < kNb) {
#pragma unroll
                for (int c = 0; c < kNb; ++c) dk[r * kNb + c] = L[r][c];
            }
        }
    }
    __syncthreads();
    if (r < nb) dinv[r] = 1.0 / L[r][r];  // the substitution below multiplies by reciprocals
    __syncthreads();
    const int64_t i = k0 + nb + static_cast<int64_t>(blockIdx.x) * blockDim.x + r;
    if (i >= m) return;
    double* prow = A + i * lda + k0;
    double x[kNb];
#pragma unroll
    for (int j = 0; j < kNb; ++j) {
        if (j < nb) {
            double v = prow[j];
            for (int l = 0; l < j; ++l) v -= x[l] * L[j][l];
            x[j] = v * dinv[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kNb; ++j)
        if (j < nb) prow[j] = x[j];
}

// Trailing update A[i][j] -= sum_l L[i][l] L[j][l] over the panel columns [k0, k0 + nb), for
// rows and columns past the panel, lower triangle; 32 x 32 output tiles, 4 entries per thread.
// The workgroup of tile (0, 0), which updates the next panel's diagonal block, then factors
// it (its first wave, from the updated values kept in LDS) into `dk_next` and records a
// non-positive pivot in `info`: the next panel step reads the factor instead of making it.
__global__ __launch_bounds__(256) void k_syrk_update(double* __restrict__ A, int64_t m, int64_t lda, int64_t k0,
                                                     double* __restrict__ dk_next, int32_t* __restrict__ info)
{
    __shared__ double Li[32][kNb + 1];
    __shared__ double Lj[32][kNb + 1];
    __shared__ double T[kNb][kNb + 1];
    __shared__ double colbuf[kNb];
    const int64_t s0 = k0 + kNb;  // first trailing row/column (only called when a full panel precedes it)
    const int64_t ti = blockIdx.y, tj = blockIdx.x;
    if (tj > ti) return;
    const int64_t i0 = s0 + ti * 32, j0 = s0 + tj * 32;
    for (int e = threadIdx.x; e < 32 * kNb; e += blockDim.x) {
        const int r = e / kNb, c = e % kNb;
        Li[r][c] = i0 + r < m ? A[(i0 + r) * lda + k0 + c] : 0.0;
        Lj[r][c] = j0 + r < m ? A[(j0 + r) * lda + k0 + c] : 0.0;
    }
    __syncthreads();
    const int c = threadIdx.x & 31, r0 = threadIdx.x >> 5;  // rows r0, r0 + 8, r0 + 16, r0 + 24
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int l = 0; l < kNb; ++l) {
        const double b = Lj[c][l];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += Li[r0 + 8 * q][l] * b;
    }
    const int64_t j = j0 + c;
    const bool diag_tile = ti == 0 && tj == 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t i = i0 + r0 + 8 * q;
        if (i < m && j < m && j <= i) {
            const double v = A[i * lda + j] - acc[q];
            A[i * lda + j] = v;
            if (diag_tile) T[r0 + 8 * q][c] = v;
        }
    }
    if (diag_tile) {
        __syncthreads();
        if (threadIdx.x < 64) {
            const int nbn = static_cast<int>(min<int64_t>(kNb, m - s0));
            const int r = threadIdx.x;
            double row[kNb];
#pragma unroll
            for (int cc = 0; cc < kNb; ++cc) row[cc] = (r < nbn && cc <= r) ? T[r][cc] : 0.0;
            const int bad = factor_block(row, nbn, s0, colbuf);
            if (r == 0 && bad && info && *info == 0) *info = bad;
            if (r < kNb) {
#pragma unroll
                for (int cc = 0; cc < kNb; ++cc) dk_next[r * kNb + cc] = cc <= r ? row[cc] : 0.0;
            }
        }
    }
}

// x = (L L^T)^-1 b by blocked substitution, one launch per 32-row block and direction.  In
// every launch each workgroup stages the diagonal block in LDS and solves it with one wave
// (the same small solve, redundantly), then updates its share of the remaining right-hand
// side; workgroup 0 stores the block's solution.  A step reads only the block's right-hand
// side and writes only the solution and the rows past the block, so workgroups never race.
__device__ __forceinline__ void stage_diag(const double* __restrict__ dk, int nb, double (&D)[kNb][kNb + 1],
                                           double (&dinv)[kNb])
{
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int r = e / nb, c = e % nb;
        D[r][c] = c <= r ? dk[r * kNb + c] : 0.0;
    }
    if (static_cast<int>(threadIdx.x) < nb) dinv[threadIdx.x] = 1.0 / dk[threadIdx.x * (kNb + 1)];
}

// Forward step: z_k = L_kk^-1 r_k; r_i -= L_ik z_k for rows i >= k0 + nb.
__global__ __launch_bounds__(256) void k_trsv_fwd(const double* __restrict__ L, const double* __restrict__ diag,
                                                  int64_t m, int64_t lda, int64_t k0, double* __restrict__ r,
                                                  double* __restrict__ z)
{
    __shared__ double D[kNb][kNb + 1];
    __shared__ double dinv[kNb];
    __shared__ double xb[kNb];
    const int t = threadIdx.x;
    const int nb = static_cast<int>(min<int64_t>(kNb, m - k0));
    stage_diag(diag + (k0 / kNb) * kNb * kNb, nb, D, dinv);
    if (t < nb) xb[t] = r[k0 + t];
    __syncthreads();
    if (t < 64) {
        // one wave, lane t holding x_t and row t of the block: no LDS round trip per step
        double xr = t < nb ? xb[t] : 0.0, dr[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c) dr[c] = t < nb ? D[t][c] : 0.0;
#pragma unroll
        for (int j = 0; j < kNb; ++j) {
            if (j < nb) {
                const double xj = lane_bcast(xr, j) * dinv[j];
                if (t > j) xr -= dr[j] * xj;
                if (t == j) xr = xj;
            }
        }
        if (t < nb) xb[t] = xr;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t < nb) z[k0 + t] = xb[t];
    // 32 rows per workgroup, eight lanes per row, four consecutive entries per lane: each row's
    // block entries are read as one contiguous run; the eight partial dot products are added
    // by lane exchanges
    const int64_t i = k0 + nb + static_cast<int64_t>(blockIdx.x) * 32 + (t >> 3);
    const int q = 4 * (t & 7);
    double v = 0.0;
    if (i < m) {
        const double* row = L + i * lda + k0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q + u < nb) v += row[q + u] * xb[q + u];
    }
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (i < m && (t & 7) == 0) r[i] -= v;
}

// Backward step: x_k = L_kk^-T z_k; z_i -= L_ki^T x_k for rows i < k0.
__global__ __launch_bounds__(256) void k_trsv_bwd(const double* __restrict__ L, const double* __restrict__ diag,
                                                  int64_t m, int64_t lda, int64_t k0, double* __restrict__ z,
                                                  double* __restrict__ x)
{
    __shared__ double D[kNb][kNb + 1];
    __shared__ double dinv[kNb];
    __shared__ double xb[kNb];
    const int t = threadIdx.x;
    const int nb = static_cast<int>(min<int64_t>(kNb, m - k0));
    stage_diag(diag + (k0 / kNb) * kNb * kNb, nb, D, dinv);
    if (t < nb) xb[t] = z[k0 + t];
    __syncthreads();
    if (t < 64) {
        // one wave, lane t holding x_t and column t of the block
        double xr = t < nb ? xb[t] : 0.0, dc[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c) dc[c] = t < nb ? D[c][t] : 0.0;
#pragma unroll
        for (int j = kNb - 1; j >= 0; --j) {
            if (j < nb) {
                const double xj = lane_bcast(xr, j) * dinv[j];
                if (t < j) xr -= dc[j] * xj;
                if (t == j) xr = xj;
            }
        }
        if (t < nb) xb[t] = xr;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t < nb) x[k0 + t] = xb[t];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + t;
    if (i < k0) {
        double v = 0.0;
        for (int l = 0; l < nb; ++l) v += L[(k0 + l) * lda + i] * xb[l];
        z[i] -= v;
    }
}

// r = d - y (FP64 residuals).
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ d, const float* __restrict__ y, int64_t m,
                                                 double* __restrict__ r)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) r[i] = static_cast<double>(d[i]) - static_cast<double>(y[i]);
}

// Observation staging for the correction: (u = M^T (x_i - x_0) as FP32, w_i = sigma^2 alpha_i);
// lags are taken from the first observation so that the FP32 differences stay small.
__global__ __launch_bounds__(256) void k_krige_stage(const double* __restrict__ x, const double* __restrict__ alpha,
                                                    int64_t m, int dim, KrigeModel km, float4* __restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double* xi = x + i * dim;
    const double d0 = xi[0] - x[0], d1 = xi[1] - x[1], d2 = dim == 3 ? xi[2] - x[2] : 0.0;
    const double u0 = km.mt[0] * d0 + km.mt[1] * d1 + km.mt[2] * d2;
    const double u1 = km.mt[3] * d0 + km.mt[4] * d1 + km.mt[5] * d2;
    const double u2 = km.mt[6] * d0 + km.mt[7] * d1 + km.mt[8] * d2;
    out[i] = make_float4(static_cast<float>(u0), static_cast<float>(u1), static_cast<float>(u2),
                         static_cast<float>(km.s2 * alpha[i]));
}

constexpr int kKc = 256;  // observations per LDS chunk
constexpr int kKr = 4;    // cells per lane

// y[c] += sum_i w_i rho(|u(c) - u_i|) for cells of a grid (grid != nullptr) or points.
template <bool GRID, int KIND>
__global__ __launch_bounds__(256) void k_krige_apply(const float4* __restrict__ obs, const double* __restrict__ ref,
                                                    int64_t m, KrigeModel km, KrigeTarget tg, float* __restrict__ y)
{
    __shared__ float4 so[kKc];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (256 * kKr) + threadIdx.x;
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
        v0[r] = static_cast<float>(km.mt[0] * d0 + km.mt[1] * d1 + km.mt[2] * d2);
        v1[r] = static_cast<float>(km.mt[3] * d0 + km.mt[4] * d1 + km.mt[5] * d2);
        v2[r] = static_cast<float>(km.mt[6] * d0 + km.mt[7] * d1 + km.mt[8] * d2);
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
                acc[r] = fmaf(o.w, corr_r2f<KIND>(a * a + b * b + e * e), acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kKr; ++r) {
        const int64_t c = base + 256 * r;
        if (c < tg.count) y[c] += acc[r];
    }
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

hipError_t launch_cholesky(double* A, int64_t m, int64_t lda, double* diag, int32_t* info, hipStream_t s)
{
    for (int64_t k0 = 0; k0 < m; k0 += kNb) {
        const int64_t rest = m - k0 - kNb;
        const unsigned blocks = static_cast<unsigned>(rest > 0 ? (rest + 63) / 64 : 1);
        // the first panel factors its diagonal block; later ones take the factor that the
        // preceding trailing update made
        hipLaunchKernelGGL(k_potrf_trsm, dim3(blocks), dim3(64), 0, s, A, m, lda, k0, diag + (k0 / kNb) * kNb * kNb,
                           info, k0 > 0 ? 1 : 0);
        if (rest <= 0) break;
        const int64_t tiles = (rest + 31) / 32;
        hipLaunchKernelGGL(k_syrk_update, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(tiles)), dim3(256),
                           0, s, A, m, lda, k0, diag + (k0 / kNb + 1) * kNb * kNb, info);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_chol_solve(const double* L, const double* diag, int64_t m, int64_t lda, double* b, double* x,
                             hipStream_t s)
{
    // forward: right-hand side b (updated in place), solution z in x; backward: right-hand
    // side z (x, updated in place), solution in b; then b -> x
    for (int64_t k0 = 0; k0 < m; k0 += kNb) {
        const int64_t below = m - k0 - kNb;
        const unsigned blocks = static_cast<unsigned>(below > 0 ? (below + 31) / 32 : 1);
        hipLaunchKernelGGL(k_trsv_fwd, dim3(blocks), dim3(256), 0, s, L, diag, m, lda, k0, b, x);
    }
    for (int64_t k0 = ((m - 1) / kNb) * kNb; k0 >= 0; k0 -= kNb) {
        const unsigned blocks = static_cast<unsigned>(k0 > 0 ? (k0 + 255) / 256 : 1);
        hipLaunchKernelGGL(k_trsv_bwd, dim3(blocks), dim3(256), 0, s, L, diag, m, lda, k0, x, b);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(x, b, static_cast<size_t>(m) * sizeof(double), hipMemcpyDeviceToDevice, s);
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
    const int64_t blocks = (tg.count + 256 * kKr - 1) / (256 * kKr);
    if (blocks <= 0) return hipSuccess;
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
