// Adjoint of the spectral sum (field_backward).
//
// With theta_jp = k_j . x_p + phi_j and A = sigma sqrt(2/N) (Sec. 4.1 eq. DiscreteFT,
// k = z / ell), the gradients of L given g_p = dL/dY_p are
//   dL/dphi_j = -A S_j,  dL/dk_{a,j} = -A U_{a,j},  S_j = sum_p g_p sin theta_jp,
//   U_{a,j} = sum_p g_p x_{p,a} sin theta_jp,
//   dL/dsigma = sum_p g_p Y_p / sigma = (A / sigma) sum_j C_j,  C_j = sum_p g_p cos theta_jp,
//   dL/dell_a = sum_j dL/dk_{a,j} (-z_{a,j} / ell_a^2).
//
// Layout: one lane per mode, points streamed uniformly through the block (their
// coordinates and g come in through scalar loads).  The phase is formed and reduced
// in FP64 per mode and point; sines (and cosines when Y is not saved) are recomputed,
// never stored.  Per-chunk partial sums go to the workspace and are reduced in a
// fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "grf_internal.h"

namespace grf {

namespace {

struct Geo {
    int64_t nx, ny;
    double ox, oy, oz, hx, hy, hz;
};

template <int DIM, bool GRID, bool WANT_C>
__global__ __launch_bounds__(256) void k_bwd(const double4* __restrict__ prm, int64_t ldp,
                                            const double* __restrict__ xyz, int64_t P, int64_t chunk, Geo geo,
                                            const float* __restrict__ gy, float* __restrict__ partial)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t ch = blockIdx.y;
    const int64_t p0 = ch * chunk;
    const int64_t p1 = min(P, p0 + chunk);
    const double4 m = prm[min(j, ldp - 1)];
    float s = 0.f, ux = 0.f, uy = 0.f, uz = 0.f, cc = 0.f;
    auto point = [&](int64_t p, double& x, double& y, double& z, float& g) {
        z = 0.0;
        if (GRID) {
            const int64_t i = p % geo.nx, q = p / geo.nx;
            x = geo.ox + (static_cast<double>(i) + 0.5) * geo.hx;
            y = geo.oy + (static_cast<double>(q % geo.ny) + 0.5) * geo.hy;
            if (DIM == 3) z = geo.oz + (static_cast<double>(q / geo.ny) + 0.5) * geo.hz;
        } else {
            x = xyz[p * DIM];
            y = xyz[p * DIM + 1];
            if (DIM == 3) z = xyz[p * DIM + 2];
        }
        g = gy[p];
    };
    auto term = [&](double x, double y, double z, float g) {
        double ph = DIM == 3 ? fma(m.z, z, m.w) : m.w;
        ph = fma(m.y, y, ph);
        ph = fma(m.x, x, ph);
        ph = __builtin_amdgcn_fract(ph);  // x - floor(x) in one FP64 instruction
        const float f = static_cast<float>(ph);
        const float sn = __builtin_amdgcn_sinf(f);
        s = fmaf(g, sn, s);
        ux = fmaf(g * static_cast<float>(x), sn, ux);
        uy = fmaf(g * static_cast<float>(y), sn, uy);
        if (DIM == 3) uz = fmaf(g * static_cast<float>(z), sn, uz);
        if (WANT_C) cc = fmaf(g, __builtin_amdgcn_cosf(f), cc);
    };
    // The points' (uniform) loads go out eight at a time, ahead of their terms; the sums keep
    // point order.
    constexpr int kU = 8;
    int64_t p = p0;
    for (; p + kU <= p1; p += kU) {
        double x[kU], y[kU], z[kU];
        float g[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) point(p + u, x[u], y[u], z[u], g[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u) term(x[u], y[u], z[u], g[u]);
    }
    for (; p < p1; ++p) {
        double x, y, z;
        float g;
        point(p, x, y, z, g);
        term(x, y, z, g);
    }
    if (j < ldp) {
        float* out = partial + ch * 5 * ldp;
        out[j] = s;
        out[ldp + j] = ux;
        out[2 * ldp + j] = uy;
        out[3 * ldp + j] = uz;
        out[4 * ldp + j] = cc;
    }
}

__device__ inline float block_sum(float v, float* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    float r = 0.f;
    for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

// Per-mode reduction over chunks (fixed order) and per-block partials of the scalar sums.
// ell-gradient weights: dk_a / dell_b = -R_ab z_b / ell_b^2 (R = identity for axis-aligned tables).
struct EllMap {
    double r[9];  // row-major 3 x 3
    double ell[3];
};

// Per-mode weights w_j (when given) scale every per-mode sum: the term of mode j is
// w_j cos(theta_jp).
__global__ __launch_bounds__(256) void k_bwd_reduce(const float* __restrict__ partial, int64_t nch, int64_t n,
                                                   int64_t ldp, int dim, float amp, const double* __restrict__ z,
                                                   const double* __restrict__ wt, EllMap em, float* __restrict__ gphi,
                                                   float* __restrict__ gk, float* __restrict__ scal)
{
    __shared__ float sh[4];
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    float tl[3] = {0.f, 0.f, 0.f}, tc = 0.f;
    if (j < n) {
        // Sixteen chunks' loads are in flight at a time; the adds keep chunk order.
        constexpr int kGroup = 16;
        float S = 0.f, U[3] = {0.f, 0.f, 0.f}, C = 0.f;
        int64_t c = 0;
        for (; c + kGroup <= nch; c += kGroup) {
            float v[kGroup][5];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const float* pc = partial + (c + u) * 5 * ldp + j;
#pragma unroll
                for (int q = 0; q < 5; ++q) v[u][q] = pc[q * ldp];
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                S += v[u][0];
                U[0] += v[u][1];
                U[1] += v[u][2];
                U[2] += v[u][3];
                C += v[u][4];
            }
        }
        for (; c < nch; ++c) {
            const float* pc = partial + c * 5 * ldp;
            S += pc[j];
            U[0] += pc[ldp + j];
            U[1] += pc[2 * ldp + j];
            U[2] += pc[3 * ldp + j];
            C += pc[4 * ldp + j];
        }
        const float wj = wt ? static_cast<float>(wt[j]) : 1.f;
        if (gphi) gphi[j] = -amp * (wj * S);
        float gka[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a >= dim) break;
            gka[a] = -amp * (wj * U[a]);
            if (gk) gk[a * n + j] = gka[a];
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (b >= dim) break;
            double w = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a < dim) w += static_cast<double>(gka[a]) * em.r[3 * a + b];
            tl[b] = static_cast<float>(w * (-z[b * n + j] / (em.ell[b] * em.ell[b])));
        }
        tc = wj * C;
    }
    const float r0 = block_sum(tl[0], sh);
    const float r1 = block_sum(tl[1], sh);
    const float r2 = block_sum(tl[2], sh);
    const float r3 = block_sum(tc, sh);
    if (threadIdx.x == 0) {
        scal[blockIdx.x * 4 + 0] = r0;
        scal[blockIdx.x * 4 + 1] = r1;
        scal[blockIdx.x * 4 + 2] = r2;
        scal[blockIdx.x * 4 + 3] = r3;
    }
}

// dL/dz of a table whose wavevectors are k_j = rot diag(1/ell) z_j, from dL/dk:
// grad_z[b n + j] = (1/ell_b) sum_a rot_ab grad_k[a n + j] (FP64 sum of the FP32 inputs).
__global__ __launch_bounds__(256) void k_grad_z(const float* __restrict__ gk, int dim, int64_t n, EllMap em,
                                               float* __restrict__ gz)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int b = 0; b < dim; ++b) {
        double w = 0.0;
        for (int a = 0; a < dim; ++a) w += static_cast<double>(gk[a * n + j]) * em.r[3 * a + b];
        gz[b * n + j] = static_cast<float>(w / em.ell[b]);
    }
}

// sum_p g_p y_p over chunks of the points (when Y was saved by the forward pass).
__global__ __launch_bounds__(256) void k_dot_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                    int64_t P, float* __restrict__ out)
{
    __shared__ float sh[4];
    float v = 0.f;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; p < P; p += stride) v += a[p] * b[p];
    const float r = block_sum(v, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// The block partials are summed in block order (one thread per sum); they are first loaded
// by the whole block into LDS, 1024 values at a time, so that the loads are in flight together
// instead of one after another.
__global__ __launch_bounds__(256) void k_bwd_final(const float* __restrict__ scal, int nblk, int dim,
                                                  const float* __restrict__ dotp, int ndot, float amp, float sigma,
                                                  float* __restrict__ gsigma, float* __restrict__ gell)
{
    constexpr int kStage = 1024;
    __shared__ float st[kStage];
    const int t = threadIdx.x;
    float acc = 0.f, d = 0.f;  // thread q < 4: scalar sum q; thread 4: the dot product
    const int64_t ns = static_cast<int64_t>(nblk) * 4;
    for (int64_t b0 = 0; b0 < ns; b0 += kStage) {
        const int m = static_cast<int>(ns - b0 < kStage ? ns - b0 : kStage);
        __syncthreads();
        for (int e = t; e < m; e += 256) st[e] = scal[b0 + e];
        __syncthreads();
        if (t < 4)
            for (int e = t; e < m; e += 4) acc += st[e];
    }
    if (dotp) {
        for (int64_t b0 = 0; b0 < ndot; b0 += kStage) {
            const int m = static_cast<int>(ndot - b0 < kStage ? ndot - b0 : kStage);
            __syncthreads();
            for (int e = t; e < m; e += 256) st[e] = dotp[b0 + e];
            __syncthreads();
            if (t == 4)
                for (int e = 0; e < m; ++e) d += st[e];
        }
    }
    if (gell && t < dim) gell[t] = acc;
    if (gsigma) {
        if (dotp) {
            if (t == 4) gsigma[0] = d / sigma;
        } else if (t == 3) {
            gsigma[0] = amp / sigma * acc;
        }
    }
}

// Dense adjoint on a structured grid from the per-axis revolution tables (FP64-reduced,
// psi folded into the y table): theta_jc = A_jx + B_jq with A = 2 pi Tx[x][j] and
// B = 2 pi (Ty[y][j] + Tz[z][j]).  One lane per mode; the block walks a chunk of 32 x 32
// (x, (y,z)) cell tiles.  Per tile each lane forms the cosines and sines of its mode's 32 x
// and 32 (y,z) phases; the per-cell weights g (0 outside the grid) and the tile's coordinates
// are shared through LDS (broadcast reads).  Along tile row q the angle sum gives
//   sum_x g sin(A + B) = cos B S1 + sin B S2,   sum_x g x sin(A + B) = cos B S3 + sin B S4,
//   sum_x g cos(A + B) = cos B S2 - sin B S1,
// with S1 = sum_x g sin A, S2 = sum_x g cos A and S3, S4 their x-weighted twins: four FMAs
// per cell, then s += r, u_x += r_x, u_y += y r, u_z += z r per row.
constexpr int kBT = 32;

__device__ __forceinline__ float cos_rev_b(float r) { return __builtin_amdgcn_cosf(r); }
__device__ __forceinline__ float sin_rev_b(float r) { return __builtin_amdgcn_sinf(r); }

template <bool WANT_C>
__global__ __launch_bounds__(256) void k_bwd_grid_tab(const float* __restrict__ tx, const float* __restrict__ ty,
                                                     const float* __restrict__ tz, int64_t ldp, Geo geo, int64_t nq,
                                                     int nxt, int64_t ntiles, int64_t tiles_per_chunk,
                                                     const float* __restrict__ gy, float* __restrict__ partial)
{
    constexpr int kA4 = kBT / 4;            // float4 of g per tile row
    __shared__ float4 sg[kBT * kA4];        // g of cell (row b, column a) at [kA4 b + a / 4].(a % 4)
    __shared__ float sxc[kBT];              // x of the tile's columns
    __shared__ float2 syz[kBT];             // (y, z) of the tile's rows
    const int t = threadIdx.x;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + t;
    const int64_t jc = min(j, ldp - 1);
    const int64_t ch = blockIdx.y;
    const int64_t t0 = ch * tiles_per_chunk, t1 = min(ntiles, t0 + tiles_per_chunk);
    float s = 0.f, ux = 0.f, uy = 0.f, uz = 0.f, cc = 0.f;
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t x0 = (tile % nxt) * kBT;
        const int64_t q0 = (tile / nxt) * kBT;
        float cA[kBT], sA[kBT], cB[kBT], sB[kBT];
#pragma unroll
        for (int r = 0; r < kBT; ++r) {
            const float fx = tx[min(x0 + r, geo.nx - 1) * ldp + jc];
            const int64_t q = min(q0 + r, nq - 1);
            const float fq = ty[(q % geo.ny) * ldp + jc] + tz[(q / geo.ny) * ldp + jc];
            cA[r] = cos_rev_b(fx);
            sA[r] = sin_rev_b(fx);
            cB[r] = cos_rev_b(fq);
            sB[r] = sin_rev_b(fq);
        }
        __syncthreads();  // previous tile's weights are no longer read
#pragma unroll
        for (int e = t; e < kBT * kBT; e += 256) {
            const int64_t xi = x0 + (e % kBT), q = q0 + (e / kBT);
            reinterpret_cast<float*>(sg)[e] = (xi < geo.nx && q < nq) ? gy[q * geo.nx + xi] : 0.f;
        }
        if (t < kBT) {
            sxc[t] = static_cast<float>(geo.ox + (static_cast<double>(x0 + t) + 0.5) * geo.hx);
            const int64_t qr = min(q0 + t, nq - 1);
            syz[t] = make_float2(static_cast<float>(geo.oy + (static_cast<double>(qr % geo.ny) + 0.5) * geo.hy),
                                 static_cast<float>(geo.oz + (static_cast<double>(qr / geo.ny) + 0.5) * geo.hz));
        }
        __syncthreads();
        float xs[kBT], xc[kBT];
#pragma unroll
        for (int a = 0; a < kBT; ++a) {
            const float x = sxc[a];
            xs[a] = x * sA[a];
            xc[a] = x * cA[a];
        }
#pragma unroll 2
        for (int b = 0; b < kBT; ++b) {
            float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
            for (int a4 = 0; a4 < kA4; ++a4) {
                const float4 g = sg[b * kA4 + a4];
                const float gv[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = 4 * a4 + u;
                    s1 = fmaf(gv[u], sA[a], s1);
                    s2 = fmaf(gv[u], cA[a], s2);
                    s3 = fmaf(gv[u], xs[a], s3);
                    s4 = fmaf(gv[u], xc[a], s4);
                }
            }
            const float rs = fmaf(cB[b], s1, sB[b] * s2);
            const float rx = fmaf(cB[b], s3, sB[b] * s4);
            const float2 yz = syz[b];
            s += rs;
            ux += rx;
            uy = fmaf(yz.x, rs, uy);
            uz = fmaf(yz.y, rs, uz);
            if (WANT_C) cc += fmaf(cB[b], s2, -(sB[b] * s1));
        }
    }
    if (j < ldp) {
        float* out = partial + ch * 5 * ldp;
        out[j] = s;
        out[ldp + j] = ux;
        out[2 * ldp + j] = uy;
        out[3 * ldp + j] = uz;
        out[4 * ldp + j] = cc;
    }
}

template <int DIM, bool GRID>
void launch_bwd_main(const BwdArgs& a, int64_t chunk, const Geo& geo, bool want_c, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>((a.ldp + 255) / 256), static_cast<unsigned>(a.nchunks));
    const double4* prm = reinterpret_cast<const double4*>(a.params);
    if (want_c)
        hipLaunchKernelGGL((k_bwd<DIM, GRID, true>), grid, dim3(256), 0, s, prm, a.ldp, a.xyz, a.P, chunk, geo, a.gy,
                           a.partial);
    else
        hipLaunchKernelGGL((k_bwd<DIM, GRID, false>), grid, dim3(256), 0, s, prm, a.ldp, a.xyz, a.P, chunk, geo, a.gy,
                           a.partial);
}


// ---- separable dense adjoint (grid path; x in chunks of kBwdSepK cells) -----------------
//
// On a structured grid the per-mode sums factor like the forward sum: with rows q = (y, z)
// and U_j[q] = sum_x g[q][x] Ex[x][j] (and its x-weighted twin U^x),
//   S_j = sum_c g_c e^{i theta_jc} = sum_q U_j[q] W_j[q],  W_j[q] = Ey[y_q][j] Ez[z_q][j],
// so s = Im S, c = Re S, u_x = Im sum_q U^x W, u_y = Im sum_q y_q U W, u_z = Im sum_q z_q U W.
// The products U are a real matrix product (rows q, K = x, columns 4 j + (Re Ex, Im Ex,
// x Re Ex, x Im Ex)) on bf16 matrix cores with hi+lo operands (three passes: hi hi, hi lo,
// lo hi, ~2^-16 relative), and the reduction over q with W runs in the epilogue of every
// 32 x 32 output tile, in FP32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split_bf16(float v, uint16_t* hi, uint16_t* lo, int64_t e)
{
    const __bf16 h = static_cast<__bf16>(v);
    const __bf16 l = static_cast<__bf16>(v - static_cast<float>(h));
    hi[e] = __builtin_bit_cast(uint16_t, h);
    lo[e] = __builtin_bit_cast(uint16_t, l);
}

// dL/dY rows as bf16 hi + lo for the x chunk [x0, x0 + kBwdSepK): row r = z nyp + y (y
// padded to nyp, a multiple of 32, so that a 32-row tile is one z-slice), cells past nx and
// padded rows zero.  Stored fragment-major, [r / 32][x / 16][r % 32][x % 16], so that one
// k-step of a 32-row tile (the A fragment of every lane of a wave) is one contiguous KiB.
__global__ __launch_bounds__(256) void k_bwd_sep_ga(const float* __restrict__ g, int64_t nx, int64_t x0, int64_t ny,
                                                   int64_t nyp, int64_t qp, uint16_t* __restrict__ hi,
                                                   uint16_t* __restrict__ lo)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= qp * kBwdSepK) return;
    const int64_t r = e / kBwdSepK, x = e % kBwdSepK;
    const int64_t z = r / nyp, y = r % nyp;
    const int64_t d = (((r >> 5) * (kBwdSepK / 16) + (x >> 4)) * 32 + (r & 31)) * 16 + (x & 15);
    split_bf16((y < ny && x0 + x < nx) ? g[(z * ny + y) * nx + x0 + x] : 0.f, hi, lo, d);
}

// x operand rows 4 j + (Re Ex, Im Ex, x Re Ex, x Im Ex) of the x chunk at x0, at x = ox +
// (x0 + i + 1/2) hx, phase frac(a_j x) formed and reduced in FP64, then split into bf16 hi +
// lo; zero for j >= n and x0 + i >= nx.
__global__ __launch_bounds__(256) void k_bwd_sep_ex(const double* __restrict__ zx, double fs, double ox, double hx,
                                                   int64_t n, int64_t ldp, int64_t nx, int64_t x0,
                                                   uint16_t* __restrict__ hi, uint16_t* __restrict__ lo)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ldp * kBwdSepK) return;
    const int64_t j = e / kBwdSepK, i = e % kBwdSepK;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < n && x0 + i < nx) {
        const double x = ox + (static_cast<double>(x0 + i) + 0.5) * hx;
        const double t = zx[j] * fs * x;
        double sn, cs;
        sincospi(2.0 * (t - floor(t)), &sn, &cs);
        v[0] = cs;
        v[1] = sn;
        v[2] = x * cs;
        v[3] = x * sn;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const __bf16 h = static_cast<__bf16>(static_cast<float>(v[c]));
        const __bf16 l = static_cast<__bf16>(static_cast<float>(v[c] - static_cast<double>(static_cast<float>(h))));
        const int64_t o = (4 * j + c) * kBwdSepK + i;
        hi[o] = __builtin_bit_cast(uint16_t, h);
        lo[o] = __builtin_bit_cast(uint16_t, l);
    }
}

__device__ __forceinline__ float swap_pair(float v)
{
    // quad_perm [1, 0, 3, 2]: lanes 4m <-> 4m + 1, 4m + 2 <-> 4m + 3
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}

struct BwdSepK {
    const uint16_t* ga_hi;
    const uint16_t* ga_lo;
    const uint16_t* ex_hi;
    const uint16_t* ex_lo;
    const float2* ey;
    const float2* ez;
    int64_t ldp, qp, ny, nyp;
    float oy, hy, oz, hz;
};

// Block: 4 waves, 32 modes (8 per wave: columns 4 j + comp of the wave's 32); grid.y splits
// the rows.  Each wave keeps its x-operand fragments (all K) in registers and walks 32-row
// tiles (32 consecutive y of one z-slice): 8 k-steps x 3 bf16 MFMAs, then the epilogue.
// There the lane of column (j, comp) holds 16 rows of that component and takes the partner
// component (Re <-> Im) from the neighbouring lane; with e = Ey[y][j] it accumulates its
// component of V = sum_y U e and of sum_y y U e as own e.x + partner (+-e.y) (the sign by
// comp parity).  At the end of the tile the pair exchanges V once more and applies Ez:
// comp 0 -> Re(V Ez), comp 1 -> Im(V Ez) (with y and z weights), comp 2 -> Im(V^x Ez).
// The two half-waves (rows 4h ..) are added at the end.
// The dL/dY tiles (hi then lo, 8 KiB each per 32 rows) go through LDS, two buffers, loaded
// straight from global memory (global_load_lds) one tile ahead: the four waves share each
// tile instead of each fetching it from L2, and the fetch overlaps the previous tile's work.
typedef const __attribute__((address_space(1))) void bwd_gbl_void;
typedef __attribute__((address_space(3))) void bwd_lds_void;

__global__ __launch_bounds__(256) void k_bwd_sep(BwdSepK p, float* __restrict__ partial)
{
    constexpr int kTileB = 32 * kBwdSepK * 2;  // bytes of one 32-row bf16 tile
    constexpr int kEyOff = 2 * kTileB, kEzOff = kEyOff + 32 * 32 * 8, kBufB = kEzOff + 32 * 8;
    __shared__ __attribute__((aligned(16))) char sa[2][kBufB];  // A hi, A lo, Ey rows, Ez row
    const int t = threadIdx.x, l = t & 63, h = l >> 5;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int col = l & 31, c = col & 3;
    const float sgn = (c & 1) ? 1.f : -1.f;
    const int64_t jb = static_cast<int64_t>(blockIdx.x) * 32 + w * 8;
    const int64_t j = jb + (col >> 2);
    constexpr int KS = kBwdSepK / 16;
    uint4 bh[KS], bl[KS];
    const int64_t brow = (4 * jb + col) * kBwdSepK + 8 * h;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        bh[ks] = *reinterpret_cast<const uint4*>(p.ex_hi + brow + 16 * ks);
        bl[ks] = *reinterpret_cast<const uint4*>(p.ex_lo + brow + 16 * ks);
    }
    float sIm = 0.f, sRe = 0.f, sY = 0.f, sZ = 0.f;
    const int64_t ntile = p.qp / 32;
    const int64_t per = (ntile + gridDim.y - 1) / gridDim.y;
    const int64_t t0 = static_cast<int64_t>(blockIdx.y) * per, t1 = min(ntile, t0 + per);
    // Per tile: 16 chunks of 1 KiB of dL/dY (hi 0..7, lo 8..15), four per wave; the tile's 32
    // Ey rows of the block's 32 modes (256 B each, four rows per chunk), two chunks per wave;
    // the Ez row of its slice (256 B, 16 lanes of wave 0).  Lane l moves bytes 16 l .. of a chunk.
    const int64_t jb0 = static_cast<int64_t>(blockIdx.x) * 32;
    auto issue = [&](int64_t tile, char* buf) {
        const char* gh = reinterpret_cast<const char*>(p.ga_hi + tile * 32 * kBwdSepK);
        const char* gl = reinterpret_cast<const char*>(p.ga_lo + tile * 32 * kBwdSepK);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ch = 4 * w + k;
            const char* src = (ch < 8 ? gh + ch * 1024 : gl + (ch - 8) * 1024) + 16 * l;
            __builtin_amdgcn_global_load_lds((bwd_gbl_void*)src, (bwd_lds_void*)(buf + ch * 1024), 16, 0, 0);
        }
        const int64_t zt = tile * 32 / p.nyp, yt = tile * 32 - zt * p.nyp;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int ch = 2 * w + k;
            const char* src = reinterpret_cast<const char*>(p.ey + (yt + 4 * ch + (l >> 4)) * p.ldp + jb0) + 16 * (l & 15);
            __builtin_amdgcn_global_load_lds((bwd_gbl_void*)src, (bwd_lds_void*)(buf + kEyOff + ch * 1024), 16, 0, 0);
        }
        if (w == 0 && l < 16) {
            const char* src = reinterpret_cast<const char*>(p.ez + zt * p.ldp + jb0) + 16 * l;
            __builtin_amdgcn_global_load_lds((bwd_gbl_void*)src, (bwd_lds_void*)(buf + kEzOff), 16, 0, 0);
        }
    };
    const int jl = w * 8 + (col >> 2);  // this lane's mode within the block's 32
    const int fo = (col * 16 + 8 * h) * 2;  // this lane's fragment bytes within a k-step's 1 KiB
    if (t0 < t1) issue(t0, sa[0]);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const char* cur = sa[(tile - t0) & 1];
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();  // this tile is in `cur` for every wave; every wave is done with the other buffer
        if (tile + 1 < t1) issue(tile + 1, sa[(tile + 1 - t0) & 1]);
        const int64_t q0 = tile * 32;
        // one accumulator: 128 VGPRs, four waves per SIMD to cover the loads and the epilogue
        f32x16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = 0.f;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const uint4 ah = *reinterpret_cast<const uint4*>(cur + ks * 1024 + fo);
            const uint4 al = *reinterpret_cast<const uint4*>(cur + kTileB + ks * 1024 + fo);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bh[ks]),
                                                          acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bl[ks]),
                                                          acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al), __builtin_bit_cast(bf16x8, bh[ks]),
                                                          acc, 0, 0, 0);
        }
        // lane holds rows y = y0 + 8 (e / 4) + 4 h + e % 4 of slice zi, column col
        const int64_t zi = q0 / p.nyp, y0 = q0 - zi * p.nyp + 4 * h;
        const float yb = p.oy + (static_cast<float>(y0) + 0.5f) * p.hy;
        // Ey of rows 4 h + r of the tile (the y table has nyp rows: padded rows have U = 0)
        const float2* eyr = reinterpret_cast<const float2*>(cur + kEyOff) + 4 * h * 32 + jl;
        // sum_y y U e = yb sum U e + hy sum r U e over the lane's rows r
        float vA = 0.f, vR = 0.f;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int r = 8 * (e >> 2) + (e & 3);
            const float2 ey = eyr[r * 32];
            const float own = acc[e], oth = swap_pair(own);
            const float v = fmaf(own, ey.x, oth * (sgn * ey.y));
            vA += v;
            vR = fmaf(static_cast<float>(r), v, vR);
        }
        const float vY = fmaf(yb, vA, p.hy * vR);
        const float2 ez = reinterpret_cast<const float2*>(cur + kEzOff)[jl];
        const float zc = p.oz + (static_cast<float>(zi) + 0.5f) * p.hz;
        const float oA = swap_pair(vA), oY = swap_pair(vY);
        // (re, im) of V and of sum y U e for this lane's pair
        const float ra = (c & 1) ? oA : vA, ia = (c & 1) ? vA : oA;
        const float ry = (c & 1) ? oY : vY, iy = (c & 1) ? vY : oY;
        const float im = fmaf(ra, ez.y, ia * ez.x);
        sIm += im;
        sRe += fmaf(ra, ez.x, -ia * ez.y);
        sY += fmaf(ry, ez.y, iy * ez.x);
        sZ = fmaf(zc, im, sZ);
    }
    sIm += __shfl_xor(sIm, 32);
    sRe += __shfl_xor(sRe, 32);
    sY += __shfl_xor(sY, 32);
    sZ += __shfl_xor(sZ, 32);
    if (h == 0) {
        float* out = partial + static_cast<int64_t>(blockIdx.y) * 5 * p.ldp;
        if (c == 1) {
            out[j] = sIm;
            out[2 * p.ldp + j] = sY;
            out[3 * p.ldp + j] = sZ;
        } else if (c == 0) {
            out[4 * p.ldp + j] = sRe;
        } else if (c == 2) {
            out[p.ldp + j] = sIm;
        }
    }
}

}  // namespace

int64_t bwd_chunks(int64_t P)
{
    int64_t c = (P + 127) / 128;
    if (c < 1) c = 1;
    if (c > 256) c = 256;
    return c;
}

// Row chunks of the separable adjoint: about 2048 blocks, at most 256 (the partial sums'
// workspace) and at most one per 32-row tile.
int64_t bwd_sep_chunks(int64_t ldp, int64_t qp)
{
    int64_t c = 2048 / (ldp / 32);
    c = c < 1 ? 1 : c;
    c = c > 256 ? 256 : c;
    return c < qp / 32 ? c : qp / 32;
}

hipError_t launch_backward(const BwdArgs& a, hipStream_t s)
{
    const int64_t chunk = a.P > 0 ? (a.P + a.nchunks - 1) / a.nchunks : 0;
    Geo geo{};
    const bool grid = a.xyz == nullptr;
    if (grid) {
        geo.nx = a.gn[0];
        geo.ny = a.gn[1];
        geo.ox = a.go[0];
        geo.oy = a.go[1];
        geo.oz = a.dim == 3 ? a.go[2] : 0.0;
        geo.hx = a.gh[0];
        geo.hy = a.gh[1];
        geo.hz = a.dim == 3 ? a.gh[2] : 0.0;
    }
    const bool want_c = a.gsigma != nullptr && a.ysaved == nullptr;
    if (grid && a.sep) {
        // x in chunks of kBwdSepK cells, one after another on the stream (the operand buffers
        // hold one chunk); chunk xc writes its row-chunk sums to partial slots
        // [xc chunks, (xc + 1) chunks), and the reduction adds every slot
        const BwdSep& b = *a.sep;
        const int64_t ng = b.qp * kBwdSepK, ne = a.ldp * kBwdSepK;
        const int64_t nxc = (a.gn[0] + kBwdSepK - 1) / kBwdSepK;
        BwdSepK k{b.ga_hi, b.ga_lo, b.ex_hi, b.ex_lo, b.ey, b.ez, a.ldp, b.qp, b.ny, b.nyp,
                  static_cast<float>(geo.oy), static_cast<float>(geo.hy), static_cast<float>(geo.oz),
                  static_cast<float>(geo.hz)};
        if (a.dim != 3) {
            k.oz = 0.f;
            k.hz = 0.f;
        }
        for (int64_t xc = 0; xc < nxc; ++xc) {
            const int64_t x0 = xc * kBwdSepK;
            hipLaunchKernelGGL(k_bwd_sep_ga, dim3(static_cast<unsigned>((ng + 255) / 256)), dim3(256), 0, s, a.gy,
                               a.gn[0], x0, b.ny, b.nyp, b.qp, b.ga_hi, b.ga_lo);
            hipLaunchKernelGGL(k_bwd_sep_ex, dim3(static_cast<unsigned>((ne + 255) / 256)), dim3(256), 0, s, b.zx,
                               b.fsx, a.go[0], a.gh[0], a.n, a.ldp, a.gn[0], x0, b.ex_hi, b.ex_lo);
            if (xc == 0) timer_mark(s, true);
            hipLaunchKernelGGL(k_bwd_sep, dim3(static_cast<unsigned>(a.ldp / 32), static_cast<unsigned>(b.chunks)),
                               dim3(256), 0, s, k, a.partial + xc * b.chunks * 5 * a.ldp);
        }
    } else if (grid && a.tx) {
        timer_mark(s, true);
        const int64_t nq = a.gn[1] * a.gn[2];
        const int nxt = static_cast<int>((a.gn[0] + kBT - 1) / kBT);
        const int64_t ntiles = static_cast<int64_t>(nxt) * ((nq + kBT - 1) / kBT);
        const int64_t per = (ntiles + a.nchunks - 1) / a.nchunks;
        const dim3 g(static_cast<unsigned>((a.ldp + 255) / 256), static_cast<unsigned>(a.nchunks));
        if (want_c)
            hipLaunchKernelGGL(k_bwd_grid_tab<true>, g, dim3(256), 0, s, a.tx, a.ty, a.tz, a.ldp, geo, nq, nxt, ntiles,
                               per, a.gy, a.partial);
        else
            hipLaunchKernelGGL(k_bwd_grid_tab<false>, g, dim3(256), 0, s, a.tx, a.ty, a.tz, a.ldp, geo, nq, nxt,
                               ntiles, per, a.gy, a.partial);
    } else {
        timer_mark(s, true);
        if (a.dim == 3) {
            if (grid) launch_bwd_main<3, true>(a, chunk, geo, want_c, s);
            else launch_bwd_main<3, false>(a, chunk, geo, want_c, s);
        } else {
            if (grid) launch_bwd_main<2, true>(a, chunk, geo, want_c, s);
            else launch_bwd_main<2, false>(a, chunk, geo, want_c, s);
        }
    }
    timer_mark(s, false);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    const int nblk = static_cast<int>((a.n + 255) / 256);
    EllMap em{};
    for (int i = 0; i < 9; ++i) em.r[i] = a.rot ? a.rot[i] : (i % 4 == 0 ? 1.0 : 0.0);
    for (int b = 0; b < 3; ++b) em.ell[b] = b < a.dim ? a.ell[b] : 1.0;
    hipLaunchKernelGGL(k_bwd_reduce, dim3(nblk), dim3(256), 0, s, a.partial, a.nchunks, a.n, a.ldp, a.dim, a.amp, a.z,
                       a.w, em, a.gphi, a.gk, a.scal_partial);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float* dotp = nullptr;
    int ndot = 0;
    if (a.gsigma && a.ysaved && a.P > 0) {
        ndot = 1024;
        float* dp = a.scal_partial + 4 * nblk;
        hipLaunchKernelGGL(k_dot_partial, dim3(ndot), dim3(256), 0, s, a.gy, a.ysaved, a.P, dp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        dotp = dp;
    }
    hipLaunchKernelGGL(k_bwd_final, dim3(1), dim3(256), 0, s, a.scal_partial, nblk, a.dim, dotp, ndot, a.amp, a.sigma,
                       a.gsigma, a.gell);
    return hipGetLastError();
}

hipError_t launch_grad_z(const float* gk, int dim, int64_t n, const double* rot, const double* ell, float* gz,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    EllMap em{};
    for (int i = 0; i < 9; ++i) em.r[i] = rot ? rot[i] : (i % 4 == 0 ? 1.0 : 0.0);
    for (int b = 0; b < 3; ++b) em.ell[b] = b < dim ? ell[b] : 1.0;
    hipLaunchKernelGGL(k_grad_z, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, gk, dim, n, em, gz);
    return hipGetLastError();
}

}  // namespace grf
