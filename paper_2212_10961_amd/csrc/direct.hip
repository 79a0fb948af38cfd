// Direct spectral sums (Sec. 4.1 eq. DiscreteFT, random-phase reading):
//   Y_c = A sum_j cos(2 pi r_jc),   r_jc = frac-reduced phase in revolutions,
// plus the fused epilogue (K = exp(mu + Y), facies index = #{thresholds below Y}; Secs. 4.1
// and 3.1).  At points: one hardware cosine per mode and point.  On grids the phase splits
// into an x part and a (y,z) part, and each term is their angle sum, two FMAs on cosines
// and sines formed once per grid row and mode.
//
// v_cos_f32 / v_sin_f32 take their argument in revolutions and reduce it exactly, so the
// per-axis FP64-reduced fractions are summed in FP32 (values in [0, 3)) and fed to them
// without a further reduction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "grf_internal.h"

namespace grf {

namespace {

__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

__device__ __forceinline__ void store_out(int64_t c, float yv, const Epi& e, float* __restrict__ y,
                                          float* __restrict__ k, uint8_t* __restrict__ ind)
{
    epi_store(c, yv, e, y, k, ind);
}

// ---------------------------------------------------------------------------- grid, FP32
// Block tile: 16 RA x-cells by 16 RB (y,z) pairs; 256 threads; each lane owns RA x RB cells
// (x = x0 + lx + 16 a, q = q0 + 4 RB w + (l / 16) + 4 b).  With the x phase A = 2 pi Tx and
// the (y,z) phase B = 2 pi (Ty + Tz) (psi folded in Ty), each term is the angle sum
// cos(A + B) = cos A cos B - sin A sin B: two FMAs.  Per chunk of J modes the block stages in
// LDS, for each of its x rows, cos A and sin A (hardware cosine and sine of the FP64-reduced
// fraction), and for each (y,z) row w cos B and w sin B (B from the FP32 sum of the two
// fractions, w the mode weight, 1 without weights): rows [J cosines | J sines | 4 floats of
// pad], so the 16 distinct x rows of a wave's 128-bit reads hit distinct banks.  Every cell
// is summed by one lane over the modes in order, whatever the tile and chunk: neither changes
// a result bit.  Large grids take 4 x 8 cells per lane (64 x 128 tiles, 32-mode chunks); the
// batch and mid-size grids 4 x 4 (64 x 64); small grids 2 x 2 or 1 x 1 cells for more blocks,
// with chunks of 64 or 256 modes so that the fewer terms per lane still cover each chunk's loads.
constexpr int kDgB = 64;
static_assert(kDgB == kDirectTile, "tile side shared with the batch planner");

__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }

// LDS float4 of one tile: 16 (RA + RB) rows of (2 J + 4) floats.
template <int RA, int RB, int J>
struct DirectShape {
    static constexpr int ROW = (2 * J + 4) / 4;  // float4 per padded row
    static constexpr int X4 = 16 * RA * ROW, Q4 = 16 * RB * ROW;
};

// One (16 RA) x (16 RB) (x, (y,z)) tile, mode chunks of J; `sx`, `sq` are LDS arrays of
// DirectShape<RA, RB, J>::X4 and ::Q4 float4.  Whole block.
template <int RA, int RB, int J>
__device__ __forceinline__ void direct_tile(const float* __restrict__ tx, const float* __restrict__ ty,
                                            const float* __restrict__ tz, const double* __restrict__ wt, int n,
                                            int64_t ldp, int nx, int ny, int64_t nq, int x0, int64_t q0, float amp,
                                            const Epi& epi, float* __restrict__ y, float* __restrict__ k,
                                            uint8_t* __restrict__ ind, float4* sx, float4* sq)
{
    static_assert(J % 32 == 0, "row stride 2 J + 4 must be 4 (mod 64) floats");
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    const int lx = l & 15, lq = w * 4 * RB + (l >> 4);
    constexpr int kRow = DirectShape<RA, RB, J>::ROW;
    constexpr int kG = J / 4;  // groups of 4 modes per chunk

    float acc[RA][RB];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) acc[a][b] = 0.f;

    for (int j0 = 0; j0 < n; j0 += J) {
        // (rows are ldp long, a multiple of 64: a chunk of 128 past it stages zeros it never sums)
#pragma unroll
        for (int it = 0; it < RA * J / 64; ++it) {
            const int e = it * 256 + t;
            const int row = e / kG, g = e % kG;
            const int xg = min(x0 + row, nx - 1);
            float4 c = make_float4(0.f, 0.f, 0.f, 0.f), sn = c;
            if (J <= 64 || j0 + 4 * g < ldp) {
                const float4 f = *reinterpret_cast<const float4*>(tx + static_cast<int64_t>(xg) * ldp + j0 + 4 * g);
                c = make_float4(cos_rev(f.x), cos_rev(f.y), cos_rev(f.z), cos_rev(f.w));
                sn = make_float4(sin_rev(f.x), sin_rev(f.y), sin_rev(f.z), sin_rev(f.w));
            }
            sx[row * kRow + g] = c;
            sx[row * kRow + kG + g] = sn;
        }
#pragma unroll
        for (int it = 0; it < RB * J / 64; ++it) {
            const int e = it * 256 + t;
            const int row = e / kG, g = e % kG;
            const int64_t q = min(q0 + row, nq - 1);
            const int64_t yy = q % ny, zz = q / ny;
            float4 c = make_float4(0.f, 0.f, 0.f, 0.f), sn = c;
            if (J <= 64 || j0 + 4 * g < ldp) {
                const float4 fa = *reinterpret_cast<const float4*>(ty + yy * ldp + j0 + 4 * g);
                const float4 fb = *reinterpret_cast<const float4*>(tz + zz * ldp + j0 + 4 * g);
                const float4 f = make_float4(fa.x + fb.x, fa.y + fb.y, fa.z + fb.z, fa.w + fb.w);
                c = make_float4(cos_rev(f.x), cos_rev(f.y), cos_rev(f.z), cos_rev(f.w));
                sn = make_float4(sin_rev(f.x), sin_rev(f.y), sin_rev(f.z), sin_rev(f.w));
                if (wt) {
                    // modes past n carry no weight (their terms are not summed)
                    const int j = j0 + 4 * g;
                    const float4 wv = make_float4(j < n ? static_cast<float>(wt[j]) : 0.f,
                                                  j + 1 < n ? static_cast<float>(wt[j + 1]) : 0.f,
                                                  j + 2 < n ? static_cast<float>(wt[j + 2]) : 0.f,
                                                  j + 3 < n ? static_cast<float>(wt[j + 3]) : 0.f);
                    c = make_float4(wv.x * c.x, wv.y * c.y, wv.z * c.z, wv.w * c.w);
                    sn = make_float4(wv.x * sn.x, wv.y * sn.y, wv.z * sn.z, wv.w * sn.w);
                }
            }
            sq[row * kRow + g] = c;
            sq[row * kRow + kG + g] = sn;
        }
        __syncthreads();
        const int jn = min(J, n - j0);
        const int j4 = jn >> 2;
        for (int m = 0; m < j4; ++m) {
            float4 xc[RA], xs[RA], qc[RB], qs[RB];
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                xc[r] = sx[(lx + 16 * r) * kRow + m];
                xs[r] = sx[(lx + 16 * r) * kRow + kG + m];
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                qc[r] = sq[(lq + 4 * r) * kRow + m];
                qs[r] = sq[(lq + 4 * r) * kRow + kG + m];
            }
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    float v = acc[a][b];
                    v = fmaf(xc[a].x, qc[b].x, v);
                    v = fmaf(-xs[a].x, qs[b].x, v);
                    v = fmaf(xc[a].y, qc[b].y, v);
                    v = fmaf(-xs[a].y, qs[b].y, v);
                    v = fmaf(xc[a].z, qc[b].z, v);
                    v = fmaf(-xs[a].z, qs[b].z, v);
                    v = fmaf(xc[a].w, qc[b].w, v);
                    v = fmaf(-xs[a].w, qs[b].w, v);
                    acc[a][b] = v;
                }
        }
        const float* sxf = reinterpret_cast<const float*>(sx);
        const float* sqf = reinterpret_cast<const float*>(sq);
        for (int m = j4 * 4; m < jn; ++m) {
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const float* rx = sxf + (lx + 16 * a) * kRow * 4;
                    const float* rq = sqf + (lq + 4 * b) * kRow * 4;
                    acc[a][b] = fmaf(rx[m], rq[m], acc[a][b]);
                    acc[a][b] = fmaf(-rx[J + m], rq[J + m], acc[a][b]);
                }
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < RA; ++a) {
        const int x = x0 + lx + 16 * a;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int64_t q = q0 + lq + 4 * b;
            if (x < nx && q < nq) {
                store_out(q * nx + x, amp * acc[a][b], epi, y, k, ind);
            }
        }
    }
}

template <int RA, int RB, int J>
__global__ __launch_bounds__(256, 2) void k_direct_grid(const float* __restrict__ tx, const float* __restrict__ ty,
                                                       const float* __restrict__ tz, const double* __restrict__ wt,
                                                       int n, int64_t ldp, int nx, int ny, int64_t nq, int nxt,
                                                       float amp, Epi epi, float* __restrict__ y,
                                                       float* __restrict__ k, uint8_t* __restrict__ ind)
{
    using S = DirectShape<RA, RB, J>;
    __shared__ float4 sx[S::X4];
    __shared__ float4 sq[S::Q4];
    const int64_t bid = blockIdx.x;
    direct_tile<RA, RB, J>(tx, ty, tz, wt, n, ldp, nx, ny, nq, static_cast<int>(bid % nxt) * 16 * RA,
                           (bid / nxt) * 16 * RB, amp, epi, y, k, ind, sx, sq);
}

// Persistent batched form: blocks pull (instance, tile) work items from one atomic counter
// until the queue is drained.
__global__ __launch_bounds__(256, 2) void k_direct_batch(const DirectBatchItem* __restrict__ items, int n_inst,
                                                        int64_t total, unsigned long long* counter)
{
    using S = DirectShape<4, 4, 32>;
    __shared__ float4 sx[S::X4];
    __shared__ float4 sq[S::Q4];
    __shared__ unsigned long long s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t it = static_cast<int64_t>(s_item);
        __syncthreads();
        if (it >= total) break;
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].item0 <= it) lo = mid;
            else hi = mid - 1;
        }
        const DirectBatchItem& b = items[lo];
        const int64_t local = it - b.item0;
        direct_tile<4, 4, 32>(b.tx, b.ty, b.tz, b.w, b.n, b.ldp, b.nx, b.ny, b.nq, static_cast<int>(local % b.nxt) * kDgB,
                              (local / b.nxt) * kDgB, b.amp, b.epi, b.y, b.k, b.ind, sx, sq);
    }
}

// ---------------------------------------------------------------------------- grid, FP64
// One thread per cell, FP64 per-axis fractions summed and reduced in FP64, cos by
// the device library's cospi.  For small problems and as a reference-grade path.  Grids
// too small to fill the device split the modes over blockIdx.y slices of `mslice` modes:
// each slice writes its raw FP64 sums to partial[slice][C] and k_grid_reduce_f64 adds them
// in slice order.
__device__ __forceinline__ void grid_out_f64(int64_t c, double yv, const Epi& epi, double mu64,
                                             float* __restrict__ y, float* __restrict__ k,
                                             uint8_t* __restrict__ ind, double* __restrict__ y64,
                                             double* __restrict__ k64)
{
    if (y64) y64[c] = yv;
    if (k64) k64[c] = exp(mu64 + yv);
    if (y || k || ind) store_out(c, static_cast<float>(yv), epi, y, k, ind);
}

__global__ __launch_bounds__(256) void k_direct_grid_f64(const double* __restrict__ tx, const double* __restrict__ ty,
                                                        const double* __restrict__ tz, const double* __restrict__ wt,
                                                        int n, int64_t ldp, int nx,
                                                        int ny, int64_t C, double amp, Epi epi, double mu64,
                                                        float* __restrict__ y, float* __restrict__ k,
                                                        uint8_t* __restrict__ ind, double* __restrict__ y64,
                                                        double* __restrict__ k64, int mslice,
                                                        double* __restrict__ partial)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int64_t i = c % nx, q = c / nx;
    const int64_t jy = q % ny, kz = q / ny;
    const double* rx = tx + i * ldp;
    const double* ry = ty + jy * ldp;
    const double* rz = tz + kz * ldp;
    const int j0 = static_cast<int>(blockIdx.y) * mslice;
    const int j1 = min(n, j0 + mslice);
    double s = 0.0;
    auto term = [&](double fx, double fy, double fz, double wj) {
        double f = fx + fy + fz;
        f = __builtin_amdgcn_fract(f);  // x - floor(x) in one FP64 instruction
        s += wj * cospi(2.0 * f);
    };
    // Eight modes' table entries are loaded ahead of their terms; the sum keeps mode order.
    constexpr int kMG = 8;
    int j = j0;
    for (; j + kMG <= j1; j += kMG) {
        double fx[kMG], fy[kMG], fz[kMG], ww[kMG];
#pragma unroll
        for (int u = 0; u < kMG; ++u) {
            fx[u] = rx[j + u];
            fy[u] = ry[j + u];
            fz[u] = rz[j + u];
        }
        if (wt) {
#pragma unroll
            for (int u = 0; u < kMG; ++u) ww[u] = wt[j + u];
        } else {
#pragma unroll
            for (int u = 0; u < kMG; ++u) ww[u] = 1.0;
        }
#pragma unroll
        for (int u = 0; u < kMG; ++u) term(fx[u], fy[u], fz[u], ww[u]);
    }
    for (; j < j1; ++j) term(rx[j], ry[j], rz[j], wt ? wt[j] : 1.0);
    if (partial) {
        partial[static_cast<int64_t>(blockIdx.y) * C + c] = s;
        return;
    }
    grid_out_f64(c, amp * s, epi, mu64, y, k, ind, y64, k64);
}

__global__ __launch_bounds__(256) void k_grid_reduce_f64(const double* __restrict__ partial, int slices, int64_t C,
                                                        double amp, Epi epi, double mu64, float* __restrict__ y,
                                                        float* __restrict__ k, uint8_t* __restrict__ ind,
                                                        double* __restrict__ y64, double* __restrict__ k64)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= C) return;
    // Sixteen slice loads are in flight at a time; the adds keep slice order.
    constexpr int kGroup = 16;
    double s = 0.0;
    int q = 0;
    for (; q + kGroup <= slices; q += kGroup) {
        double v[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) v[u] = partial[static_cast<int64_t>(q + u) * C + c];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) s += v[u];
    }
    for (; q < slices; ++q) s += partial[static_cast<int64_t>(q) * C + c];
    grid_out_f64(c, amp * s, epi, mu64, y, k, ind, y64, k64);
}

// ---------------------------------------------------------------------------- points
__global__ __launch_bounds__(256) void k_points_reduce(const float* __restrict__ partial, int slices, int64_t P,
                                                      float amp, Epi epi, float* __restrict__ y,
                                                      float* __restrict__ k, uint8_t* __restrict__ ind)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P) return;
    // Sixteen slice loads are in flight at a time; the adds keep slice order.
    constexpr int kGroup = 16;
    float s = 0.f;
    int q = 0;
    for (; q + kGroup <= slices; q += kGroup) {
        float v[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) v[u] = partial[static_cast<int64_t>(q + u) * P + p];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) s += v[u];
    }
    for (; q < slices; ++q) s += partial[static_cast<int64_t>(q) * P + p];
    store_out(p, amp * s, epi, y, k, ind);
}

// Each lane owns R points; every mode's (a_x, a_y, a_z, psi) in revolutions is
// uniform across the block (scalar loads).  The phase a.x + psi is formed and
// reduced in FP64 per mode and point, then the cosine and the sum run in FP32.
// With few points the modes are split over blockIdx.y slices of `mslice` modes each:
// every slice writes its raw partial sums to partial[slice][P] and k_points_reduce adds
// them in slice order and applies the epilogue.
template <int DIM, int R>
__global__ __launch_bounds__(256) void k_direct_points(const double4* __restrict__ prm, const double* __restrict__ wt,
                                                      int n, const double* __restrict__ xyz, int64_t P, float amp,
                                                      Epi epi, float* __restrict__ y, float* __restrict__ k,
                                                      uint8_t* __restrict__ ind, int mslice,
                                                      float* __restrict__ partial)
{
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (256 * R) + threadIdx.x;
    const int j0 = static_cast<int>(blockIdx.y) * mslice;
    const int j1 = min(n, j0 + mslice);
    double px[R], py[R], pz[R];
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = min(base + 256 * r, P - 1);
        px[r] = xyz[p * DIM];
        py[r] = xyz[p * DIM + 1];
        pz[r] = DIM == 3 ? xyz[p * DIM + 2] : 0.0;
        acc[r] = 0.f;
    }
    auto mode = [&](const double4& m, float wj) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double ph = DIM == 3 ? fma(m.z, pz[r], m.w) : m.w;
            ph = fma(m.y, py[r], ph);
            ph = fma(m.x, px[r], ph);
            ph = __builtin_amdgcn_fract(ph);  // x - floor(x) in one FP64 instruction
            acc[r] = fmaf(wj, cos_rev(static_cast<float>(ph)), acc[r]);
        }
    };
    // The (uniform) mode records are loaded four at a time, ahead of their terms; each point
    // still sums the modes in order.
    constexpr int kMG = 4;
    int j = j0;
    for (; j + kMG <= j1; j += kMG) {
        double4 mm[kMG];
        float ww[kMG];
#pragma unroll
        for (int u = 0; u < kMG; ++u) mm[u] = prm[j + u];
        if (wt) {
#pragma unroll
            for (int u = 0; u < kMG; ++u) ww[u] = static_cast<float>(wt[j + u]);
        } else {
#pragma unroll
            for (int u = 0; u < kMG; ++u) ww[u] = 1.f;
        }
#pragma unroll
        for (int u = 0; u < kMG; ++u) mode(mm[u], ww[u]);
    }
    for (; j < j1; ++j) mode(prm[j], wt ? static_cast<float>(wt[j]) : 1.f);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = base + 256 * r;
        if (p >= P) continue;
        if (partial) partial[static_cast<int64_t>(blockIdx.y) * P + p] = acc[r];
        else store_out(p, amp * acc[r], epi, y, k, ind);
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_direct_points_f64(const double4* __restrict__ prm,
                                                          const double* __restrict__ wt, int n,
                                                          const double* __restrict__ xyz, int64_t P, double amp,
                                                          Epi epi, float* __restrict__ y, float* __restrict__ k,
                                                          uint8_t* __restrict__ ind)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double px = xyz[p * DIM], py = xyz[p * DIM + 1], pz = DIM == 3 ? xyz[p * DIM + 2] : 0.0;
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
        const double4 m = prm[j];
        double ph = fma(m.x, px, fma(m.y, py, fma(m.z, pz, m.w)));
        ph = __builtin_amdgcn_fract(ph);  // x - floor(x) in one FP64 instruction
        s += (wt ? wt[j] : 1.0) * cospi(2.0 * ph);
    }
    store_out(p, static_cast<float>(amp * s), epi, y, k, ind);
}

// ---------------------------------------------------------------------------- epilogue
// Stand-alone epilogue: 4 cells per thread, 16-byte loads and stores.
__global__ __launch_bounds__(256) void k_epilogue(const float* __restrict__ y, int64_t n, Epi epi,
                                                 float* __restrict__ k, uint8_t* __restrict__ ind)
{
    const int64_t n4 = n >> 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 v = reinterpret_cast<const float4*>(y)[i];
        if (k)
            reinterpret_cast<float4*>(k)[i] =
                make_float4(expf(epi.mu + v.x), expf(epi.mu + v.y), expf(epi.mu + v.z), expf(epi.mu + v.w));
        if (ind) {
            int f0 = 0, f1 = 0, f2 = 0, f3 = 0;
            for (int t = 0; t < epi.nthr; ++t) {
                const float th = epi.thr[t];
                f0 += v.x > th;
                f1 += v.y > th;
                f2 += v.z > th;
                f3 += v.w > th;
            }
            reinterpret_cast<uint32_t*>(ind)[i] = static_cast<uint32_t>(f0) | (static_cast<uint32_t>(f1) << 8) |
                                                  (static_cast<uint32_t>(f2) << 16) | (static_cast<uint32_t>(f3) << 24);
        }
    }
    // ragged tail (n not a multiple of 4)
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const int64_t c = n4 * 4 + threadIdx.x;
        store_out(c, y[c], epi, nullptr, k, ind);
    }
}

// Bitruncated rule over two stored fields.
__device__ __forceinline__ int pluri_facies(float a, float b, const PluriEpi& pe)
{
    int i = 0, j = 0;
    for (int q = 0; q < pe.nt; ++q) i += (a > pe.t[q]) ? 1 : 0;
    for (int q = 0; q < pe.ns; ++q) j += (b > pe.s[q]) ? 1 : 0;
    return pe.rule[i * (pe.ns + 1) + j];
}

// Four cells per thread and step (16-byte loads of both fields, one 4-byte facies store and a
// 16-byte value store); the caller guarantees 16-byte aligned fields and value, 4-byte aligned
// facies.  Cells past the last multiple of four go through the per-cell form.
__global__ __launch_bounds__(256) void k_pluri4(const float* __restrict__ y1, const float* __restrict__ y2, int64_t n,
                                               PluriEpi pe, uint8_t* __restrict__ facies, float* __restrict__ value)
{
    const int64_t n4 = n >> 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n4; q += stride) {
        const float4 a = reinterpret_cast<const float4*>(y1)[q];
        const float4 b = reinterpret_cast<const float4*>(y2)[q];
        const int f0 = pluri_facies(a.x, b.x, pe), f1 = pluri_facies(a.y, b.y, pe);
        const int f2 = pluri_facies(a.z, b.z, pe), f3 = pluri_facies(a.w, b.w, pe);
        if (facies)
            reinterpret_cast<uint32_t*>(facies)[q] = static_cast<uint32_t>(f0) | (static_cast<uint32_t>(f1) << 8) |
                                                     (static_cast<uint32_t>(f2) << 16) | (static_cast<uint32_t>(f3) << 24);
        if (value)
            reinterpret_cast<float4*>(value)[q] = make_float4(pe.values[f0], pe.values[f1], pe.values[f2], pe.values[f3]);
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const int64_t c = n4 * 4 + threadIdx.x;
        const int f = pluri_facies(y1[c], y2[c], pe);
        if (facies) facies[c] = static_cast<uint8_t>(f);
        if (value) value[c] = pe.values[f];
    }
}

// One cell per thread and step (unaligned buffers).
__global__ __launch_bounds__(256) void k_pluri(const float* __restrict__ y1, const float* __restrict__ y2, int64_t n,
                                              PluriEpi pe, uint8_t* __restrict__ facies, float* __restrict__ value)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < n; c += stride) {
        const int f = pluri_facies(y1[c], y2[c], pe);
        if (facies) facies[c] = static_cast<uint8_t>(f);
        if (value) value[c] = pe.values[f];
    }
}

__global__ __launch_bounds__(256) void k_epilogue_scalar(const float* __restrict__ y, int64_t n, Epi epi,
                                                        float* __restrict__ k, uint8_t* __restrict__ ind)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < n; c += stride)
        store_out(c, y[c], epi, nullptr, k, ind);
}

}  // namespace

hipError_t launch_direct_grid_f32(const float* tx, const float* ty, const float* tz, const double* w, int64_t n,
                                  int64_t ldp, const int64_t* gn, float amp, const Epi& epi, float* y, float* k,
                                  uint8_t* ind, hipStream_t s)
{
    const int nx = static_cast<int>(gn[0]), ny = static_cast<int>(gn[1]);
    const int64_t nq = gn[1] * gn[2];
    // the widest tile that still gives two blocks per CU (512), else 1 x 1 cells per lane
    auto blocks_of = [&](int sx_, int sq_) -> int64_t {
        return static_cast<int64_t>((nx + sx_ - 1) / sx_) * ((nq + sq_ - 1) / sq_);
    };
    int v = 3;
    if (blocks_of(64, 128) >= 512) v = 0;
    else if (blocks_of(64, 64) >= 512) v = 1;
    else if (blocks_of(32, 32) >= 512) v = 2;
    static constexpr int kSx[4] = {64, 64, 32, 16}, kSq[4] = {128, 64, 32, 16};
    const int nxt = (nx + kSx[v] - 1) / kSx[v];
    const int64_t blocks = blocks_of(kSx[v], kSq[v]);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g(static_cast<unsigned>(blocks));
    const int nn = static_cast<int>(n);
    switch (v) {
    case 0: hipLaunchKernelGGL((k_direct_grid<4, 8, 32>), g, dim3(256), 0, s, tx, ty, tz, w, nn, ldp, nx, ny, nq, nxt, amp, epi, y, k, ind); break;
    case 1: hipLaunchKernelGGL((k_direct_grid<4, 4, 32>), g, dim3(256), 0, s, tx, ty, tz, w, nn, ldp, nx, ny, nq, nxt, amp, epi, y, k, ind); break;
    case 2: hipLaunchKernelGGL((k_direct_grid<2, 2, 64>), g, dim3(256), 0, s, tx, ty, tz, w, nn, ldp, nx, ny, nq, nxt, amp, epi, y, k, ind); break;
    default: hipLaunchKernelGGL((k_direct_grid<1, 1, 256>), g, dim3(256), 0, s, tx, ty, tz, w, nn, ldp, nx, ny, nq, nxt, amp, epi, y, k, ind); break;
    }
    return hipGetLastError();
}

ModeSlices direct_grid_f64_slices(const int64_t* gn, int64_t n)
{
    // about 1024 blocks in all, at least 32 modes per slice, at most 64 slices
    const int64_t blocks = (gn[0] * gn[1] * gn[2] + 255) / 256;
    ModeSlices r{1, n};
    if (blocks <= 0 || n <= 0 || blocks >= 512) return r;
    int64_t sl = std::min<int64_t>(std::min<int64_t>((1024 + blocks - 1) / blocks, n / 32), 64);
    if (sl <= 1) return r;
    r.mslice = (n + sl - 1) / sl;
    r.slices = static_cast<int>((n + r.mslice - 1) / r.mslice);
    return r;
}

hipError_t launch_direct_grid_f64(const double* tx, const double* ty, const double* tz, const double* w, int64_t n,
                                  int64_t ldp, const int64_t* gn, double amp, const Epi& epi, double mu64, float* y,
                                  float* k, uint8_t* ind, double* y64, double* k64, double* partial, hipStream_t s)
{
    const int64_t C = gn[0] * gn[1] * gn[2];
    const int64_t blocks = (C + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const ModeSlices ms = direct_grid_f64_slices(gn, n);
    if (ms.slices > 1 && !partial) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_direct_grid_f64, dim3(static_cast<unsigned>(blocks), static_cast<unsigned>(ms.slices)),
                       dim3(256), 0, s, tx, ty, tz, w, static_cast<int>(n), ldp, static_cast<int>(gn[0]),
                       static_cast<int>(gn[1]), C, amp, epi, mu64, y, k, ind, y64, k64, static_cast<int>(ms.mslice),
                       ms.slices > 1 ? partial : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ms.slices == 1) return e;
    hipLaunchKernelGGL(k_grid_reduce_f64, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, partial, ms.slices, C,
                       amp, epi, mu64, y, k, ind, y64, k64);
    return hipGetLastError();
}

hipError_t launch_direct_points(const double* params, const double* w, int64_t n, int dim, const double* xyz,
                                int64_t P, bool fp64, float amp, const Epi& epi, float* y, float* k, uint8_t* ind,
                                float* partial, hipStream_t s)
{
    const double4* prm = reinterpret_cast<const double4*>(params);
    if (fp64) {
        const int64_t blocks = (P + 255) / 256;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        if (dim == 3)
            hipLaunchKernelGGL(k_direct_points_f64<3>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, prm, w,
                               static_cast<int>(n), xyz, P, static_cast<double>(amp), epi, y, k, ind);
        else
            hipLaunchKernelGGL(k_direct_points_f64<2>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, prm, w,
                               static_cast<int>(n), xyz, P, static_cast<double>(amp), epi, y, k, ind);
        return hipGetLastError();
    }
    constexpr int R = kPointsPerLane;
    const int64_t blocks = (P + 256 * R - 1) / (256 * R);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const int slices = points_mode_slices(P, n);
    const int mslice = static_cast<int>((n + slices - 1) / slices);
    float* part = slices > 1 ? partial : nullptr;
    const dim3 g(static_cast<unsigned>(blocks), static_cast<unsigned>(slices));
    if (dim == 3)
        hipLaunchKernelGGL((k_direct_points<3, R>), g, dim3(256), 0, s, prm, w, static_cast<int>(n), xyz, P, amp, epi,
                           y, k, ind, mslice, part);
    else
        hipLaunchKernelGGL((k_direct_points<2, R>), g, dim3(256), 0, s, prm, w, static_cast<int>(n), xyz, P, amp, epi,
                           y, k, ind, mslice, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || slices == 1) return e;
    hipLaunchKernelGGL(k_points_reduce, dim3(static_cast<unsigned>((P + 255) / 256)), dim3(256), 0, s, partial, slices,
                       P, amp, epi, y, k, ind);
    return hipGetLastError();
}

hipError_t launch_points_reduce(const float* partial, int slices, int64_t P, float amp, const Epi& epi, float* y,
                                float* k, uint8_t* ind, hipStream_t s)
{
    hipLaunchKernelGGL(k_points_reduce, dim3(static_cast<unsigned>((P + 255) / 256)), dim3(256), 0, s, partial, slices,
                       P, amp, epi, y, k, ind);
    return hipGetLastError();
}

int bin_mode_slices(int64_t P, int64_t n)
{
    // about 8192 work-item waves (several per SIMD); each slice keeps >= 64 modes
    if (P <= 0 || n <= 0) return 1;
    const int64_t waves = (P + kBinItemSlots - 1) / kBinItemSlots;
    int64_t s = (8192 + waves - 1) / waves;
    s = std::min<int64_t>(s, std::max<int64_t>(n / 64, 1));
    s = std::min<int64_t>(s, 64);
    return static_cast<int>(std::max<int64_t>(s, 1));
}

int points_mode_slices(int64_t P, int64_t n)
{
    // Enough blocks to fill 256 CUs several times over; each slice keeps >= 64 modes.
    if (P <= 0 || n <= 0) return 1;
    const int64_t pblocks = (P + 256 * kPointsPerLane - 1) / (256 * kPointsPerLane);
    int64_t s = (2048 + pblocks - 1) / pblocks;
    s = std::min<int64_t>(s, std::max<int64_t>(n / 64, 1));
    s = std::min<int64_t>(s, 64);
    return static_cast<int>(std::max<int64_t>(s, 1));
}

hipError_t launch_direct_batch(const DirectBatchItem* items, int n_inst, int64_t total, unsigned long long* counter,
                               int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_direct_batch, dim3(grid), dim3(256), 0, s, items, n_inst, total, counter);
    return hipGetLastError();
}

int direct_batch_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_direct_batch, 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_pluri_epilogue(const float* y1, const float* y2, int64_t n, const PluriEpi& pe, uint8_t* facies,
                                 float* value, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const bool aligned = reinterpret_cast<uintptr_t>(y1) % 16 == 0 && reinterpret_cast<uintptr_t>(y2) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(value) % 16 == 0 && reinterpret_cast<uintptr_t>(facies) % 4 == 0;
    if (aligned) {
        int64_t blocks = ((n >> 2) + 255) / 256;
        if (blocks < 1) blocks = 1;
        if (blocks > 256 * 64) blocks = 256 * 64;
        hipLaunchKernelGGL(k_pluri4, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, y1, y2, n, pe, facies,
                           value);
        return hipGetLastError();
    }
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_pluri, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, y1, y2, n, pe, facies, value);
    return hipGetLastError();
}

hipError_t launch_epilogue(const float* y, int64_t n, const Epi& epi, float* k, uint8_t* ind, hipStream_t s)
{
    const bool aligned = (reinterpret_cast<uintptr_t>(y) % 16 == 0) && (reinterpret_cast<uintptr_t>(k) % 16 == 0) &&
                         (reinterpret_cast<uintptr_t>(ind) % 4 == 0);
    if (!aligned) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 256 * 64) blocks = 256 * 64;
        hipLaunchKernelGGL(k_epilogue_scalar, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, y, n, epi, k, ind);
        return hipGetLastError();
    }
    const int64_t n4 = n >> 2;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_epilogue, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, y, n, epi, k, ind);
    return hipGetLastError();
}

}  // namespace grf
