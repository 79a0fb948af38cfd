// Separable (matrix-core) form of the spectral sum on structured grids.
//
// On a grid the mode phase splits per axis (Sec. 4.1, per-axis rescaling), so
//   Y[z][y][x] = A Re sum_j e^{2 pi i (a_{j,x} x)} e^{2 pi i (a_{j,z} z)} e^{2 pi i (a_{j,y} y + psi_j)}
//              = A Re sum_j P_z[x, j] Q[y, j],     P_z = Ex * Ez[z]  (3-D),  P = Ex (2-D).
// Writing the complex products as reals with K = 2N,
//   A_mat[y, 2j] = Re Q, A_mat[y, 2j+1] = Im Q,  B_mat[2j, x] = Re P, B_mat[2j+1, x] = -Im P,
// every z-slice is a dense GEMM Y_z = A_mat B_mat evaluated on MFMA (32x32x16, fp16 or
// bf16 operands, FP32 accumulation).  The split-precision variants store every operand
// as hi + lo and accumulate A_hi B_hi + A_hi B_lo + A_lo B_hi.
//
// Tables are unit-modulus (the amplitude is applied in the epilogue), and their phases
// were reduced in FP64 before rounding.  Output rows are y, columns x, so each wave's
// stores are 128-byte runs along x.
#include <hip/hip_runtime.h>

#include "grf_internal.h"

namespace grf {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kJC = 32;              // modes per LDS stage (64 reals of K)
constexpr int kRowW = kJC + 4;       // padded LDS row, in 32-bit words

__device__ __forceinline__ uint32_t pack_pair(float re, float im, bool bf)
{
    if (bf) {
        const __bf16 r = static_cast<__bf16>(re), i = static_cast<__bf16>(im);
        return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, r)) |
               (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, i)) << 16);
    }
    const _Float16 r = static_cast<_Float16>(re), i = static_cast<_Float16>(im);
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, r)) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, i)) << 16);
}

__device__ __forceinline__ float lo16f(uint32_t v, bool bf)
{
    const uint16_t b = static_cast<uint16_t>(v & 0xffff);
    return bf ? static_cast<float>(__builtin_bit_cast(__bf16, b)) : static_cast<float>(__builtin_bit_cast(_Float16, b));
}
__device__ __forceinline__ float hi16f(uint32_t v, bool bf)
{
    const uint16_t b = static_cast<uint16_t>(v >> 16);
    return bf ? static_cast<float>(__builtin_bit_cast(__bf16, b)) : static_cast<float>(__builtin_bit_cast(_Float16, b));
}

template <bool BF>
__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c)
{
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                       0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0,
                                                      0);
}

// WM x WN waves; each wave owns TM x TN MFMA tiles of 32x32 (rows y, cols x).
template <int WM, int WN, int TM, int TN, bool BF, bool X3, bool D3>
__global__ __launch_bounds__(WM* WN * 64) void k_sep(SepArgs a, int tiles_x, int tiles_y)
{
    constexpr int NT = WM * WN * 64;
    constexpr int BM = WM * TM * 32;   // y rows per block
    constexpr int BN = WN * TN * 32;   // x cols per block
    constexpr int NB = X3 ? 2 : 1;     // hi (+ lo) copies
    __shared__ uint4 smem[(NB * (BM + BN) * kRowW) / 4];
    uint32_t* sA = reinterpret_cast<uint32_t*>(smem);           // [NB][BM][kRowW]
    uint32_t* sB = sA + NB * BM * kRowW;                         // [NB][BN][kRowW]

    const int t = threadIdx.x;
    const int wave = t >> 6, l = t & 63;
    const int wm = wave / WN, wn = wave % WN;
    const int64_t bid = blockIdx.x;
    const int tx = static_cast<int>(bid % tiles_x);
    const int64_t rest = bid / tiles_x;
    const int ty = static_cast<int>(rest % tiles_y);
    const int64_t z0 = rest / tiles_y;
    const int64_t x0 = static_cast<int64_t>(tx) * BN, y0 = static_cast<int64_t>(ty) * BM;
    const int64_t ldp = a.ldp;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

    // staging assignment: 16-byte chunks (4 modes) of a row; 8 chunks per row per stage
    constexpr int CA = BM * (kJC / 4) / NT;  // chunks of A per thread
    constexpr int CB = BN * (kJC / 4) / NT;
    static_assert(CA * NT == BM * kJC / 4 && CB * NT == BN * kJC / 4, "tile/thread mismatch");

    const uint32_t* qy = static_cast<const uint32_t*>(a.qy);
    const uint32_t* qy_lo = static_cast<const uint32_t*>(a.qy_lo);

    for (int64_t j0 = 0; j0 < ldp; j0 += kJC) {
        // ---- stage A (Q rows, y side)
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = t + NT * i;
            const int row = c >> 3, c4 = c & 7;
            const int64_t yg = min(y0 + row, a.ny - 1);
            const int64_t off = yg * ldp + j0 + 4 * c4;
            *reinterpret_cast<uint4*>(sA + row * kRowW + 4 * c4) = *reinterpret_cast<const uint4*>(qy + off);
            if constexpr (X3)
                *reinterpret_cast<uint4*>(sA + (BM + row) * kRowW + 4 * c4) = *reinterpret_cast<const uint4*>(qy_lo + off);
        }
        // ---- stage B (P columns, x side)
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = t + NT * i;
            const int row = c >> 3, c4 = c & 7;
            const int64_t xg = min(x0 + row, a.nx - 1);
            const int64_t off = xg * ldp + j0 + 4 * c4;
            if constexpr (D3) {
                const float4* ex = reinterpret_cast<const float4*>(static_cast<const float2*>(a.px) + off);
                const float4* ez = reinterpret_cast<const float4*>(a.ez + z0 * ldp + j0 + 4 * c4);
                const float4 e01 = ex[0], e23 = ex[1], z01 = ez[0], z23 = ez[1];
                // P = Ex * Ez, stored as (Re P, -Im P)
                const float pr[4] = {e01.x * z01.x - e01.y * z01.y, e01.z * z01.z - e01.w * z01.w,
                                     e23.x * z23.x - e23.y * z23.y, e23.z * z23.z - e23.w * z23.w};
                const float pi[4] = {-(e01.x * z01.y + e01.y * z01.x), -(e01.z * z01.w + e01.w * z01.z),
                                     -(e23.x * z23.y + e23.y * z23.x), -(e23.z * z23.w + e23.w * z23.z)};
                uint4 hi, lo;
                uint32_t* h = reinterpret_cast<uint32_t*>(&hi);
                uint32_t* o = reinterpret_cast<uint32_t*>(&lo);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    h[m] = pack_pair(pr[m], pi[m], BF);
                    if constexpr (X3) o[m] = pack_pair(pr[m] - lo16f(h[m], BF), pi[m] - hi16f(h[m], BF), BF);
                }
                *reinterpret_cast<uint4*>(sB + row * kRowW + 4 * c4) = hi;
                if constexpr (X3) *reinterpret_cast<uint4*>(sB + (BN + row) * kRowW + 4 * c4) = lo;
            } else {
                const uint32_t* px = static_cast<const uint32_t*>(a.px);
                *reinterpret_cast<uint4*>(sB + row * kRowW + 4 * c4) = *reinterpret_cast<const uint4*>(px + off);
                if constexpr (X3) {
                    const uint32_t* pl = static_cast<const uint32_t*>(a.px_lo);
                    *reinterpret_cast<uint4*>(sB + (BN + row) * kRowW + 4 * c4) = *reinterpret_cast<const uint4*>(pl + off);
                }
            }
        }
        __syncthreads();

        // ---- MFMA over the stage: 4 k-steps of 8 modes (16 reals)
#pragma unroll
        for (int ks = 0; ks < kJC / 8; ++ks) {
            const int kw = 8 * ks + 4 * (l >> 5);
            uint4 fa[TM], fb[TN];
            uint4 fal[X3 ? TM : 1], fbl[X3 ? TN : 1];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = (wm * TM + i) * 32 + (l & 31);
                fa[i] = *reinterpret_cast<const uint4*>(sA + row * kRowW + kw);
                if constexpr (X3) fal[i] = *reinterpret_cast<const uint4*>(sA + (BM + row) * kRowW + kw);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int col = (wn * TN + j) * 32 + (l & 31);
                fb[j] = *reinterpret_cast<const uint4*>(sB + col * kRowW + kw);
                if constexpr (X3) fbl[j] = *reinterpret_cast<const uint4*>(sB + (BN + col) * kRowW + kw);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    acc[i][j] = mfma<BF>(fa[i], fb[j], acc[i][j]);
                    if constexpr (X3) {
                        acc[i][j] = mfma<BF>(fa[i], fbl[j], acc[i][j]);
                        acc[i][j] = mfma<BF>(fal[i], fb[j], acc[i][j]);
                    }
                }
        }
        __syncthreads();
    }

    // ---- epilogue: D[row][col], lane holds rows 8(e/4) + 4(l/32) + e%4, col l%32
    const int64_t plane = z0 * a.ny * a.nx;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t x = x0 + (wn * TN + j) * 32 + (l & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t y = y0 + (wm * TM + i) * 32 + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
                if (x < a.nx && y < a.ny) {
                    const int64_t c = plane + y * a.nx + x;
                    const float yv = a.amp * acc[i][j][e];
                    if (a.y) a.y[c] = yv;
                    if (a.k) a.k[c] = expf(a.epi.mu + yv);
                    if (a.ind) {
                        int f = 0;
                        for (int q = 0; q < a.epi.nthr; ++q) f += (yv > a.epi.thr[q]) ? 1 : 0;
                        a.ind[c] = static_cast<uint8_t>(f);
                    }
                }
            }
        }
}

struct TileCfg {
    int bm, bn;
};
// tile selectors: 0 = 128x128 (4 waves), 1 = 256x256 (8 waves), 2 = 64x64 (4 waves), 3 = 128x256 (8 waves)
constexpr TileCfg kTiles[] = {{128, 128}, {256, 256}, {64, 64}, {128, 256}};

template <bool BF, bool X3, bool D3>
hipError_t launch_t(const SepArgs& a, int tile, hipStream_t s)
{
    const int bm = kTiles[tile].bm, bn = kTiles[tile].bn;
    const int tiles_x = static_cast<int>((a.nx + bn - 1) / bn);
    const int tiles_y = static_cast<int>((a.ny + bm - 1) / bm);
    const int64_t blocks = static_cast<int64_t>(tiles_x) * tiles_y * a.nz;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g(static_cast<unsigned>(blocks));
    switch (tile) {
    case 0:
        hipLaunchKernelGGL((k_sep<2, 2, 2, 2, BF, X3, D3>), g, dim3(256), 0, s, a, tiles_x, tiles_y);
        break;
    case 1:
        hipLaunchKernelGGL((k_sep<2, 4, 4, 2, BF, X3, D3>), g, dim3(512), 0, s, a, tiles_x, tiles_y);
        break;
    case 2:
        hipLaunchKernelGGL((k_sep<2, 2, 1, 1, BF, X3, D3>), g, dim3(256), 0, s, a, tiles_x, tiles_y);
        break;
    default:
        hipLaunchKernelGGL((k_sep<2, 4, 2, 2, BF, X3, D3>), g, dim3(512), 0, s, a, tiles_x, tiles_y);
        break;
    }
    return hipGetLastError();
}

template <bool BF, bool X3>
hipError_t launch_d(const SepArgs& a, int tile, hipStream_t s)
{
    return a.ez ? launch_t<BF, X3, true>(a, tile, s) : launch_t<BF, X3, false>(a, tile, s);
}

}  // namespace

int sep_tile_count() { return static_cast<int>(sizeof(kTiles) / sizeof(kTiles[0])); }

void sep_tile_shape(int tile, int* bm, int* bn)
{
    *bm = kTiles[tile].bm;
    *bn = kTiles[tile].bn;
}

hipError_t launch_sep(const SepArgs& a, hipStream_t s)
{
    int tile = a.tile;
    if (tile < 0 || tile >= sep_tile_count()) return hipErrorInvalidValue;
    switch (a.method) {
    case GRF_SEP_BF16: return launch_d<true, false>(a, tile, s);
    case GRF_SEP_F16: return launch_d<false, false>(a, tile, s);
    case GRF_SEP_BF16_X3: return launch_d<true, true>(a, tile, s);
    case GRF_SEP_F16_X3: return launch_d<false, true>(a, tile, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace grf
