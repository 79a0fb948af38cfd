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
//
// Pipeline: global loads for stage s+1 are issued into registers before the MFMAs of
// stage s; the 3-D operand P_z = Ex * Ez[z] is formed from those registers while they
// are written to the other LDS buffer (double-buffered when both copies fit in LDS).
#include <hip/hip_runtime.h>

#include "grf_internal.h"

namespace grf {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

constexpr int kJC = 32;         // modes per LDS stage (64 reals of K)
constexpr int kRowW = kJC + 4;  // padded LDS row, in 32-bit words

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

// LDS words one tile shape needs (NBUF stages of hi (+ lo) A and B rows).
template <int WM, int WN, int TM, int TN, bool X3>
struct SepShape {
    static constexpr int NT = WM * WN * 64;
    static constexpr int BM = WM * TM * 32;  // y rows per tile
    static constexpr int BN = WN * TN * 32;  // x cols per tile
    static constexpr int NB = X3 ? 2 : 1;    // hi (+ lo) copies
    static constexpr int STAGE_W = NB * (BM + BN) * kRowW;  // words per LDS stage
    static constexpr int NBUF = (2 * STAGE_W * 4 <= 160 * 1024) ? 2 : 1;
    static constexpr int LDS_WORDS = NBUF * STAGE_W;
};

// One output tile (rows y0.., cols x0.., slice z0) of the separable contraction.
// WM x WN waves; each wave owns TM x TN MFMA tiles of 32x32 (rows y, cols x).
// `smem` must hold SepShape<...>::LDS_WORDS words.  Called by whole blocks.
template <int WM, int WN, int TM, int TN, bool BF, bool X3, bool D3>
__device__ __forceinline__ void sep_tile(const SepArgs& a, int64_t tx, int64_t ty, int64_t z0, uint4* smem)
{
    using S = SepShape<WM, WN, TM, TN, X3>;
    constexpr int NT = S::NT, BM = S::BM, BN = S::BN, NB = S::NB, STAGE_W = S::STAGE_W, NBUF = S::NBUF;
    constexpr int CA = BM * (kJC / 4) / NT;  // 16-byte chunks of A per thread
    constexpr int CB = BN * (kJC / 4) / NT;
    static_assert(CA * NT == BM * kJC / 4 && CB * NT == BN * kJC / 4, "tile/thread mismatch");
    static_assert(NT % 8 == 0, "a thread's chunk column must not change across its chunks");

    const int t = threadIdx.x;
    const int wave = t >> 6, l = t & 63;
    const int wm = wave / WN, wn = wave % WN;
    const int64_t x0 = tx * BN, y0 = ty * BM;
    const int64_t ldp = a.ldp;
    const int c4 = t & 7;  // this thread's 4-mode chunk within a stage (same for all its chunks)

    const uint32_t* qy = static_cast<const uint32_t*>(a.qy);
    const uint32_t* qy_lo = static_cast<const uint32_t*>(a.qy_lo);

    // global row offsets of this thread's chunks
    // Operand tables are stage-major, [ldp / 32][rows][32]: stage j0 of row r starts at
    // j0 * rows + r * 32, so a stage of consecutive rows is one contiguous run.
    constexpr bool PK = D3 && !X3 && !BF;  // one-pass fp16 3-D: Ez in half pairs, packed fp16 product
    // Many tiles read the same operand rows at the same time (every z-slice shares Q and Ex).
    // Each tile visits its rows in a rotated order so that concurrent requests from different
    // CUs land on different cache lines (and L2 channels) instead of queueing on one.
    const int rot = static_cast<int>((z0 * 37 + tx * 11 + ty * 5) & 31) * 8;  // rows, multiple of 8
    int rowa[CA], rowb[CB];
#pragma unroll
    for (int i = 0; i < CA; ++i) rowa[i] = (((t + NT * i) >> 3) + rot) % BM;
#pragma unroll
    for (int i = 0; i < CB; ++i) rowb[i] = (((t + NT * i) >> 3) + rot) % BN;
    int64_t offa[CA], offb[CB];
#pragma unroll
    for (int i = 0; i < CA; ++i) offa[i] = min(y0 + rowa[i], a.ny - 1) * kJC + 4 * c4;
#pragma unroll
    for (int i = 0; i < CB; ++i) offb[i] = min(x0 + rowb[i], a.nx - 1) * kJC + 4 * c4;

    // Raw global data of one stage held by this thread: CA chunks (4 modes each) of A, CB of B;
    // 3-D: B chunks are Ex (pairs when !X3, float2 when X3) plus this thread's Ez chunk.
    uint4 ra[CA], ral[X3 ? CA : 1], rb[D3 && X3 ? 2 * CB : CB], rbl[!D3 && X3 ? CB : 1];
    float4 rez0 = make_float4(0.f, 0.f, 0.f, 0.f), rez1 = rez0;
    uint4 rezh = make_uint4(0u, 0u, 0u, 0u);

    auto load = [&](int64_t j0) {
        const int64_t sa = j0 * a.ny, sb = j0 * a.nx;
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            ra[i] = *reinterpret_cast<const uint4*>(qy + sa + offa[i]);
            if constexpr (X3) ral[i] = *reinterpret_cast<const uint4*>(qy_lo + sa + offa[i]);
        }
        if constexpr (D3) {
            if constexpr (PK) {
                rezh = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint32_t*>(a.ez) + z0 * ldp + j0 + 4 * c4);
            } else {
                const float4* ez = reinterpret_cast<const float4*>(a.ez + z0 * ldp + j0 + 4 * c4);
                rez0 = ez[0];
                rez1 = ez[1];
            }
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                if constexpr (X3) {
                    const uint4* ex = reinterpret_cast<const uint4*>(static_cast<const float2*>(a.px) + sb + offb[i]);
                    rb[2 * i] = ex[0];
                    rb[2 * i + 1] = ex[1];
                } else {
                    rb[i] = *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.px) + sb + offb[i]);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                rb[i] = *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.px) + sb + offb[i]);
                if constexpr (X3) rbl[i] = *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(a.px_lo) + sb + offb[i]);
            }
        }
    };

    auto store = [&](uint32_t* sA) {
        uint32_t* sB = sA + NB * BM * kRowW;
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int row = rowa[i];
            *reinterpret_cast<uint4*>(sA + row * kRowW + 4 * c4) = ra[i];
            if constexpr (X3) *reinterpret_cast<uint4*>(sA + (BM + row) * kRowW + 4 * c4) = ral[i];
        }
        // packed fp16 factors of this thread's Ez chunk: P' = er (zr, -zi) + ei (zi, zr)
        h2 z1[4], z2[4];
        if constexpr (PK) {
            const uint32_t zw[4] = {rezh.x, rezh.y, rezh.z, rezh.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const h2 z = __builtin_bit_cast(h2, zw[m]);
                z1[m] = h2{z.x, static_cast<_Float16>(-z.y)};
                z2[m] = h2{z.y, z.x};
            }
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int row = rowb[i];
            if constexpr (PK) {
                const uint32_t w[4] = {rb[i].x, rb[i].y, rb[i].z, rb[i].w};
                uint32_t h[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const h2 e = __builtin_bit_cast(h2, w[m]);  // (Re Ex, -Im Ex)
                    const h2 p = h2{e.x, e.x} * z1[m] + h2{e.y, e.y} * z2[m];
                    h[m] = __builtin_bit_cast(uint32_t, p);
                }
                *reinterpret_cast<uint4*>(sB + row * kRowW + 4 * c4) = make_uint4(h[0], h[1], h[2], h[3]);
            } else if constexpr (D3) {
                // P = Ex * Ez, stored as (Re P, -Im P); Ex arrives as (Re, -Im)
                float er[4], ei[4];
                if constexpr (X3) {
                    const float4 e01 = __builtin_bit_cast(float4, rb[2 * i]);
                    const float4 e23 = __builtin_bit_cast(float4, rb[2 * i + 1]);
                    er[0] = e01.x; ei[0] = e01.y; er[1] = e01.z; ei[1] = e01.w;
                    er[2] = e23.x; ei[2] = e23.y; er[3] = e23.z; ei[3] = e23.w;
                } else {
                    const uint4 w = rb[i];
                    er[0] = lo16f(w.x, BF); ei[0] = hi16f(w.x, BF);
                    er[1] = lo16f(w.y, BF); ei[1] = hi16f(w.y, BF);
                    er[2] = lo16f(w.z, BF); ei[2] = hi16f(w.z, BF);
                    er[3] = lo16f(w.w, BF); ei[3] = hi16f(w.w, BF);
                }
                const float zr[4] = {rez0.x, rez0.z, rez1.x, rez1.z};
                const float zi[4] = {rez0.y, rez0.w, rez1.y, rez1.w};
                uint32_t h[4], o[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    // (er + i ei)(zr + i zi) with ei holding -Im Ex: Re P = er zr + ei zi, -Im P = ei zr - er zi
                    const float pr = er[m] * zr[m] + ei[m] * zi[m];
                    const float pi = ei[m] * zr[m] - er[m] * zi[m];
                    h[m] = pack_pair(pr, pi, BF);
                    if constexpr (X3) o[m] = pack_pair(pr - lo16f(h[m], BF), pi - hi16f(h[m], BF), BF);
                    else o[m] = 0u;
                }
                *reinterpret_cast<uint4*>(sB + row * kRowW + 4 * c4) = make_uint4(h[0], h[1], h[2], h[3]);
                if constexpr (X3)
                    *reinterpret_cast<uint4*>(sB + (BN + row) * kRowW + 4 * c4) = make_uint4(o[0], o[1], o[2], o[3]);
            } else {
                *reinterpret_cast<uint4*>(sB + row * kRowW + 4 * c4) = rb[i];
                if constexpr (X3) *reinterpret_cast<uint4*>(sB + (BN + row) * kRowW + 4 * c4) = rbl[i];
            }
        }
    };

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

    auto compute = [&](const uint32_t* sA) {
        const uint32_t* sB = sA + NB * BM * kRowW;
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
    };

    uint32_t* sbase = reinterpret_cast<uint32_t*>(smem);
    load(0);
    store(sbase);
    __syncthreads();
    const int64_t nstage = ldp / kJC;
    // Loads and stores are unconditional (the last iteration re-stages the last stage into
    // the idle buffer) so that the prefetch registers stay in registers.
    for (int64_t s = 0; s < nstage; ++s) {
        uint32_t* cur = sbase + (NBUF == 2 ? (s & 1) * STAGE_W : 0);
        load(min(s + 1, nstage - 1) * kJC);
        compute(cur);
        if constexpr (NBUF == 1) __syncthreads();
        store(sbase + (NBUF == 2 ? ((s + 1) & 1) * STAGE_W : 0));
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

template <int WM, int WN, int TM, int TN, bool BF, bool X3, bool D3>
__global__ __launch_bounds__(WM* WN * 64) void k_sep(SepArgs a, int tiles_x, int tiles_y)
{
    __shared__ uint4 smem[SepShape<WM, WN, TM, TN, X3>::LDS_WORDS / 4];
    const int64_t bid = blockIdx.x;
    const int64_t rest = bid / tiles_x;
    sep_tile<WM, WN, TM, TN, BF, X3, D3>(a, bid % tiles_x, rest % tiles_y, rest / tiles_y, smem);
}

// Persistent batched form: blocks pull (instance, tile, slice) work items from one atomic
// counter until the queue is drained (every block exits when the counter passes `total`).
// Instances are ordered by descending tile cost on the host; each instance uses the
// 128x128 (variant 0) or 64x64 (variant 1) tile the plan picked for its size class.
using BigT = SepShape<2, 2, 2, 2, false>;
using BigT3 = SepShape<2, 2, 2, 2, true>;
using SmallT = SepShape<2, 2, 1, 1, false>;
using SmallT3 = SepShape<2, 2, 1, 1, true>;

template <bool BF, bool X3, bool D3>
__global__ __launch_bounds__(256) void k_sep_batch(const SepBatchItem* __restrict__ items, int n_inst, int64_t total,
                                                   unsigned long long* counter)
{
    constexpr int W0 = X3 ? BigT3::LDS_WORDS : BigT::LDS_WORDS;
    constexpr int W1 = X3 ? SmallT3::LDS_WORDS : SmallT::LDS_WORDS;
    __shared__ uint4 smem[(W0 > W1 ? W0 : W1) / 4];
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
        const SepBatchItem& b = items[lo];
        const int64_t local = it - b.item0;
        const int64_t rest = local / b.tiles_x;
        if (b.variant == 0)
            sep_tile<2, 2, 2, 2, BF, X3, D3>(b.a, local % b.tiles_x, rest % b.tiles_y, rest / b.tiles_y, smem);
        else
            sep_tile<2, 2, 1, 1, BF, X3, D3>(b.a, local % b.tiles_x, rest % b.tiles_y, rest / b.tiles_y, smem);
    }
}

template <bool BF, bool X3, bool D3>
hipError_t launch_batch_t(const SepBatchItem* items, int n_inst, int64_t total, unsigned long long* counter, int grid,
                          hipStream_t s)
{
    hipLaunchKernelGGL((k_sep_batch<BF, X3, D3>), dim3(grid), dim3(256), 0, s, items, n_inst, total, counter);
    return hipGetLastError();
}

template <bool BF, bool X3, bool D3>
int batch_occupancy_t()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sep_batch<BF, X3, D3>, 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

struct TileCfg {
    int bm, bn;
};
// tile selectors: 0 = 256x256 (8 waves), 1 = 128x128 (4 waves), 2 = 64x64 (4 waves), 3 = 128x256 (8 waves),
// 4 = 256x256 (4 waves of 128x128)
constexpr TileCfg kTiles[] = {{256, 256}, {128, 128}, {64, 64}, {128, 256}, {256, 256}};

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
        hipLaunchKernelGGL((k_sep<2, 4, 4, 2, BF, X3, D3>), g, dim3(512), 0, s, a, tiles_x, tiles_y);
        break;
    case 1:
        hipLaunchKernelGGL((k_sep<2, 2, 2, 2, BF, X3, D3>), g, dim3(256), 0, s, a, tiles_x, tiles_y);
        break;
    case 2:
        hipLaunchKernelGGL((k_sep<2, 2, 1, 1, BF, X3, D3>), g, dim3(256), 0, s, a, tiles_x, tiles_y);
        break;
    case 3:
        hipLaunchKernelGGL((k_sep<2, 4, 2, 2, BF, X3, D3>), g, dim3(512), 0, s, a, tiles_x, tiles_y);
        break;
    default:
        hipLaunchKernelGGL((k_sep<2, 2, 4, 4, BF, X3, D3>), g, dim3(256), 0, s, a, tiles_x, tiles_y);
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

int sep_default_tile(int method, int64_t nx, int64_t ny, int64_t nz)
{
    // Large slices: 256x256 (operand reuse), or 128x256 for the hi+lo forms whose doubled
    // LDS stages do not fit twice at 256x256; small or thin grids: smaller tiles keep the
    // device busy and waste less on ragged edges.
    const int64_t t256 = ((nx + 255) / 256) * ((ny + 255) / 256) * nz;
    if (nx >= 192 && ny >= 192 && t256 >= 128) return (method == GRF_SEP_F16_X3 || method == GRF_SEP_BF16_X3) ? 3 : 0;
    const int64_t t128 = ((nx + 127) / 128) * ((ny + 127) / 128) * nz;
    if (nx >= 96 && ny >= 96 && t128 >= 64) return 1;
    return 2;
}

hipError_t launch_sep_batch(int method, bool d3, const SepBatchItem* items, int n_inst, int64_t total,
                            unsigned long long* counter, int grid, hipStream_t s)
{
    switch (method) {
    case GRF_SEP_BF16:
        return d3 ? launch_batch_t<true, false, true>(items, n_inst, total, counter, grid, s)
                  : launch_batch_t<true, false, false>(items, n_inst, total, counter, grid, s);
    case GRF_SEP_F16:
        return d3 ? launch_batch_t<false, false, true>(items, n_inst, total, counter, grid, s)
                  : launch_batch_t<false, false, false>(items, n_inst, total, counter, grid, s);
    case GRF_SEP_BF16_X3:
        return d3 ? launch_batch_t<true, true, true>(items, n_inst, total, counter, grid, s)
                  : launch_batch_t<true, true, false>(items, n_inst, total, counter, grid, s);
    case GRF_SEP_F16_X3:
        return d3 ? launch_batch_t<false, true, true>(items, n_inst, total, counter, grid, s)
                  : launch_batch_t<false, true, false>(items, n_inst, total, counter, grid, s);
    default: return hipErrorInvalidValue;
    }
}

int sep_batch_blocks_per_cu(int method, bool d3)
{
    switch (method) {
    case GRF_SEP_BF16: return d3 ? batch_occupancy_t<true, false, true>() : batch_occupancy_t<true, false, false>();
    case GRF_SEP_F16: return d3 ? batch_occupancy_t<false, false, true>() : batch_occupancy_t<false, false, false>();
    case GRF_SEP_BF16_X3: return d3 ? batch_occupancy_t<true, true, true>() : batch_occupancy_t<true, true, false>();
    default: return d3 ? batch_occupancy_t<false, true, true>() : batch_occupancy_t<false, true, false>();
    }
}

hipError_t launch_sep(const SepArgs& a, hipStream_t s)
{
    int tile = a.tile < 0 ? sep_default_tile(a.method, a.nx, a.ny, a.nz) : a.tile;
    if (tile >= sep_tile_count()) return hipErrorInvalidValue;
    switch (a.method) {
    case GRF_SEP_BF16: return launch_d<true, false>(a, tile, s);
    case GRF_SEP_F16: return launch_d<false, false>(a, tile, s);
    case GRF_SEP_BF16_X3: return launch_d<true, true>(a, tile, s);
    case GRF_SEP_F16_X3: return launch_d<false, true>(a, tile, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace grf
