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
// Pipeline: the operands of stage s+1 (32 modes) are loaded while the MFMAs consume stage s
// from the other LDS buffer.  Most forms load straight into LDS; the 3-D forms that need
// FP32 products (bf16, hi+lo) stage through registers and form P_z = Ex * Ez[z] there.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "grf_internal.h"

namespace grf {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// P' = (Re P, -Im P) of P = Ex Ez in packed fp16, from e = (Re Ex, -Im Ex) and z = (Re Ez, Im Ez):
// (ex zr + ey zi, ey zr - ex zi) = (ex, -ex) * z + (ey, ey) * (zi, zr), written with vector
// shuffles so that the broadcasts, the sign and the swap become operand modifiers of one
// v_pk_mul_f16 and one v_pk_fma_f16.
__device__ __forceinline__ uint32_t ez_prod(uint32_t ew, uint32_t zw)
{
    const h2 e = __builtin_bit_cast(h2, ew);
    const h2 z = __builtin_bit_cast(h2, zw);
    const h2 ne = -e;
    const h2 t = __builtin_shufflevector(e, ne, 0, 2) * z;
    const h2 zs = __builtin_shufflevector(z, z, 1, 0);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_fma(__builtin_shufflevector(e, e, 1, 1), zs, t));
}

constexpr int kJC = 32;         // modes per LDS stage (64 reals of K)
constexpr int kRowW = kJC + 4;  // padded LDS row, in 32-bit words

// (re, im) rounded to nearest-even fp16 / bf16 and packed (re low): one v_cvt_pk_f16_f32 /
// v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint32_t pack_pair(float re, float im, bool bf)
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const f2 v = {re, im};
    if (bf) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2));
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

// exp(x) for the log-normal stores of interior tiles: 2^t with t = x log2(e) carried as an
// exact FMA split t_hi + t_lo, the hardware base-2 exponential of t_hi and a first-order
// correction for t_lo (|t_lo| <= 2^-24 |t|).  Error: that of v_exp_f32 plus ~1 ulp, i.e. a few
// ulp; inf above ~88.7, 0 far below -87, NaN in, NaN out.
__device__ __forceinline__ float exp_split(float x)
{
    constexpr float kLog2e = 1.44269502162933349609375f;  // log2(e) rounded to FP32
    constexpr float kLog2eLo = 1.925963033500011e-08f;    // log2(e) - kLog2e
    constexpr float kLn2 = 0.693147180559945309f;
    const float th = x * kLog2e;
    const float tl = fmaf(x, kLog2eLo, fmaf(x, kLog2e, -th));
    const float e = __builtin_amdgcn_exp2f(th);
    return fmaf(e, tl * kLn2, e);
}

// Epilogue of one wave for one z-slice: D[row][col] of its TM x TN accumulator tiles, lane
// holding rows 8(e/4) + 4(l/32) + e%4 and column l%32 of each 32x32 tile; the wave's tiles
// start at row y0 + r0 and column x0 + c0 of the plane's cells (plane + y nx + x).  A block
// tile (BM x BN at y0, x0) that lies inside the grid and writes one FP32 output (Y or K)
// branches once and stores through a uniform row base plus 32-bit lane offsets (K by
// exp_split); otherwise every cell is bounds-checked and goes through epi_store.  FAST =
// false keeps the per-cell form only (the widest per-wave tiles: their accumulators leave no
// registers for the other).
template <int TM, int TN, int BM, int BN, bool FAST>
__device__ __forceinline__ void store_tiles(const SepArgs& a, const Epi& epi, int64_t plane, int64_t x0, int64_t y0,
                                            int r0, int c0, int l, const f32x16 (&acc)[TM][TN])
{
    const int h = l >> 5;
    const int only = (a.ind || (a.y && a.k)) ? 0 : (a.k ? 2 : (a.y ? 1 : 0));
    if (FAST && only != 0 && x0 + BN <= a.nx && y0 + BM <= a.ny && a.nx < (int64_t(1) << 22)) {
        // byte offsets below 2^32: rows < 256 and nx < 2^22
        __attribute__((address_space(1))) char* const out =
            (__attribute__((address_space(1))) char*)((only == 2 ? a.k : a.y) + plane + y0 * a.nx + x0);
        const uint32_t nxb = static_cast<uint32_t>(a.nx) * 4u;
        auto cell = [&](int i, int j, int e) {
            const uint32_t lo = static_cast<uint32_t>(r0 + i * 32 + 4 * h + 8 * (e >> 2) + (e & 3)) * nxb +
                                static_cast<uint32_t>((c0 + j * 32 + (l & 31)) * 4);
            return (__attribute__((address_space(1))) float*)(out + lo);
        };
        if (only == 2) {
#pragma clang fp contract(off)  // Y rounded before mu is added, as in the per-cell path
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e) *cell(i, j, e) = exp_split(epi.mu + a.amp * acc[i][j][e]);
        } else {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int e = 0; e < 16; ++e) *cell(i, j, e) = a.amp * acc[i][j][e];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t x = x0 + c0 + j * 32 + (l & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t y = y0 + r0 + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                if (x < a.nx && y < a.ny) epi_store(plane + y * a.nx + x, a.amp * acc[i][j][e], epi, a.y, a.k, a.ind);
            }
        }
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

// One output tile (rows y0.., cols x0.., slice z0) of the separable contraction, with the
// operand stages staged through registers (used where the B operand needs FP32 arithmetic:
// the 3-D bf16 and hi+lo forms).
// WM x WN waves; each wave owns TM x TN MFMA tiles of 32x32 (rows y, cols x).
// `smem` must hold SepShape<...>::LDS_WORDS words.  Called by whole blocks.
template <int WM, int WN, int TM, int TN, bool BF, bool X3, bool D3>
__device__ __forceinline__ void sep_tile_reg(const SepArgs& a, const Epi& epi, int64_t tx, int64_t ty, int64_t z0,
                                             uint4* smem, int64_t s0, int64_t s1)
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
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int row = rowb[i];
            if constexpr (PK) {
                // packed fp16 product with this thread's Ez chunk
                *reinterpret_cast<uint4*>(sB + row * kRowW + 4 * c4) =
                    make_uint4(ez_prod(rb[i].x, rezh.x), ez_prod(rb[i].y, rezh.y), ez_prod(rb[i].z, rezh.z),
                               ez_prod(rb[i].w, rezh.w));
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
    load(s0 * kJC);
    store(sbase);
    __syncthreads();
    // Stages [s0, s1), s0 even.  Loads and stores are unconditional (the last iteration
    // re-stages the last stage into the idle buffer) so that the prefetch registers stay in
    // registers.
    for (int64_t s = s0; s < s1; ++s) {
        uint32_t* cur = sbase + (NBUF == 2 ? (s & 1) * STAGE_W : 0);
        load(min(s + 1, s1 - 1) * kJC);
        compute(cur);
        if constexpr (NBUF == 1) __syncthreads();
        store(sbase + (NBUF == 2 ? ((s + 1) & 1) * STAGE_W : 0));
        __syncthreads();
    }

    store_tiles<TM, TN, WM * TM * 32, WN * TN * 32, TM * TN <= 8>(a, epi, z0 * a.ny * a.nx, x0, y0, wm * TM * 32,
                                                                  wn * TN * 32, l, acc);
}

// ---- direct-to-LDS staging -------------------------------------------------------------
//
// Operand stages go from global memory straight into LDS (global_load_lds_dwordx4: the 64
// lanes of one instruction fill one contiguous 1 KiB run, lane l at byte 16 l), so no
// registers, LDS stores or waits sit between a prefetch and the MFMAs.  LDS rows are
// unpadded (one stage of one table row = 32 words = 8 chunks of 16 bytes); chunk c of row r
// lives at chunk c ^ swz(r) of that row, which puts the 16 lanes of a fragment read (16
// consecutive rows, one logical chunk) on distinct banks.  The two stage buffers are
// separate LDS objects so that waits for the buffer in flight do not land on reads of the
// other one.  In 3-D the one-pass fp16 operand P_z = Ex * Ez[z] is formed on the B
// fragments in registers (packed fp16), and a block may cover ZS consecutive z-slices that
// share every A and Ex fragment it reads.
typedef __attribute__((address_space(3))) void lds_void;
typedef const __attribute__((address_space(1))) void gbl_void;

__device__ __forceinline__ int swz(int r) { return (r ^ (r >> 3)) & 7; }

__device__ __forceinline__ void load_to_lds(const uint32_t* g, char* s)
{
    __builtin_amdgcn_global_load_lds((gbl_void*)g, (lds_void*)s, 16, 0, 0);
}

// The same from a uniform base plus an unsigned 32-bit byte offset.
__device__ __forceinline__ void load_to_lds_b(const char* base, uint32_t off, char* s)
{
    __builtin_amdgcn_global_load_lds((gbl_void*)(base + off), (lds_void*)s, 16, 0, 0);
}

__device__ __forceinline__ void wait_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// LDS stage: A rows (hi, lo), B rows (hi, lo), then EZR rows of Ez (one per z-slice, 3-D).
template <int WM, int WN, int TM, int TN, bool X3, int EZR>
struct DlShape {
    static constexpr int NW = WM * WN;
    static constexpr int BM = WM * TM * 32, BN = WN * TN * 32;
    static constexpr int NB = X3 ? 2 : 1;
    static constexpr int ROW_B = kJC * 4;  // bytes of one stage of one table row
    static constexpr int EZ_OFF = NB * (BM + BN) * ROW_B;
    static constexpr int STAGE_B = EZ_OFF + EZR * ROW_B;
    static constexpr bool FITS = 2 * STAGE_B <= 160 * 1024 && (BM / 8) % NW == 0 && (BN / 8) % NW == 0;
};

// Forms that stage directly into LDS: every table reaches the MFMAs unchanged, except the
// one-pass fp16 3-D product, which is formed in packed fp16 on the fragments.
template <int WM, int WN, int TM, int TN, int ZS, bool BF, bool X3, bool D3>
constexpr bool use_dl()
{
    return DlShape<WM, WN, TM, TN, X3, D3 ? ZS : 0>::FITS && !(D3 && (X3 || BF));
}

// One output tile (rows y0.., cols x0.., slices zb*ZS .. zb*ZS+ZS-1) with direct-to-LDS
// staging, summed over the mode stages [s0, s1) (s0 and s1 even).  `lds0` and `lds1` each hold
// DlShape<..., D3 ? ZS : 0>::STAGE_B bytes.  Called by whole blocks.
template <int WM, int WN, int TM, int TN, int ZS, bool BF, bool X3, bool D3>
__device__ __forceinline__ void sep_tile_dl(const SepArgs& a, const Epi& epi, int64_t tx, int64_t ty, int64_t zb, uint4* lds0,
                                            uint4* lds1, int64_t s0, int64_t s1)
{
    using S = DlShape<WM, WN, TM, TN, X3, D3 ? ZS : 0>;
    constexpr int BM = S::BM, BN = S::BN, NB = S::NB, ROW_B = S::ROW_B, NW = S::NW, EZ_OFF = S::EZ_OFF;
    constexpr int KA = BM / 8 / NW, KB = BN / 8 / NW;  // 1 KiB load instructions per wave and stage
    static_assert(!D3 || (!X3 && !BF), "3-D direct staging is the one-pass fp16 form");
    static_assert(D3 || ZS == 1, "2-D tiles cover one slice");

    const int l = threadIdx.x & 63, h = l >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int wm = wave / WN, wn = wave % WN;
    const int64_t x0 = tx * BN, y0 = ty * BM, z0 = zb * ZS;
    const int64_t ldp = a.ldp;

    const uint32_t* qy = static_cast<const uint32_t*>(a.qy);
    const uint32_t* qy_lo = static_cast<const uint32_t*>(a.qy_lo);
    const uint32_t* px = static_cast<const uint32_t*>(a.px);
    const uint32_t* px_lo = static_cast<const uint32_t*>(a.px_lo);

    // Load assignment: instruction k of this wave fills LDS rows 8 rb .. 8 rb + 7 of its
    // operand.  Tiles start at rotated row blocks so that concurrent requests of different
    // CUs (every z-slice reads the same Q and Ex rows) spread over cache lines and channels.
    const int rot = static_cast<int>((zb * 37 + tx * 11 + ty * 5) & 31);
    // byte offsets from the stage's uniform table base (32-bit and unsigned, so the loads take
    // the scalar-base address form: one register per load and no 64-bit address arithmetic)
    uint32_t offa[KA], offb[KB];
    int lda[KA], ldb[KB];
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        const int rb = (wave * KA + k + rot) & (BM / 8 - 1);
        const int row = rb * 8 + (l >> 3);
        offa[k] = static_cast<uint32_t>(min(y0 + row, a.ny - 1) * kJC + 4 * ((l & 7) ^ swz(row))) * 4u;
        lda[k] = rb * 8 * ROW_B;
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int rb = (wave * KB + k + rot) & (BN / 8 - 1);
        const int row = rb * 8 + (l >> 3);
        offb[k] = static_cast<uint32_t>(min(x0 + row, a.nx - 1) * kJC + 4 * ((l & 7) ^ swz(row))) * 4u;
        ldb[k] = rb * 8 * ROW_B;
    }

    // 3-D: lanes 0 .. 8 ZS - 1 of wave 0 also stage the Ez words (half pairs) of the z-slices
    const uint32_t* ezl =
        D3 ? reinterpret_cast<const uint32_t*>(a.ez) + min(z0 + (l >> 3), a.nz - 1) * ldp + 4 * (l & 7) : nullptr;

    auto issue = [&](int64_t j0, char* buf) {
        if constexpr (D3) {
            if (wave == 0 && l < 8 * ZS) load_to_lds(ezl + j0, buf + EZ_OFF);
        }
        const char* sa = reinterpret_cast<const char*>(qy + j0 * a.ny);
#pragma unroll
        for (int k = 0; k < KA; ++k) load_to_lds_b(sa, offa[k], buf + lda[k]);
        if constexpr (X3) {
            const char* sl = reinterpret_cast<const char*>(qy_lo + j0 * a.ny);
#pragma unroll
            for (int k = 0; k < KA; ++k) load_to_lds_b(sl, offa[k], buf + BM * ROW_B + lda[k]);
        }
        const char* sb = reinterpret_cast<const char*>(px + j0 * a.nx);
#pragma unroll
        for (int k = 0; k < KB; ++k) load_to_lds_b(sb, offb[k], buf + NB * BM * ROW_B + ldb[k]);
        if constexpr (X3) {
            const char* sl = reinterpret_cast<const char*>(px_lo + j0 * a.nx);
#pragma unroll
            for (int k = 0; k < KB; ++k) load_to_lds_b(sl, offb[k], buf + (NB * BM + BN) * ROW_B + ldb[k]);
        }
    };

    // fragment rows of this lane: byte offset of the row and the chunk swizzle (with h folded in)
    int fra[TM], ga[TM], frb[TN], gb[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int row = (wm * TM + i) * 32 + (l & 31);
        fra[i] = row * ROW_B;
        ga[i] = swz(row) ^ h;
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int col = (wn * TN + j) * 32 + (l & 31);
        frb[j] = col * ROW_B;
        gb[j] = swz(col) ^ h;
    }

    f32x16 acc[ZS][TM][TN];
#pragma unroll
    for (int zs = 0; zs < ZS; ++zs)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[zs][i][j][e] = 0.f;

    // Fragments of one k-step (8 modes): A rows (hi, lo), B columns (hi, lo), Ez words.
    struct Frag {
        uint4 a[TM], al[X3 ? TM : 1], b[TN], bl[X3 ? TN : 1], ez[D3 ? ZS : 1];
    };
    auto read = [&](const char* buf, int ks, Frag& f) {
        const char* sA = buf;
        const char* sB = buf + NB * BM * ROW_B;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int o = fra[i] + (((2 * ks) ^ ga[i]) << 4);
            f.a[i] = *reinterpret_cast<const uint4*>(sA + o);
            if constexpr (X3) f.al[i] = *reinterpret_cast<const uint4*>(sA + BM * ROW_B + o);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int o = frb[j] + (((2 * ks) ^ gb[j]) << 4);
            f.b[j] = *reinterpret_cast<const uint4*>(sB + o);
            if constexpr (X3) f.bl[j] = *reinterpret_cast<const uint4*>(sB + BN * ROW_B + o);
        }
        if constexpr (D3) {
            // this lane's Ez words are modes 8 ks + 4 h .. + 3 (a broadcast read)
#pragma unroll
            for (int zs = 0; zs < ZS; ++zs)
                f.ez[zs] = *reinterpret_cast<const uint4*>(buf + EZ_OFF + zs * ROW_B + ((2 * ks + h) << 4));
        }
    };
    auto mac = [&](const Frag& f) {
        if constexpr (D3) {
#pragma unroll
            for (int zs = 0; zs < ZS; ++zs) {
                // P' = (Re P, -Im P) of P = Ex Ez on the B fragments
                const uint4 z = f.ez[zs];
                uint4 fp[TN];
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    fp[j] = make_uint4(ez_prod(f.b[j].x, z.x), ez_prod(f.b[j].y, z.y), ez_prod(f.b[j].z, z.z),
                                       ez_prod(f.b[j].w, z.w));
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[zs][i][j] = mfma<false>(f.a[i], fp[j], acc[zs][i][j]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    acc[0][i][j] = mfma<BF>(f.a[i], f.b[j], acc[0][i][j]);
                    if constexpr (X3) {
                        acc[0][i][j] = mfma<BF>(f.a[i], f.bl[j], acc[0][i][j]);
                        acc[0][i][j] = mfma<BF>(f.al[i], f.b[j], acc[0][i][j]);
                    }
                }
        }
    };
    // Two z-slices per block: each k-step is split into two fenced scheduling regions, the
    // LDS reads of the next k-step riding along the MFMAs of slice 0 and the Ez products of
    // the next k-step along the MFMAs of slice 1.  With one wave per SIMD (four-wave blocks)
    // nothing else would cover the read -> product -> MFMA chain; with two (eight-wave
    // blocks of 128 x 32 waves) it still measured ~1.5% faster than the compiler's order.
    constexpr bool PIPE = D3 && ZS == 2 && ((NW == 4 && TM * TN == 8) || (NW == 8 && TM * TN == 4));
    constexpr int NMF = TM * TN, NRD = TM + TN + ZS;
    constexpr int RPM = (NRD + NMF - 1) / NMF;  // DS reads per MFMA in the interleave
    // VALU ops of the next k-step's products (two per word, four words per fragment and slice)
    // per MFMA: spread evenly, each group fits under the MFMA before it (measured ~1% faster
    // than a looser bound that packed them behind the first MFMAs)
    constexpr int VPM = (8 * TN * ZS + NMF - 1) / NMF;
    auto prod = [&](const Frag& f, int zs, uint4(&fp)[TN]) {
        // P' = (Re P, -Im P) of P = Ex Ez on the B fragments
        const uint4 z = f.ez[zs];
#pragma unroll
        for (int j = 0; j < TN; ++j)
            fp[j] = make_uint4(ez_prod(f.b[j].x, z.x), ez_prod(f.b[j].y, z.y), ez_prod(f.b[j].z, z.z),
                               ez_prod(f.b[j].w, z.w));
    };
    auto compute_pipe = [&](const char* buf) {
        if constexpr (PIPE) {
        Frag f[2];
        uint4 fp[2][2][TN];
        read(buf, 0, f[0]);
        prod(f[0], 0, fp[0][0]);
        prod(f[0], 1, fp[0][1]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < kJC / 8; ++ks) {
            const int c = ks & 1, n = c ^ 1;
            if (ks + 1 < kJC / 8) read(buf, ks + 1, f[n]);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[0][i][j] = mfma<false>(f[c].a[i], fp[c][0][j], acc[0][i][j]);
            if (ks + 1 < kJC / 8) {
#pragma unroll
                for (int r = 0; r < NMF; ++r) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, RPM, 0);  // DS read
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            if (ks + 1 < kJC / 8) {
                prod(f[n], 0, fp[n][0]);
                prod(f[n], 1, fp[n][1]);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[1][i][j] = mfma<false>(f[c].a[i], fp[c][1][j], acc[1][i][j]);
            if (ks + 1 < kJC / 8) {
#pragma unroll
                for (int r = 0; r < NMF; ++r) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);         // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, VPM, 0);  // VALU
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        }
    };
    auto compute = [&](const char* buf) {
        if constexpr (PIPE) {
            compute_pipe(buf);
        } else {
#pragma unroll
            for (int ks = 0; ks < kJC / 8; ++ks) {
                Frag f;
                read(buf, ks, f);
                mac(f);
            }
        }
    };

    // Two stages per iteration (ldp is a multiple of 64, so the stage count is even): the
    // loads of the next stage are in flight while the current buffer feeds the MFMAs.
    char* b0 = reinterpret_cast<char*>(lds0);
    char* b1 = reinterpret_cast<char*>(lds1);
    issue(s0 * kJC, b0);
    for (int64_t s = s0; s < s1; s += 2) {
        wait_loads();
        __syncthreads();  // stage s is in b0 for every wave; every wave is done with b1
        issue((s + 1) * kJC, b1);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs it overlaps
        compute(b0);
        wait_loads();
        __syncthreads();  // stage s + 1 is in b1; every wave is done with b0
        if (s + 2 < s1) issue((s + 2) * kJC, b0);
        __builtin_amdgcn_sched_barrier(0);
        compute(b1);
    }

    // ---- epilogue: D[row][col], lane holds rows 8(e/4) + 4(l/32) + e%4, col l%32
    // Interior tiles with one FP32 output (Y or K, the latter by exp_split) branch once per
    // tile and address cells by a uniform 64-bit row base plus a 32-bit lane offset; the rest
    // check every cell.  (Not for the widest per-wave tiles: their accumulators leave no
    // registers for it.)
    constexpr bool kFastEpi = TM * TN * ZS <= 8;
    const bool interior =
        kFastEpi && x0 + BN <= a.nx && y0 + BM <= a.ny && a.nx < (int64_t(1) << 22);
    const int only = (a.ind || (a.y && a.k)) ? 0 : (a.k ? 2 : (a.y ? 1 : 0));
#pragma unroll
    for (int zs = 0; zs < ZS; ++zs) {
        if (z0 + zs >= a.nz) break;
        const int64_t plane = (z0 + zs) * a.ny * a.nx;
        if (kFastEpi && interior && only != 0) {
            // byte offsets below 2^32: rows < 256 and nx < 2^22
            char* const out = reinterpret_cast<char*>((only == 2 ? a.k : a.y) + plane + y0 * a.nx + x0);
            const uint32_t nxb = static_cast<uint32_t>(a.nx) * 4u;
            auto cell = [&](int i, int j, int e) {
                const uint32_t lo = static_cast<uint32_t>((wm * TM + i) * 32 + 4 * h + 8 * (e >> 2) + (e & 3)) * nxb +
                                    static_cast<uint32_t>(((wn * TN + j) * 32 + (l & 31)) * 4);
                return reinterpret_cast<float*>(out + lo);
            };
            if (only == 2) {
#pragma clang fp contract(off)  // Y rounded before mu is added, as in the per-cell path
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int e = 0; e < 16; ++e) *cell(i, j, e) = exp_split(epi.mu + a.amp * acc[zs][i][j][e]);
            } else {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int e = 0; e < 16; ++e) *cell(i, j, e) = a.amp * acc[zs][i][j][e];
            }
            continue;
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int64_t x = x0 + (wn * TN + j) * 32 + (l & 31);
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t y = y0 + (wm * TM + i) * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                    if (x < a.nx && y < a.ny) {
                        const int64_t c = plane + y * a.nx + x;
                        const float yv = a.amp * acc[zs][i][j][e];
                        epi_store(c, yv, epi, a.y, a.k, a.ind);
                    }
                }
            }
    }
}

// Tile body for one block: direct-to-LDS staging where the form allows it, else registers.
// ZS applies to the direct 3-D form only; the other forms cover one slice per block.
template <int WM, int WN, int TM, int TN, int ZS, bool BF, bool X3, bool D3>
constexpr int slices_per_block()
{
    return (use_dl<WM, WN, TM, TN, ZS, BF, X3, D3>() && D3) ? ZS : 1;
}

template <int WM, int WN, int TM, int TN, int ZS, bool BF, bool X3, bool D3>
// Blocks [0, per_field) evaluate field `a`, blocks [per_field, 2 per_field) field `b` (two
// fields on one grid in one launch; `b` is unused when the grid covers one field).
__global__ __launch_bounds__(WM* WN * 64) void k_sep(SepArgs fa, SepArgs fb, int tiles_x, int tiles_y, int per_field)
{
    // The field's arguments as a local copy with the second field's pointers swapped in
    // (uniform selects); the shared epilogue parameters are read from `fa` directly, so the
    // copy is never indexed and stays in scalar registers.
    const bool second = static_cast<int>(blockIdx.x) >= per_field;
    SepArgs a = fa;
    if (second) {
        a.px = fb.px;
        a.px_lo = fb.px_lo;
        a.qy = fb.qy;
        a.qy_lo = fb.qy_lo;
        a.ez = fb.ez;
        a.amp = fb.amp;
        a.y = fb.y;
        a.k = fb.k;
        a.ind = fb.ind;
        a.partial = fb.partial;
    }
    const int64_t bid = second ? blockIdx.x - per_field : blockIdx.x;
    const int64_t rest = bid / tiles_x;
    int64_t s0 = 0, s1 = fa.ldp / kJC;
    if (a.partial) {
        // mode split: this slice's stage pairs, raw sums into the slice's plane of partial
        s0 = static_cast<int64_t>(blockIdx.y) * 2 * fa.pairs;
        s1 = min(s1, s0 + 2 * fa.pairs);
        a.y = a.partial + static_cast<int64_t>(blockIdx.y) * (fa.nx * fa.ny * fa.nz);
        a.k = nullptr;
        a.ind = nullptr;
        a.amp = 1.f;
    }
    if constexpr (use_dl<WM, WN, TM, TN, ZS, BF, X3, D3>()) {
        constexpr int Q = DlShape<WM, WN, TM, TN, X3, D3 ? ZS : 0>::STAGE_B / 16;
        __shared__ uint4 lds0[Q];
        __shared__ uint4 lds1[Q];
        sep_tile_dl<WM, WN, TM, TN, slices_per_block<WM, WN, TM, TN, ZS, BF, X3, D3>(), BF, X3, D3>(
            a, fa.epi, bid % tiles_x, rest % tiles_y, rest / tiles_y, lds0, lds1, s0, s1);
    } else {
        __shared__ uint4 smem[SepShape<WM, WN, TM, TN, X3>::LDS_WORDS / 4];
        sep_tile_reg<WM, WN, TM, TN, BF, X3, D3>(a, fa.epi, bid % tiles_x, rest % tiles_y, rest / tiles_y, smem, s0,
                                                 s1);
    }
}

// Persistent batched form: blocks pull (instance, tile, slice) work items from one atomic
// counter until the queue is drained (every block exits when the counter passes `total`).
// Instances are ordered by descending tile cost on the host; each instance uses the
// 128x128 (variant 0) or 64x64 (variant 1) tile the plan picked for its size class.
using BigT = SepShape<2, 2, 2, 2, false>;
using BigT3 = SepShape<2, 2, 2, 2, true>;
using SmallT = SepShape<2, 2, 1, 1, false>;
using SmallT3 = SepShape<2, 2, 1, 1, true>;

// ---- operands generated on chip (2-D one-pass fp16/bf16, batched ensembles) ------------
//
// On a 2-D grid the per-axis tables hold (nx + ny) N complex entries against nx ny cells: for
// the grids of an ensemble (sides of a few hundred) writing whole tables and streaming them
// back costs more than the contraction.  Here the x side of a tile is the instance's local
// table R_j(r) = e^{2 pi i a_x r hx} (r < kGenRows, the same for every tile of the instance:
// see GenArgs), staged straight into LDS, and the block generates the y side, which carries
// the tile's x0 phase, in LDS itself: thread (p, segment) owns mode p of the stage and RPT
// consecutive rows (16 of the 128-row tile); the first row's phase psi' + a_y (y0 + r0) hy +
// a_x x0 hx is formed and reduced in FP64 (hardware cos/sin of the fraction in revolutions,
// times w), and each further row is one FP32 complex product with the step
// e^{2 pi i frac(a_y hy)} (at most 15 of them: a relative error ~2e-6, far below the
// fp16/bf16 rounding of the operand).  Stage
// s + 1 is generated and loaded while the MFMAs consume stage s; the LDS layout and the
// fragment reads are those of the staged tiles.
template <bool BF>
__device__ __forceinline__ uint32_t pack2(float re, float im)
{
    if constexpr (BF) {
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(uint32_t, b2{static_cast<__bf16>(re), static_cast<__bf16>(im)});
    } else {
        return __builtin_bit_cast(uint32_t, h2{static_cast<_Float16>(re), static_cast<_Float16>(im)});
    }
}

// One 2-D output tile of a 4-wave block (2 x 2 waves of TM x TN fragments of 32 x 32):
// rows y0 = ty BM .., columns x0 = tx BN ..  `lds0`, `lds1`: (BM + BN) x 128 bytes each.
template <int TM, int TN, bool BF>
__device__ __forceinline__ void sep_tile_gen(const SepArgs& a, const GenArgs& g, int64_t tx, int64_t ty,
                                             uint4* lds0, uint4* lds1)
{
    constexpr int WN = 2;
    constexpr int BM = 2 * TM * 32, BN = WN * TN * 32;
    constexpr int ROW_B = kJC * 4;
    constexpr int RPT = BM / 8;         // rows per thread: 32 modes x 8 segments
    constexpr int KB = BN / 32;         // B load instructions per wave and stage (8 rows each)
    static_assert(RPT >= 1 && RPT <= 16 && BN <= kGenRows, "tile shape");
    const int t = threadIdx.x;
    const int l = t & 63, h = l >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int64_t x0 = tx * BN, y0 = ty * BM;

    // generation role: mode p of every stage, rows r0 .. r0 + RPT - 1 of the y operand (each
    // mode's FP64 phase, cosine and sine are formed by 8 threads, its record loaded 8 times)
    const int p = t & 31, seg = t >> 5;
    const int r0 = seg * RPT;
    const double yoff = static_cast<double>(y0 + r0) * g.hy, xoff = static_cast<double>(x0) * g.hx;
    int soff[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) soff[r] = (r0 + r) * ROW_B + (((p >> 2) ^ swz(r0 + r)) << 4) + ((p & 3) << 2);

    // x-side rows [BM, BM + BN) of a stage: instruction k of this wave fills rows 8 rb .. 8 rb + 7
    int32_t offb[KB];
    int ldb[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int rb = wave * KB + k;
        const int row = rb * 8 + (l >> 3);
        offb[k] = row * kJC + 4 * ((l & 7) ^ swz(row));
        ldb[k] = BM * ROW_B + rb * 8 * ROW_B;
    }
    auto issue = [&](int64_t s, char* buf) {
        const uint32_t* src = g.rx + s * (kGenRows * kJC);
#pragma unroll
        for (int k = 0; k < KB; ++k) load_to_lds(src + offb[k], buf + ldb[k]);
    };

    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef const u32x4 __attribute__((address_space(1)))* gq;
    struct Params {
        GenMode m;
    };
    auto load = [&](int64_t s, Params& pr) {
        // three 16-byte global loads (address-space cast: global, not flat, loads)
        const gq src = (gq)(g.md + s * kJC + p);
        struct Raw {
            u32x4 q[3];
        } raw;
#pragma unroll
        for (int c = 0; c < 3; ++c) raw.q[c] = src[c];
        pr.m = __builtin_bit_cast(GenMode, raw);
    };
    auto gen = [&](const Params& pr, char* buf) {
        const double t0 = fma(pr.m.ay, yoff, fma(pr.m.ax, xoff, pr.m.psi));
        const float f0 = static_cast<float>(t0 - floor(t0));  // exact in FP64
        float er = __builtin_amdgcn_cosf(f0) * pr.m.w;
        float ei = __builtin_amdgcn_sinf(f0) * pr.m.w;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            *reinterpret_cast<uint32_t*>(buf + soff[r]) = pack2<BF>(er, ei);
            if (r + 1 < RPT) {
                float nr = fmaf(er, pr.m.rc, -ei * pr.m.rs);
                float ni = fmaf(er, pr.m.rs, ei * pr.m.rc);
                // opaque: the next row's pack converts these values (one v_cvt_pk) instead
                // of the compiler recomputing the products in mixed precision
                asm("" : "+v"(nr), "+v"(ni));
                er = nr;
                ei = ni;
            }
        }
    };

    int fra[TM], ga[TM], frb[TN], gb[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int row = (wm * TM + i) * 32 + (l & 31);
        fra[i] = row * ROW_B;
        ga[i] = swz(row) ^ h;
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int col = (wn * TN + j) * 32 + (l & 31);
        frb[j] = BM * ROW_B + col * ROW_B;
        gb[j] = swz(col) ^ h;
    }
    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
    auto compute = [&](const char* buf) {
#pragma unroll
        for (int ks = 0; ks < kJC / 8; ++ks) {
            uint4 fa[TM], fb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) fa[i] = *reinterpret_cast<const uint4*>(buf + fra[i] + (((2 * ks) ^ ga[i]) << 4));
#pragma unroll
            for (int j = 0; j < TN; ++j) fb[j] = *reinterpret_cast<const uint4*>(buf + frb[j] + (((2 * ks) ^ gb[j]) << 4));
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma<BF>(fa[i], fb[j], acc[i][j]);
        }
    };

    // two stages per iteration (ldp is a multiple of 64): stage s + 1 is loaded and generated
    // into the other buffer while stage s feeds the MFMAs; the barrier after each half hands
    // it over
    char* b0 = reinterpret_cast<char*>(lds0);
    char* b1 = reinterpret_cast<char*>(lds1);
    const int64_t nstage = a.ldp / kJC;
    Params p0, p1;
    load(0, p0);
    load(1, p1);
    issue(0, b0);
    gen(p0, b0);
    wait_loads();
    __syncthreads();
    for (int64_t s = 0; s < nstage; s += 2) {
        issue(s + 1, b1);
        if (s + 2 < nstage) load(s + 2, p0);
        gen(p1, b1);
        compute(b0);
        wait_loads();
        __syncthreads();
        if (s + 2 < nstage) issue(s + 2, b0);
        if (s + 3 < nstage) load(s + 3, p1);
        if (s + 2 < nstage) gen(p0, b0);
        compute(b1);
        wait_loads();
        __syncthreads();
    }

    store_tiles<TM, TN, BM, BN, true>(a, a.epi, 0, x0, y0, wm * TM * 32, wn * TN * 32, l, acc);
}

// Index of the accelerator complex (XCD) this wave runs on (hardware register XCC_ID).
__device__ __forceinline__ unsigned xcc_id()
{
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 15u;
}

template <bool BF, bool X3, bool D3, bool GEN>
__global__ __launch_bounds__(256, GEN ? 2 : 1) void k_sep_batch(const SepBatchItem* __restrict__ items, int n_inst,
                                                   const BatchQueue* __restrict__ queues, int nq,
                                                   unsigned long long* counters)
{
    static_assert(!GEN || (!X3 && !D3), "generated operands: 2-D one-pass forms");
    constexpr bool DL = !GEN && use_dl<2, 2, 2, 2, 1, BF, X3, D3>();
    static_assert(GEN || DL == use_dl<2, 2, 1, 1, 1, BF, X3, D3>(), "both batch tiles stage the same way");
    constexpr int QD = GEN ? (128 + 128) * kJC * 4 / 16 : DlShape<2, 2, 2, 2, X3, D3 ? 1 : 0>::STAGE_B / 16;
    constexpr int W0 = X3 ? BigT3::LDS_WORDS : BigT::LDS_WORDS;
    constexpr int W1 = X3 ? SmallT3::LDS_WORDS : SmallT::LDS_WORDS;
    constexpr int Q0 = (DL || GEN) ? QD : (W0 > W1 ? W0 : W1) / 4;
    __shared__ uint4 lds0[Q0];
    __shared__ uint4 lds1[(DL || GEN) ? QD : 1];
    __shared__ unsigned long long s_item;
    // Own queue first, then the others in turn; every queue is finite, so every block ends
    // after at most nq exhausted pulls.
    int q = static_cast<int>(xcc_id() % static_cast<unsigned>(nq));
    for (int drained = 0; drained < nq;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counters + q * kQueueStride, 1ull);
        __syncthreads();
        const int64_t loc = static_cast<int64_t>(s_item);
        __syncthreads();
        const BatchQueue bq = queues[q];
        if (loc >= bq.count) {
            q = q + 1 == nq ? 0 : q + 1;
            ++drained;
            continue;
        }
        const int64_t it = bq.start + loc;
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].item0 <= it) lo = mid;
            else hi = mid - 1;
        }
        const SepBatchItem& b = items[lo];
        const int64_t local = it - b.item0;
        const int64_t rest = local / b.tiles_x;
        if constexpr (GEN) {
            if (b.variant == 0) sep_tile_gen<2, 2, BF>(b.a, b.g, local % b.tiles_x, rest, lds0, lds1);
            else sep_tile_gen<1, 1, BF>(b.a, b.g, local % b.tiles_x, rest, lds0, lds1);
        } else if constexpr (DL) {
            const int64_t ns = b.a.ldp / kJC;
            if (b.variant == 0)
                sep_tile_dl<2, 2, 2, 2, 1, BF, X3, D3>(b.a, b.a.epi, local % b.tiles_x, rest % b.tiles_y, rest / b.tiles_y, lds0,
                                                       lds1, 0, ns);
            else
                sep_tile_dl<2, 2, 1, 1, 1, BF, X3, D3>(b.a, b.a.epi, local % b.tiles_x, rest % b.tiles_y, rest / b.tiles_y, lds0,
                                                       lds1, 0, ns);
        } else {
            if (b.variant == 0)
                sep_tile_reg<2, 2, 2, 2, BF, X3, D3>(b.a, b.a.epi, local % b.tiles_x, rest % b.tiles_y, rest / b.tiles_y, lds0,
                                                     0, b.a.ldp / kJC);
            else
                sep_tile_reg<2, 2, 1, 1, BF, X3, D3>(b.a, b.a.epi, local % b.tiles_x, rest % b.tiles_y, rest / b.tiles_y, lds0,
                                                     0, b.a.ldp / kJC);
        }
    }
}

template <bool BF, bool X3, bool D3, bool GEN = !X3 && !D3>
hipError_t launch_batch_t(const SepBatchItem* items, int n_inst, const BatchQueue* queues, int nq,
                          unsigned long long* counters, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_sep_batch<BF, X3, D3, GEN>), dim3(grid), dim3(256), 0, s, items, n_inst, queues, nq,
                       counters);
    return hipGetLastError();
}

template <bool BF, bool X3, bool D3, bool GEN = !X3 && !D3>
int batch_occupancy_t()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sep_batch<BF, X3, D3, GEN>, 256, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

struct TileCfg {
    int bm, bn;
};
// tile selectors (rows y x cols x per block): 0 = 256x256 (8 waves), 1 = 128x128 (4 waves),
// 2 = 64x64 (4 waves), 3 = 128x256 (8 waves); covering two z-slices per block in the one-pass
// fp16 3-D form (one slice in the other forms): 4 = 128x256 (8 waves), 5 = 128x128 (4 waves),
// 6 = 128x256 (8 waves of 128x32), 7 = 256x128 (8 waves of 128x32), 8 = 256x128 (4 waves of
// 128x64); 9 = 256x256 (4 waves of 128x128, one slice).  sep_tile_slices gives the slices.
constexpr TileCfg kTiles[] = {{256, 256}, {128, 128}, {64, 64},  {128, 256}, {128, 256},
                              {128, 128}, {128, 256}, {256, 128}, {256, 128}, {256, 256}};

template <int WM, int WN, int TM, int TN, int ZS, bool BF, bool X3, bool D3>
hipError_t launch_k(const SepArgs& a, const SepArgs* b, hipStream_t s)
{
    constexpr int BM = WM * TM * 32, BN = WN * TN * 32;
    constexpr int zs = slices_per_block<WM, WN, TM, TN, ZS, BF, X3, D3>();
    const int tiles_x = static_cast<int>((a.nx + BN - 1) / BN);
    const int tiles_y = static_cast<int>((a.ny + BM - 1) / BM);
    const int64_t blocks = static_cast<int64_t>(tiles_x) * tiles_y * ((a.nz + zs - 1) / zs);
    if (2 * blocks > 0x7fffffff) return hipErrorInvalidValue;
    const bool split = a.partial != nullptr;
    const dim3 grid(static_cast<unsigned>(b ? 2 * blocks : blocks), static_cast<unsigned>(split ? a.slices : 1)),
        block(WM * WN * 64);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (a.timed && !split && timer_take_pair(&t0, &t1))  // start/stop stamped on the dispatch itself
        hipExtLaunchKernelGGL((k_sep<WM, WN, TM, TN, ZS, BF, X3, D3>), grid, block, 0, s, t0, t1, 0u, a, b ? *b : a,
                              tiles_x, tiles_y, static_cast<int>(blocks));
    else
        hipLaunchKernelGGL((k_sep<WM, WN, TM, TN, ZS, BF, X3, D3>), grid, block, 0, s, a, b ? *b : a, tiles_x,
                           tiles_y, static_cast<int>(blocks));
    return hipGetLastError();
}

template <bool BF, bool X3, bool D3>
hipError_t launch_t(const SepArgs& a, const SepArgs* b, int tile, hipStream_t s)
{
    switch (tile) {
    case 0: return launch_k<2, 4, 4, 2, 1, BF, X3, D3>(a, b, s);
    case 1: return launch_k<2, 2, 2, 2, 1, BF, X3, D3>(a, b, s);
    case 2: return launch_k<2, 2, 1, 1, 1, BF, X3, D3>(a, b, s);
    case 3: return launch_k<2, 4, 2, 2, 1, BF, X3, D3>(a, b, s);
    case 4: return D3 ? launch_k<2, 4, 2, 2, 2, BF, X3, D3>(a, b, s) : launch_k<2, 4, 2, 2, 1, BF, X3, D3>(a, b, s);
    case 5: return D3 ? launch_k<2, 2, 2, 2, 2, BF, X3, D3>(a, b, s) : launch_k<2, 2, 2, 2, 1, BF, X3, D3>(a, b, s);
    case 6: return launch_k<1, 8, 4, 1, 2, BF, X3, D3>(a, b, s);
    case 7: return launch_k<2, 4, 4, 1, 2, BF, X3, D3>(a, b, s);
    case 8: return launch_k<2, 2, 4, 2, 2, BF, X3, D3>(a, b, s);
    default: return launch_k<2, 2, 4, 4, 1, BF, X3, D3>(a, b, s);
    }
}

// z-slices one block of tile selector `tile` covers (mirrors launch_t).
template <bool BF, bool X3, bool D3>
int slices_t(int tile)
{
    switch (tile) {
    case 4: return D3 ? slices_per_block<2, 4, 2, 2, 2, BF, X3, D3>() : 1;
    case 5: return D3 ? slices_per_block<2, 2, 2, 2, 2, BF, X3, D3>() : 1;
    case 6: return slices_per_block<1, 8, 4, 1, 2, BF, X3, D3>();
    case 7: return slices_per_block<2, 4, 4, 1, 2, BF, X3, D3>();
    case 8: return slices_per_block<2, 2, 4, 2, 2, BF, X3, D3>();
    default: return 1;
    }
}

template <bool BF, bool X3>
hipError_t launch_d(const SepArgs& a, const SepArgs* b, int tile, hipStream_t s)
{
    return a.ez ? launch_t<BF, X3, true>(a, b, tile, s) : launch_t<BF, X3, false>(a, b, tile, s);
}

}  // namespace

int sep_tile_count() { return static_cast<int>(sizeof(kTiles) / sizeof(kTiles[0])); }

void sep_tile_shape(int tile, int* bm, int* bn)
{
    *bm = kTiles[tile].bm;
    *bn = kTiles[tile].bn;
}

int sep_tile_slices(int tile, int method, bool d3)
{
    switch (method) {
    case GRF_SEP_BF16: return d3 ? slices_t<true, false, true>(tile) : slices_t<true, false, false>(tile);
    case GRF_SEP_F16: return d3 ? slices_t<false, false, true>(tile) : slices_t<false, false, false>(tile);
    case GRF_SEP_BF16_X3: return d3 ? slices_t<true, true, true>(tile) : slices_t<true, true, false>(tile);
    default: return d3 ? slices_t<false, true, true>(tile) : slices_t<false, true, false>(tile);
    }
}

int sep_default_tile(int method, int64_t nx, int64_t ny, int64_t nz)
{
    // Large slices: 256x256 (operand reuse), or 128x256 for the hi+lo forms whose doubled
    // LDS stages do not fit twice at 256x256; small or thin grids: smaller tiles keep the
    // device busy and waste less on ragged edges.
    const int64_t t256 = ((nx + 255) / 256) * ((ny + 255) / 256) * nz;
    if (nx >= 192 && ny >= 192 && t256 >= 128) {
        if (method == GRF_SEP_F16_X3 || method == GRF_SEP_BF16_X3) return 3;
        // one-pass fp16 over several slices: 256x128 blocks covering two z-slices
        if (method == GRF_SEP_F16 && nz >= 2) return 7;
        return 0;
    }
    const int64_t t128 = ((nx + 127) / 128) * ((ny + 127) / 128) * nz;
    if (nx >= 96 && ny >= 96 && t128 >= 64) return 1;
    return 2;
}

int sep_mode_slices(int method, int dim, int64_t nx, int64_t ny, int64_t nz, int64_t ldp, int64_t* pairs)
{
    // Default tiles that give fewer blocks than CUs: the modes split into slices of at least two
    // stage pairs (128 modes) so that the launch has about two blocks per CU; the slices' sums
    // (at most 32 MiB) are added by a second pass.
    constexpr int64_t kCUs = 256, kMaxBytes = int64_t(32) << 20;
    const int64_t np = ldp / (2 * kJC);
    *pairs = np;
    if (method < GRF_SEP_BF16 || method > GRF_SEP_F16_X3) return 1;
    const int tile = sep_default_tile(method, nx, ny, nz);
    const int zs = dim == 3 ? sep_tile_slices(tile, method, true) : 1;
    const int64_t blocks = ((nx + kTiles[tile].bn - 1) / kTiles[tile].bn) * ((ny + kTiles[tile].bm - 1) / kTiles[tile].bm) *
                           ((nz + zs - 1) / zs);
    const int64_t cells = nx * ny * nz;
    if (blocks >= kCUs || np < 4) return 1;
    int64_t sl = std::min<int64_t>((2 * kCUs + blocks - 1) / blocks, np / 2);
    sl = std::min<int64_t>(sl, kMaxBytes / (4 * cells));
    if (sl < 2) return 1;
    const int64_t per = (np + sl - 1) / sl;
    *pairs = per;
    return static_cast<int>((np + per - 1) / per);
}

hipError_t launch_sep_batch(int method, bool d3, const SepBatchItem* items, int n_inst, const BatchQueue* queues,
                            int nq, unsigned long long* counters, int grid, hipStream_t s)
{
    if (nq < 1 || nq > kMaxQueues || n_inst < 1) return hipErrorInvalidValue;
    switch (method) {
    case GRF_SEP_BF16:
        return d3 ? launch_batch_t<true, false, true>(items, n_inst, queues, nq, counters, grid, s)
                  : launch_batch_t<true, false, false>(items, n_inst, queues, nq, counters, grid, s);
    case GRF_SEP_F16:
        return d3 ? launch_batch_t<false, false, true>(items, n_inst, queues, nq, counters, grid, s)
                  : launch_batch_t<false, false, false>(items, n_inst, queues, nq, counters, grid, s);
    case GRF_SEP_BF16_X3:
        return d3 ? launch_batch_t<true, true, true>(items, n_inst, queues, nq, counters, grid, s)
                  : launch_batch_t<true, true, false>(items, n_inst, queues, nq, counters, grid, s);
    case GRF_SEP_F16_X3:
        return d3 ? launch_batch_t<false, true, true>(items, n_inst, queues, nq, counters, grid, s)
                  : launch_batch_t<false, true, false>(items, n_inst, queues, nq, counters, grid, s);
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

hipError_t launch_sep(const SepArgs& a, hipStream_t s) { return launch_sep_pair(a, nullptr, s); }

hipError_t launch_sep_pair(const SepArgs& a, const SepArgs* b, hipStream_t s)
{
    int tile = a.tile < 0 ? sep_default_tile(a.method, a.nx, a.ny, a.nz) : a.tile;
    if (tile >= sep_tile_count()) return hipErrorInvalidValue;
    if (a.ldp <= 0 || a.ldp % (2 * kJC) != 0) return hipErrorInvalidValue;  // whole pairs of stages
    if (b && (b->method != a.method || b->nx != a.nx || b->ny != a.ny || b->nz != a.nz || b->ldp != a.ldp ||
              (b->ez == nullptr) != (a.ez == nullptr)))
        return hipErrorInvalidValue;
    const bool split = a.partial != nullptr;
    if (split && (a.tile >= 0 || a.slices < 1 || a.pairs < 1 || (b && b->partial == nullptr) ||
                  static_cast<int64_t>(a.slices) * a.pairs * 2 * kJC < a.ldp))
        return hipErrorInvalidValue;
    TimedScope timed(s, split && a.timed);  // the contraction and the slice sums
    hipError_t e;
    switch (a.method) {
    case GRF_SEP_BF16: e = launch_d<true, false>(a, b, tile, s); break;
    case GRF_SEP_F16: e = launch_d<false, false>(a, b, tile, s); break;
    case GRF_SEP_BF16_X3: e = launch_d<true, true>(a, b, tile, s); break;
    case GRF_SEP_F16_X3: e = launch_d<false, true>(a, b, tile, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || !split) return e;
    const int64_t C = a.nx * a.ny * a.nz;
    e = launch_points_reduce(a.partial, a.slices, C, a.amp, a.epi, a.y, a.k, a.ind, s);
    if (e == hipSuccess && b) e = launch_points_reduce(b->partial, a.slices, C, b->amp, a.epi, b->y, b->k, b->ind, s);
    return e;
}

}  // namespace grf
