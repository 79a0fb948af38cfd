// Per-axis phase tables and per-mode parameters: the only FP64 step of the
// separable and grid-direct paths.
//
// For a structured grid the phase of mode j at cell (i0, i1, i2) splits per axis
// (Sec. 4.1, per-axis rescaling of frequency space):
//   theta / 2 pi = sum_a a_{j,a} x_{a,i_a} + psi_j,   a_{j,a} = z_{j,a} / (2 pi ell_a),
// so each axis contributes frac(a_{j,a} x_{a,i}) in revolutions.  The product is
// formed and reduced in FP64, where frac() is exact; only then is the value rounded
// to the table format.
#include <hip/hip_runtime.h>

#include <cstring>

#include "grf_internal.h"

namespace grf {

namespace {

constexpr double kInvTwoPi = 0.15915494309189533576888376337251;

__device__ inline uint32_t pack_half2(float re, float im)
{
    _Float16 r = static_cast<_Float16>(re), i = static_cast<_Float16>(im);
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, r)) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, i)) << 16);
}

__device__ inline uint32_t pack_bf162(float re, float im)
{
    __bf16 r = static_cast<__bf16>(re), i = static_cast<__bf16>(im);
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, r)) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, i)) << 16);
}

// Table stores are streaming (non-temporal): the tables are read by the next kernel, and
// stores that do not stay dirty in this XCD's L2 leave less to write back at the kernel's
// end (measured ~2.5 us less per 256^3 step).
template <typename T>
__device__ __forceinline__ void st(void* base, int64_t e, T v)
{
    __builtin_nontemporal_store(v, static_cast<T*>(base) + e);
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <>
__device__ __forceinline__ void st<float2>(void* base, int64_t e, float2 v)
{
    const f32x2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, static_cast<f32x2*>(base) + e);
}

__device__ inline float half_to_float(uint16_t b) { return static_cast<float>(__builtin_bit_cast(_Float16, b)); }
__device__ inline float bf16_to_float(uint16_t b) { return static_cast<float>(__builtin_bit_cast(__bf16, b)); }

// Rows of one table that a work block covers; a work block is (row group, 256-mode chunk),
// one mode per thread, so the per-mode factors are loaded and scaled once per row group.
constexpr int kTabRows = 16;

// Rows i0 .. i1-1 of the table for this thread's mode j: f = frac(a_j x_i (+ psi_j)) formed
// and reduced in FP64, then stored in format FMT.  `a` is a register copy of the descriptor,
// so no field is re-read from memory between the stores.
template <int FMT, bool FAST, bool BLOCKED>
__device__ __forceinline__ void axis_table_rows(const AxisTableArgs a, int64_t i0, int64_t i1, int64_t j, double az,
                                                double ps, double wj, bool zero)
{
    const double sgn = a.conj ? -1.0 : 1.0;
    for (int64_t i = i0; i < i1; ++i) {
        // row-major [count][ldp], or stage-major [ldp / 32][count][32]
        const int64_t e = BLOCKED ? ((j >> 5) * a.count + i) * 32 + (j & 31) : i * a.ldp + j;
        const double x = a.origin + (static_cast<double>(i) + 0.5) * a.h;
        const double t = az * x + ps;  // ps = 0 (exact) for tables without the phase
        const double f = zero ? 0.0 : t - floor(t);  // exact in FP64

        if constexpr (FMT == TF_REV_F32) {
            st<float>(a.out, e, static_cast<float>(f));
        } else if constexpr (FMT == TF_REV_F64) {
            st<double>(a.out, e, f);
        } else if constexpr (FAST && (FMT == TF_CPLX_F32 || FMT == TF_F16 || FMT == TF_BF16)) {
            // one rounding to the table format: the hardware cos/sin of the FP64-reduced
            // fraction in revolutions (|err| ~1e-7) is far below it
            const float fr = static_cast<float>(f);
            const float wf = static_cast<float>(wj);
            const float cs = zero ? 0.f : __builtin_amdgcn_cosf(fr) * wf;
            const float sn = zero ? 0.f : __builtin_amdgcn_sinf(fr) * static_cast<float>(sgn) * wf;
            if constexpr (FMT == TF_CPLX_F32) st<float2>(a.out, e, make_float2(cs, sn));
            else if constexpr (FMT == TF_F16) st<uint32_t>(a.out, e, pack_half2(cs, sn));
            else st<uint32_t>(a.out, e, pack_bf162(cs, sn));
        } else {
            double sn, cs;
            sincospi(2.0 * f, &sn, &cs);
            if (zero) { sn = 0.0; cs = 0.0; }
            sn *= sgn * wj;
            cs *= wj;
            if constexpr (FMT == TF_CPLX_F32) {
                st<float2>(a.out, e, make_float2(static_cast<float>(cs), static_cast<float>(sn)));
            } else if constexpr (FMT == TF_F16 || FMT == TF_F16_HILO) {
                const uint32_t hi = pack_half2(static_cast<float>(cs), static_cast<float>(sn));
                st<uint32_t>(a.out, e, hi);
                if constexpr (FMT == TF_F16_HILO) {
                    const double rl = cs - static_cast<double>(half_to_float(static_cast<uint16_t>(hi & 0xffff)));
                    const double il = sn - static_cast<double>(half_to_float(static_cast<uint16_t>(hi >> 16)));
                    st<uint32_t>(a.out_lo, e, pack_half2(static_cast<float>(rl), static_cast<float>(il)));
                }
            } else {
                const uint32_t hi = pack_bf162(static_cast<float>(cs), static_cast<float>(sn));
                st<uint32_t>(a.out, e, hi);
                if constexpr (FMT == TF_BF16_HILO) {
                    const double rl = cs - static_cast<double>(bf16_to_float(static_cast<uint16_t>(hi & 0xffff)));
                    const double il = sn - static_cast<double>(bf16_to_float(static_cast<uint16_t>(hi >> 16)));
                    st<uint32_t>(a.out_lo, e, pack_bf162(static_cast<float>(rl), static_cast<float>(il)));
                }
            }
        }
    }
}

template <int FMT>
__device__ __forceinline__ void axis_table_rows_t(const AxisTableArgs& a, int64_t i0, int64_t i1, int64_t j,
                                                  double az, double ps, double wj, bool zero)
{
    if (a.blocked) {
        if (a.fast_trig) axis_table_rows<FMT, true, true>(a, i0, i1, j, az, ps, wj, zero);
        else axis_table_rows<FMT, false, true>(a, i0, i1, j, az, ps, wj, zero);
    } else {
        if (a.fast_trig) axis_table_rows<FMT, true, false>(a, i0, i1, j, az, ps, wj, zero);
        else axis_table_rows<FMT, false, false>(a, i0, i1, j, az, ps, wj, zero);
    }
}

// Work block w of one table: rows kTabRows (w / jchunks) .., modes 256 (w % jchunks) + tid.
__device__ __forceinline__ void axis_table_block(const AxisTableArgs a, int64_t w)
{
    const int64_t jchunks = (a.ldp + 255) / 256;
    const int64_t rg = w / jchunks;
    const int64_t j = (w - rg * jchunks) * 256 + threadIdx.x;
    if (j >= a.ldp) return;
    const bool zero = j >= a.n;
    double az = 0.0, ps = 0.0, wj = 1.0;
    if (!zero) {
        if (a.z) az = a.z[static_cast<int64_t>(a.axis) * a.n + j] * a.freq_scale;
        if (a.with_psi) ps = a.phi[j] * kInvTwoPi;
        if (a.w) wj = a.w[j];
    }
    const int64_t i0 = rg * kTabRows;
    const int64_t i1 = min(i0 + kTabRows, a.count);
    switch (a.format) {
    case TF_REV_F32: axis_table_rows<TF_REV_F32, true, false>(a, i0, i1, j, az, ps, wj, zero); break;
    case TF_REV_F64: axis_table_rows<TF_REV_F64, true, false>(a, i0, i1, j, az, ps, wj, zero); break;
    case TF_CPLX_F32: axis_table_rows_t<TF_CPLX_F32>(a, i0, i1, j, az, ps, wj, zero); break;
    case TF_F16: axis_table_rows_t<TF_F16>(a, i0, i1, j, az, ps, wj, zero); break;
    case TF_F16_HILO: axis_table_rows_t<TF_F16_HILO>(a, i0, i1, j, az, ps, wj, zero); break;
    case TF_BF16: axis_table_rows_t<TF_BF16>(a, i0, i1, j, az, ps, wj, zero); break;
    default: axis_table_rows_t<TF_BF16_HILO>(a, i0, i1, j, az, ps, wj, zero); break;
    }
}

// Up to six tables (the axes of one grid, or of two fields on one grid) in one launch; table
// t owns work blocks [start[t], start[t + 1]).  Constant indices only: a by-value argument
// indexed per block would be copied to scratch memory.
struct TableSet {
    AxisTableArgs d[6];
    int64_t start[7];
};

__global__ __launch_bounds__(256) void k_axis_tables3(TableSet ts)
{
    const int64_t b = blockIdx.x;
    if (b >= ts.start[5]) axis_table_block(ts.d[5], b - ts.start[5]);
    else if (b >= ts.start[4]) axis_table_block(ts.d[4], b - ts.start[4]);
    else if (b >= ts.start[3]) axis_table_block(ts.d[3], b - ts.start[3]);
    else if (b >= ts.start[2]) axis_table_block(ts.d[2], b - ts.start[2]);
    else if (b >= ts.start[1]) axis_table_block(ts.d[1], b - ts.start[1]);
    else axis_table_block(ts.d[0], b);
}

// Many tables in one launch: entry b of `blk` packs (descriptor << 40) | local work block,
// one load per block instead of a search over the descriptor prefix.
__global__ __launch_bounds__(256) void k_axis_tables_batched(const AxisTableArgs* __restrict__ descs,
                                                             const uint64_t* __restrict__ blk)
{
    const uint64_t w = blk[blockIdx.x];
    axis_table_block(descs[w >> 40], static_cast<int64_t>(w & ((uint64_t(1) << 40) - 1)));
}

// Copies a bitruncated rule's bin -> facies table and facies values to device memory.
struct RuleTables {
    uint8_t rule[256];
    float values[GRF_MAX_FACIES];
};

__global__ __launch_bounds__(256) void k_rule_tables(RuleTables r, uint8_t* rule, float* values)
{
    const int t = threadIdx.x;
    rule[t] = r.rule[t];
    if (t < GRF_MAX_FACIES) values[t] = r.values[t];
}

// Wavevectors of a rotated table, k_j = R diag(1/ell) z_j, written as an axis-aligned table.
struct RotArgs {
    double r[9];  // row-major 3 x 3
    double ell[3];
};

template <int DIM>
__global__ __launch_bounds__(256) void k_rotate_modes(const double* __restrict__ z, int64_t n, RotArgs ra,
                                                      double* __restrict__ out)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double u[DIM];
#pragma unroll
    for (int b = 0; b < DIM; ++b) u[b] = z[b * n + j] / ra.ell[b];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) v += ra.r[3 * a + b] * u[b];
        out[a * n + j] = v;
    }
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int n, int stride)
{
    if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < n) p[threadIdx.x * stride] = v;
}

__global__ __launch_bounds__(256) void k_mode_params(const double* z, const double* phi, int dim, int64_t n,
                                                     int64_t ldp, double ex, double ey, double ez,
                                                     double4* out)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= ldp) return;
    double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
    if (j < n) {
        p.x = z[j] * kInvTwoPi / ex;
        p.y = z[n + j] * kInvTwoPi / ey;
        if (dim == 3) p.z = z[2 * n + j] * kInvTwoPi / ez;
        p.w = phi[j] * kInvTwoPi;
    }
    out[j] = p;
}

// Per-mode inputs of the generated batch tiles, one block row per instance.
__global__ __launch_bounds__(256) void k_gen_modes(const GenModeDesc* __restrict__ descs)
{
    const GenModeDesc d = descs[blockIdx.y];
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (j >= d.ldp) return;
    GenMode m{};
    m.rc = 1.f;
    if (j < d.n) {
        constexpr double kInvTwoPi = 0.15915494309189533576888376337251;
        const double ax = d.z[j] * d.fsx, ay = d.z[d.n + j] * d.fsy;
        m.ax = ax;
        m.ay = ay;
        m.psi = d.phi[j] * kInvTwoPi + ay * (d.oy + 0.5 * d.hy) + ax * (d.ox + 0.5 * d.hx);
        m.w = d.w ? static_cast<float>(d.w[j]) : 1.f;
        const double th = ay * d.hy;
        const float fh = static_cast<float>(th - floor(th));  // exact in FP64
        m.rc = __builtin_amdgcn_cosf(fh);
        m.rs = __builtin_amdgcn_sinf(fh);
    }
    d.out[j] = m;
}

}  // namespace

int64_t axis_table_blocks(const AxisTableArgs& a) { return ((a.count + kTabRows - 1) / kTabRows) * ((a.ldp + 255) / 256); }

hipError_t launch_axis_tables(const AxisTableArgs* d, int nd, hipStream_t s)
{
    if (nd < 0 || nd > 6) return hipErrorInvalidValue;
    TableSet ts{};
    int64_t b = 0;
    for (int t = 0; t < 6; ++t) {
        ts.start[t] = b;
        if (t < nd) {
            ts.d[t] = d[t];
            b += axis_table_blocks(d[t]);
        }
    }
    ts.start[6] = b;
    if (b <= 0) return hipSuccess;
    if (b > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_axis_tables3, dim3(static_cast<unsigned>(b)), dim3(256), 0, s, ts);
    return hipGetLastError();
}

hipError_t launch_axis_table(const AxisTableArgs& a, hipStream_t s) { return launch_axis_tables(&a, 1, s); }

hipError_t launch_axis_tables_batched(const AxisTableArgs* descs, const uint64_t* blk, int64_t total_blocks,
                                      hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    if (total_blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_axis_tables_batched, dim3(static_cast<unsigned>(total_blocks)), dim3(256), 0, s, descs, blk);
    return hipGetLastError();
}

hipError_t launch_rule_tables(const grf_trunc2& r, void* dst, hipStream_t s)
{
    static_assert(sizeof(r.rule) <= 256, "rule table");
    RuleTables t{};
    std::memcpy(t.rule, r.rule, sizeof(r.rule));
    for (int i = 0; i < r.n_values && i < GRF_MAX_FACIES; ++i) t.values[i] = r.values[i];
    uint8_t* rule = static_cast<uint8_t*>(dst);
    hipLaunchKernelGGL(k_rule_tables, dim3(1), dim3(256), 0, s, t, rule, reinterpret_cast<float*>(rule + 256));
    return hipGetLastError();
}

hipError_t launch_rotate_modes(const double* z, int dim, int64_t n, const double* rot, const double* ell, double* out,
                               hipStream_t s)
{
    RotArgs ra{};
    for (int i = 0; i < 9; ++i) ra.r[i] = rot[i];
    for (int a = 0; a < 3; ++a) ra.ell[a] = a < dim ? ell[a] : 1.0;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (dim == 3)
        hipLaunchKernelGGL(k_rotate_modes<3>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, z, n, ra, out);
    else
        hipLaunchKernelGGL(k_rotate_modes<2>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, z, n, ra, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, int stride, hipStream_t s)
{
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, p, v, n, stride);
    return hipGetLastError();
}

hipError_t launch_mode_params(const double* z, const double* phi, int dim, int64_t n, int64_t ldp,
                              const double* ell, double* out, hipStream_t s)
{
    const int64_t blocks = (ldp + 255) / 256;
    hipLaunchKernelGGL(k_mode_params, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, z, phi, dim, n, ldp,
                       ell[0], ell[1], dim == 3 ? ell[2] : 1.0, reinterpret_cast<double4*>(out));
    return hipGetLastError();
}

hipError_t launch_gen_modes(const GenModeDesc* d, int n_inst, int64_t ldp_max, hipStream_t s)
{
    if (n_inst < 1) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((ldp_max + 255) / 256), static_cast<unsigned>(n_inst));
    hipLaunchKernelGGL(k_gen_modes, grid, dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace grf
