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

__device__ inline float half_to_float(uint16_t b) { return static_cast<float>(__builtin_bit_cast(_Float16, b)); }
__device__ inline float bf16_to_float(uint16_t b) { return static_cast<float>(__builtin_bit_cast(__bf16, b)); }

// Entry e (= i * ldp + j) of one per-axis table.
__device__ __forceinline__ void axis_table_entry(const AxisTableArgs& a, int64_t i, int64_t j)
{
    // row-major [count][ldp], or stage-major [ldp / 32][count][32]
    const int64_t e = a.blocked ? ((j >> 5) * a.count + i) * 32 + (j & 31) : i * a.ldp + j;

    double f = 0.0;
    bool zero = j >= a.n;
    if (!zero) {
        const double x = a.origin + (static_cast<double>(i) + 0.5) * a.h;
        double t = 0.0;
        if (a.z) t = (a.z[static_cast<int64_t>(a.axis) * a.n + j] * a.freq_scale) * x;
        if (a.with_psi) t += a.phi[j] * kInvTwoPi;
        f = t - floor(t);  // exact in FP64
    }

    switch (a.format) {
    case TF_REV_F32:
        static_cast<float*>(a.out)[e] = static_cast<float>(f);
        break;
    case TF_REV_F64:
        static_cast<double*>(a.out)[e] = f;
        break;
    default: {
        double sn, cs;
        if (a.fast_trig) {
            const float fr = static_cast<float>(f);  // revolutions in [0, 1)
            cs = static_cast<double>(__builtin_amdgcn_cosf(fr));
            sn = static_cast<double>(__builtin_amdgcn_sinf(fr));
        } else {
            sincospi(2.0 * f, &sn, &cs);
        }
        if (zero) { sn = 0.0; cs = 0.0; }
        if (a.conj) sn = -sn;
        if (a.format == TF_CPLX_F32) {
            static_cast<float2*>(a.out)[e] = make_float2(static_cast<float>(cs), static_cast<float>(sn));
        } else if (a.format == TF_F16 || a.format == TF_F16_HILO) {
            const uint32_t hi = pack_half2(static_cast<float>(cs), static_cast<float>(sn));
            static_cast<uint32_t*>(a.out)[e] = hi;
            if (a.format == TF_F16_HILO) {
                const double rl = cs - static_cast<double>(half_to_float(static_cast<uint16_t>(hi & 0xffff)));
                const double il = sn - static_cast<double>(half_to_float(static_cast<uint16_t>(hi >> 16)));
                static_cast<uint32_t*>(a.out_lo)[e] = pack_half2(static_cast<float>(rl), static_cast<float>(il));
            }
        } else {
            const uint32_t hi = pack_bf162(static_cast<float>(cs), static_cast<float>(sn));
            static_cast<uint32_t*>(a.out)[e] = hi;
            if (a.format == TF_BF16_HILO) {
                const double rl = cs - static_cast<double>(bf16_to_float(static_cast<uint16_t>(hi & 0xffff)));
                const double il = sn - static_cast<double>(bf16_to_float(static_cast<uint16_t>(hi >> 16)));
                static_cast<uint32_t*>(a.out_lo)[e] = pack_bf162(static_cast<float>(rl), static_cast<float>(il));
            }
        }
    }
    }
}

// Block b of a table covers row b / jblocks, modes 256 (b % jblocks) + threadIdx.x, with
// jblocks = ceil(ldp / 256): the row/mode split is a per-block (scalar) division.
__device__ __forceinline__ void axis_table_block(const AxisTableArgs& a, int64_t b)
{
    const int64_t jblocks = (a.ldp + 255) / 256;
    const int64_t i = b / jblocks;
    const int64_t j = (b - i * jblocks) * 256 + threadIdx.x;
    if (j < a.ldp) axis_table_entry(a, i, j);
}

__global__ __launch_bounds__(256) void k_axis_table(AxisTableArgs a) { axis_table_block(a, blockIdx.x); }

// Many tables in one launch: descriptor d owns blocks [bprefix[d], bprefix[d+1]).  The
// descriptor lookup depends only on the block index, so it runs once per block on the
// scalar unit.
__global__ __launch_bounds__(256) void k_axis_tables_batched(const AxisTableArgs* __restrict__ descs,
                                                             const int64_t* __restrict__ bprefix, int ndesc)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bprefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    axis_table_block(descs[lo], b - bprefix[lo]);
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
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

}  // namespace

int64_t axis_table_blocks(const AxisTableArgs& a) { return a.count * ((a.ldp + 255) / 256); }

hipError_t launch_axis_table(const AxisTableArgs& a, hipStream_t s)
{
    const int64_t blocks = axis_table_blocks(a);
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_axis_table, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_axis_tables_batched(const AxisTableArgs* descs, const int64_t* bprefix, int ndesc,
                                      int64_t total_blocks, hipStream_t s)
{
    if (total_blocks <= 0 || ndesc <= 0) return hipSuccess;
    if (total_blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_axis_tables_batched, dim3(static_cast<unsigned>(total_blocks)), dim3(256), 0, s, descs,
                       bprefix, ndesc);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, p, v);
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

}  // namespace grf
