// Binned form of the direct point sum (Sec. 4.1: on unstructured meshes the spectral sum is
// evaluated at every cell centre).
//
// The per-point form reduces every phase a_j . x_p + psi_j in FP64 (three FP64 FMAs, a fract
// and a conversion per mode and point).  Here the points are first sorted into cells of their
// bounding box (each cell's slots padded to whole work items of 256), and the phase of
// mode j at point p of a cell with centre c is
//   r_jp = frac(a_j . c + psi_j) + a_j . (x_p - c),
// the first part reduced in FP64 once per (mode, work item), the second small (cells are
// small).  For 16 modes and 16 points both parts together are one matrix product on the
// matrix cores, [a_x a_y a_z frac(a.c + psi)] (16 x 4) times [dx dy dz 1]^T (4 x 16), taken in
// fp16 with FP32 accumulation and every factor split hi + lo (FP32-accurate), so the vector
// units spend one hardware cosine (argument in revolutions) and one FMA per term.
// Modes whose local part can reach kLocalRev revolutions in a cell (heavy spectral tails) take
// weight 0 in that pass and are added in a second pass that reduces a_j . x_p + psi_j per
// point in FP64 from the FP64 offsets (a branch uniform over the wave).  A point's value
// depends only on its cell, its offset and the table, not on which points share its work
// item, so the atomics that order points within a cell leave the results deterministic.
// Results are written (or stored as mode-slice partial sums) at each point's input index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "grf_internal.h"

namespace grf {

namespace {

constexpr int kItem = kBinItemSlots;  // slots (points) per work item: one wave
constexpr int kGroups = kItem / 16;    // 16-point column blocks of the matrix product
constexpr int kPipe = 4;               // groups whose products are in flight together
constexpr double kLocalRev = 4.0;      // local phases up to this many revolutions stay in FP32

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// Per-block bounding-box partials: lo[3], hi[3] per block.
template <int DIM>
__global__ __launch_bounds__(256) void k_bin_bbox(const double* __restrict__ xyz, int64_t P, double* __restrict__ part)
{
    __shared__ double s[6][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; p < P; p += stride)
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double v = xyz[p * DIM + a];
            if (isfinite(v)) {  // a non-finite coordinate spoils only its own point's value
                lo[a] = fmin(lo[a], v);
                hi[a] = fmax(hi[a], v);
            }
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + w]);
                s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// Cell geometry from the bounding box (one block): cells of side about s holding about
// `target` points on average, at most `cap` cells; each axis of extent e > 0 is cut into
// n = round(e / s) >= 1 cells of side e / n, so that no row of cells sticks out of the box (a
// partly filled last row pads its cells to whole work items for few points).  Clears the
// cell counters.
__global__ __launch_bounds__(256) void k_bin_geom(const double* __restrict__ part, int nb, int dim, int64_t P,
                                                  double target, int64_t cap, BinGeom* __restrict__ geom,
                                                  int32_t* __restrict__ count)
{
    __shared__ double red[6][256];
    __shared__ double lo[3], hi[3];
    __shared__ int64_t ncell_s;
    {
        double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] = q < 3 ? fmin(v[q], part[b * 6 + q]) : fmax(v[q], part[b * 6 + q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = v[q];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w)
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    red[q][threadIdx.x] = q < 3 ? fmin(red[q][threadIdx.x], red[q][threadIdx.x + w])
                                                : fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x < 3) {
            lo[threadIdx.x] = red[threadIdx.x][0];
            hi[threadIdx.x] = red[3 + threadIdx.x][0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        BinGeom g{};
        double ext[3] = {0.0, 0.0, 0.0};
        double vol = 1.0;
        int deff = 0;
        for (int a = 0; a < dim; ++a) {
            ext[a] = hi[a] - lo[a];
            if (ext[a] > 0.0) {
                vol *= ext[a];
                ++deff;
            }
        }
        double emax = 0.0;
        for (int a = 0; a < dim; ++a) emax = fmax(emax, ext[a]);
        double s = 1.0;
        if (deff > 0) s = pow(vol * target / static_cast<double>(P), 1.0 / deff);
        if (!(s > 0.0) || !isfinite(s)) s = emax > 0.0 && isfinite(emax) ? emax : 1.0;  // under/overflow
        int64_t n[3];
        for (int it = 0;; ++it) {
            int64_t tot = 1;
            for (int a = 0; a < 3; ++a) {
                const double q = (a < dim && ext[a] > 0.0) ? floor(ext[a] / s + 0.5) : 1.0;
                n[a] = !(q >= 1.0) ? 1 : (q >= double(1 << 20) ? int64_t(1) << 20 : static_cast<int64_t>(q));
                tot *= n[a];
            }
            if (tot <= cap || it >= 400) break;  // 1.25^400: every side down to one cell
            s *= 1.25;
        }
        if (n[0] * n[1] * n[2] > cap) n[0] = n[1] = n[2] = 1;
        for (int a = 0; a < 3; ++a) {
            g.lo[a] = a < dim && isfinite(lo[a]) ? lo[a] : 0.0;  // (no finite coordinate: any)
            g.n[a] = static_cast<int32_t>(n[a]);
            // the side that tiles the extent; s on flat axes (and for extents so small that the
            // reciprocal would overflow)
            double sa = (a < dim && ext[a] > 0.0) ? ext[a] / static_cast<double>(n[a]) : s;
            if (!(sa > 0.0) || !isfinite(sa) || !isfinite(1.0 / sa)) sa = s;
            g.s[a] = sa;
            g.inv_s[a] = 1.0 / sa;
        }
        g.ncell = static_cast<int32_t>(n[0] * n[1] * n[2]);
        *geom = g;
        ncell_s = g.ncell;
    }
    __syncthreads();
    for (int64_t c = threadIdx.x; c < ncell_s; c += 256) count[c] = 0;
}

template <int DIM>
__device__ __forceinline__ int32_t cell_of(const BinGeom& g, const double* x)
{
    int32_t c = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double f = floor((x[a] - g.lo[a]) * g.inv_s[a]);
        if (!(f >= 0.0)) f = 0.0;  // also NaN
        if (f > static_cast<double>(g.n[a] - 1)) f = static_cast<double>(g.n[a] - 1);
        c += static_cast<int32_t>(f) * stride;
        stride *= g.n[a];
    }
    return c;
}

// Cell of every point and its rank among the cell's points (order of arrival).  A block takes
// kCountChunk consecutive points; with at most kLdsCells cells it counts them in LDS first and
// reserves each cell's range with one global atomic (rank = base + rank within the block).
constexpr int kCountPer = 16;                 // points per thread
constexpr int kCountChunk = 256 * kCountPer;  // points per block
constexpr int kLdsCells = 16384;

template <int DIM>
__global__ __launch_bounds__(256) void k_bin_count(const double* __restrict__ xyz, int64_t P,
                                                   const BinGeom* __restrict__ geom, int32_t* __restrict__ count,
                                                   int2* __restrict__ cellrank)
{
    __shared__ int32_t hist[kLdsCells];
    const BinGeom g = *geom;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCountChunk;
    const bool lds = g.ncell <= kLdsCells;
    if (lds) {
        for (int c = threadIdx.x; c < g.ncell; c += 256) hist[c] = 0;
        __syncthreads();
    }
    int32_t cell[kCountPer], rank[kCountPer];
#pragma unroll
    for (int q = 0; q < kCountPer; ++q) {
        const int64_t p = base + q * 256 + threadIdx.x;
        cell[q] = -1;
        rank[q] = 0;
        if (p < P) {
            double x[3];
#pragma unroll
            for (int a = 0; a < DIM; ++a) x[a] = xyz[p * DIM + a];
            cell[q] = cell_of<DIM>(g, x);
            rank[q] = lds ? atomicAdd(hist + cell[q], 1) : atomicAdd(count + cell[q], 1);
        }
    }
    if (lds) {
        __syncthreads();
        for (int c = threadIdx.x; c < g.ncell; c += 256) {
            const int32_t h = hist[c];
            hist[c] = h > 0 ? atomicAdd(count + c, h) : 0;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kCountPer; ++q) {
        const int64_t p = base + q * 256 + threadIdx.x;
        if (p < P) cellrank[p] = make_int2(cell[q], rank[q] + (lds ? hist[cell[q]] : 0));
    }
}

// Exclusive scan of the cell counts padded to whole work items (one block of 1024 threads):
// the slot offset of every cell, the slot and work-item totals.
__global__ __launch_bounds__(1024) void k_bin_scan(BinGeom* __restrict__ geom, const int32_t* __restrict__ count,
                                                   int32_t* __restrict__ offset)
{
    __shared__ int64_t part[1024];
    const int ncell = geom->ncell;
    const int t = threadIdx.x;
    const int per = (ncell + 1023) / 1024;
    const int c0 = min(t * per, ncell), c1 = min(c0 + per, ncell);
    int64_t sum = 0;
    for (int c = c0; c < c1; ++c) sum += (count[c] + kItem - 1) / kItem * kItem;
    part[t] = sum;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {  // inclusive Hillis-Steele scan
        const int64_t v = t >= w ? part[t - w] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t off = part[t] - sum;
    for (int c = c0; c < c1; ++c) {
        offset[c] = static_cast<int32_t>(off);
        off += (count[c] + kItem - 1) / kItem * kItem;
    }
    if (t == 1023) {
        geom->nslot = part[1023];
        geom->nitem = part[1023] / kItem;
    }
}

// One block per work item (of the capacity): the item's cell (the last cell whose offset is
// at or below the item's first slot), and empty records (offset 0, input index -1) in all its
// slots; the points are scattered over them next.
__global__ __launch_bounds__(256) void k_bin_items(const BinGeom* __restrict__ geom, const int32_t* __restrict__ offset,
                                                   int32_t* __restrict__ item_cell, double4* __restrict__ rec)
{
    const int64_t item = blockIdx.x;
    if (item >= geom->nitem) return;
    rec[item * kItem + threadIdx.x] = make_double4(0.0, 0.0, 0.0, -1.0);
    if (threadIdx.x == 0) {
        const int64_t slot = item * kItem;
        int lo = 0, hi = geom->ncell - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (offset[mid] <= slot) lo = mid;
            else hi = mid - 1;
        }
        item_cell[item] = lo;
    }
}

// Sorted slots: one record per point, its FP64 offset from the cell centre and its input
// index (exact in FP64).
template <int DIM>
__global__ __launch_bounds__(256) void k_bin_scatter(const double* __restrict__ xyz, int64_t P,
                                                     const BinGeom* __restrict__ geom,
                                                     const int32_t* __restrict__ offset,
                                                     const int2* __restrict__ cellrank, double4* __restrict__ rec)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= P) return;
    const BinGeom g = *geom;
    const int2 cr = cellrank[p];
    const int64_t slot = static_cast<int64_t>(offset[cr.x]) + cr.y;
    double d[3] = {0.0, 0.0, 0.0};
    int32_t rest = cr.x;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int32_t i = rest % g.n[a];
        rest /= g.n[a];
        d[a] = xyz[p * DIM + a] - (g.lo[a] + (static_cast<double>(i) + 0.5) * g.s[a]);
    }
    rec[slot] = make_double4(d[0], d[1], d[2], static_cast<double>(p));
}

__device__ __forceinline__ uint32_t pack_h2(_Float16 a, _Float16 b)
{
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, a)) | (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, b)) << 16);
}

__device__ __forceinline__ void split16(float v, _Float16& hi, _Float16& lo)
{
    hi = static_cast<_Float16>(v);
    lo = static_cast<_Float16>(v - static_cast<float>(hi));
}

// FP32 copies of the per-mode parameters in revolutions per cell side, the weight of each mode
// in the matrix pass (0 for padding modes and for the FP64 modes) and in the FP64 pass, and the
// flag of modes whose local phase can reach kLocalRev revolutions within a cell.
struct ModeF {
    float ax, ay, az;
    float w;       // weight in the matrix pass
    int32_t fp64;  // 1: reduce this mode's phase per point in FP64 (second pass)
    float w64;     // weight in the FP64 pass
    int32_t pad[2];
};

// Indices of the modes flagged for the FP64 pass, in ascending order (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_bin_flags(const ModeF* __restrict__ pf, int64_t n, BinGeom* __restrict__ geom,
                                                    int32_t* __restrict__ list)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t j0 = min<int64_t>(t * per, n), j1 = min<int64_t>(j0 + per, n);
    int32_t cnt = 0;
    for (int64_t j = j0; j < j1; ++j) cnt += pf[j].fp64;
    part[t] = cnt;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
        const int32_t v = t >= w ? part[t - w] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t o = part[t] - cnt;
    for (int64_t j = j0; j < j1; ++j)
        if (pf[j].fp64) list[o++] = static_cast<int32_t>(j);
    if (t == 1023) geom->n64 = part[1023];
}

__global__ __launch_bounds__(256) void k_bin_modes(const double4* __restrict__ prm, const double* __restrict__ wt,
                                                   int64_t n, int64_t ldp, int dim, const BinGeom* __restrict__ geom,
                                                   ModeF* __restrict__ out, float* __restrict__ wmat,
                                                   uint2* __restrict__ abase)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (j >= ldp) return;
    const double4 m = prm[j];
    const BinGeom& g = *geom;
    // offsets from the centre are at most half a side per axis
    const double reach = 0.5 * (fabs(m.x) * g.s[0] + fabs(m.y) * g.s[1] + (dim == 3 ? fabs(m.z) * g.s[2] : 0.0));
    ModeF f;
    // revolutions per cell side: the matrix pass multiplies them by offsets in cell sides
    f.ax = static_cast<float>(m.x * g.s[0]);
    f.ay = static_cast<float>(m.y * g.s[1]);
    f.az = static_cast<float>(dim == 3 ? m.z * g.s[2] : 0.0);
    const float wj = j < n ? (wt ? static_cast<float>(wt[j]) : 1.f) : 0.f;
    f.fp64 = reach > kLocalRev ? 1 : 0;
    if (f.fp64) f.ax = f.ay = f.az = 0.f;  // finite fp16 operands (weight 0 in the matrix pass)
    f.w = f.fp64 ? 0.f : wj;
    f.w64 = wj;
    f.pad[0] = f.pad[1] = 0;
    out[j] = f;
    wmat[j] = f.w;
    // the mode's K entries of the matrix pass per lane quarter q (the t_h, t_l slots of q = 2,
    // which depend on the cell, are left zero and filled in by the sum kernel)
    _Float16 bh[3], bl[3];
    split16(f.ax, bh[0], bl[0]);
    split16(f.ay, bh[1], bl[1]);
    split16(f.az, bh[2], bl[2]);
    const _Float16 z = static_cast<_Float16>(0.f);
    abase[j * 4 + 0] = make_uint2(pack_h2(bh[0], bh[0]), pack_h2(bl[0], bh[1]));
    abase[j * 4 + 1] = make_uint2(pack_h2(bh[1], bl[1]), pack_h2(bh[2], bh[2]));
    abase[j * 4 + 2] = make_uint2(pack_h2(bl[2], z), pack_h2(z, z));
    abase[j * 4 + 3] = make_uint2(0u, 0u);
}


// The sum: wave w of the launch takes work item w (kItem slots of one cell).  With offsets
// u = (x - c) / s per axis in cell sides and b = a s in revolutions per side, the phase of mode j at
// point p is t_j + b_j . u_p with t_j = frac(a_j . c + psi_j) reduced in FP64.  For a tile of 16
// modes and a group of 16 points that is one fp16 matrix product with FP32 accumulation,
// [16 x 16] x [16 x 16], whose K entries carry each factor split as hi + lo (fp16 each):
//   k:  bx_h ux_h, bx_h ux_l, bx_l ux_h, by_h uy_h, by_h uy_l, by_l uy_h, bz_h uz_h, bz_h uz_l,
//       bz_l uz_h, t_h 1, t_l 1, then zeros
// (the lo x lo products are below 2^-21 of the local phase, which is under kLocalRev).  Lane l
// holds A[l % 16][4 (l / 16) + e] (mode jt + l % 16) and B[4 (l / 16) + e][l % 16] (point
// 16 g + l % 16), e < 4; the product's lane l holds the phases of modes jt + 4 (l / 16) + e at
// point 16 g + l % 16.  Each lane sums weight x cosine over its four modes; the four lane
// quarters are added at the end.  Modes [j0, j1) of slice blockIdx.y (multiples of 16); with
// several slices the raw sums go to partial[slice][P] at the input index.
typedef _Float16 half4 __attribute__((ext_vector_type(4)));

template <int DIM>
__global__ __launch_bounds__(256, 5) void k_points_binned(const double4* __restrict__ prm, const ModeF* __restrict__ pf,
                                                       const float* __restrict__ wmat,
                                                       const uint2* __restrict__ abase,
                                                       const int32_t* __restrict__ list64, int n,
                                                       const BinGeom* __restrict__ geom,
                                                       const int32_t* __restrict__ item_cell,
                                                       const double4* __restrict__ rec, int64_t P,
                                                       float amp, Epi epi, float* __restrict__ y,
                                                       float* __restrict__ k, uint8_t* __restrict__ ind, int mslice,
                                                       float* __restrict__ partial)
{
    const int lane = threadIdx.x & 63;
    const int64_t item = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const BinGeom gm = *geom;
    if (item >= gm.nitem) return;  // the whole wave
    const int kq = lane >> 4, jl = lane & 15;
    const int j0 = static_cast<int>(blockIdx.y) * mslice;
    const int j1 = min(n, j0 + mslice);
    const int64_t slot0 = item * kItem;

    // the cell centre (FP64)
    double cen[3] = {0.0, 0.0, 0.0};
    int32_t rest = item_cell[item];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int32_t i = rest % gm.n[a];
        rest /= gm.n[a];
        cen[a] = gm.lo[a] + (static_cast<double>(i) + 0.5) * gm.s[a];
    }
    // point operand of each 16-point group: this lane's four K entries of point 16 g + jl
    const _Float16 one = static_cast<_Float16>(1.f), zero = static_cast<_Float16>(0.f);
    half4 bop[kGroups];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const double4 r = rec[slot0 + 16 * g + jl];
        float u[3] = {static_cast<float>(r.x * gm.inv_s[0]), static_cast<float>(r.y * gm.inv_s[1]),
                      DIM == 3 ? static_cast<float>(r.z * gm.inv_s[2]) : 0.f};
        _Float16 h[3], lo[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            asm("" : "+v"(u[a]));  // split the FP32 value (not a fused FP64 -> fp16 conversion)
            split16(u[a], h[a], lo[a]);
        }
        bop[g] = kq == 0 ? half4{h[0], lo[0], h[0], h[1]}
                 : kq == 1 ? half4{lo[1], h[1], h[2], lo[2]}
                 : kq == 2 ? half4{h[2], one, one, zero}
                           : half4{zero, zero, zero, zero};
    }
    float acc[kGroups];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) acc[g] = 0.f;
    const uint32_t msk2 = kq == 2 ? 0xffffffffu : 0u;

    for (int jt = j0; jt < j1; jt += 16) {
        // mode operand: this lane's four K entries of mode jt + jl, the reduced phase at the
        // cell centre (FP64) filling the t_h, t_l slots of the third quarter
        const double4 m = prm[jt + jl];
        const uint2 ab = abase[(jt + jl) * 4 + kq];
        const float4 w = *reinterpret_cast<const float4*>(wmat + jt + 4 * kq);
        double t = DIM == 3 ? fma(m.z, cen[2], m.w) : m.w;
        t = fma(m.y, cen[1], t);
        t = fma(m.x, cen[0], t);
        _Float16 th, tl;
        float tf = static_cast<float>(__builtin_amdgcn_fract(t));
        asm("" : "+v"(tf));  // opaque: the fp16 split converts this FP32 value (one cvt each)
        split16(tf, th, tl);
        const half4 aop = __builtin_bit_cast(
            half4, make_uint2(ab.x | (pack_h2(zero, th) & msk2), ab.y | (pack_h2(tl, zero) & msk2)));
        // a quarter of the groups' products first, then their cosines (no wait on a product just
        // issued; a quarter of the result registers of issuing all of them first)
#pragma unroll
        for (int h = 0; h < kGroups; h += kPipe) {
            f32x4 d[kPipe];
#pragma unroll
            for (int g = 0; g < kPipe; ++g)
                d[g] = __builtin_amdgcn_mfma_f32_16x16x16f16(aop, bop[h + g], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int g = 0; g < kPipe; ++g) {
                const float c0 = cos_rev(d[g][0]), c1 = cos_rev(d[g][1]), c2 = cos_rev(d[g][2]),
                            c3 = cos_rev(d[g][3]);
                float a = acc[h + g];
                a = fmaf(w.x, c0, a);
                a = fmaf(w.y, c1, a);
                a = fmaf(w.z, c2, a);
                a = fmaf(w.w, c3, a);
                acc[h + g] = a;
            }
            // the products, then per group four cosines and four FMAs (independent cosines
            // back to back instead of each waiting on the FMA before it)
            __builtin_amdgcn_sched_group_barrier(0x008, kPipe, 0);
#pragma unroll
            for (int g = 0; g < kPipe; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x400, 4, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
            }
        }
    }
    // totals per point: add the four lane quarters; lane l keeps groups g = kq + 4 u
    float own[kGroups / 4];
#pragma unroll
    for (int u = 0; u < kGroups / 4; ++u) own[u] = 0.f;
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        float v = acc[g] + __shfl_xor(acc[g], 16);
        v += __shfl_xor(v, 32);
        if ((g & 3) == kq) own[g >> 2] = v;
    }
    // modes flagged for the FP64 reduction, in ascending order
    const int n64 = gm.n64;
    if (n64 > 0) {
        double d64[3][kGroups / 4];
#pragma unroll
        for (int u = 0; u < kGroups / 4; ++u) {
            const double4 r = rec[slot0 + 16 * (kq + 4 * u) + jl];
            d64[0][u] = r.x;
            d64[1][u] = r.y;
            d64[2][u] = r.z;
        }
        for (int q = 0; q < n64; ++q) {
            const int j = list64[q];
            if (j < j0 || j >= j1) continue;
            const ModeF f = pf[j];
            const double4 m = prm[j];
            double t = DIM == 3 ? fma(m.z, cen[2], m.w) : m.w;
            t = fma(m.y, cen[1], t);
            t = fma(m.x, cen[0], t);
#pragma unroll
            for (int u = 0; u < kGroups / 4; ++u) {
                double ph = DIM == 3 ? fma(m.z, d64[2][u], t) : t;
                ph = fma(m.y, d64[1][u], ph);
                ph = fma(m.x, d64[0][u], ph);
                own[u] = fmaf(f.w64, cos_rev(static_cast<float>(__builtin_amdgcn_fract(ph))), own[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kGroups / 4; ++u) {
        const double pw = rec[slot0 + 16 * (kq + 4 * u) + jl].w;  // input index, -1 for padding
        if (pw < 0.0) continue;
        const int64_t p = static_cast<int64_t>(pw);
        if (partial) partial[static_cast<int64_t>(blockIdx.y) * P + p] = own[u];
        else epi_store(p, amp * own[u], epi, y, k, ind);
    }
}

}  // namespace

size_t bin_ws_bytes(int64_t P, int64_t ldp)
{
    const BinCaps c = bin_caps(P);
    Carve w(nullptr);
    w.take<double>(6 * kBinBboxBlocks);
    w.take<BinGeom>(1);
    w.take<int32_t>(c.cells);      // counts
    w.take<int32_t>(c.cells);      // offsets
    w.take<int2>(P);               // cell and rank
    w.take<int32_t>(c.items);      // item -> cell
    w.take<double4>(c.slots);      // records: FP64 offset and input index
    w.take<ModeF>(ldp);            // FP32 mode parameters
    w.take<float>(ldp);            // weights of the matrix pass
    w.take<int32_t>(ldp);          // modes of the FP64 pass
    w.take<uint2>(4 * ldp);        // mode operands of the matrix pass
    return w.used;
}

hipError_t launch_points_binned(const double* params, const double* w, int64_t n, int64_t ldp, int dim,
                                const double* xyz, int64_t P, float amp, const Epi& epi, float* y, float* k,
                                uint8_t* ind, void* ws, float* partial, hipStream_t s)
{
    const BinCaps c = bin_caps(P);
    Carve wk(ws);
    double* bbox = wk.take<double>(6 * kBinBboxBlocks);
    BinGeom* geom = wk.take<BinGeom>(1);
    int32_t* count = wk.take<int32_t>(c.cells);
    int32_t* offset = wk.take<int32_t>(c.cells);
    int2* cellrank = wk.take<int2>(P);
    int32_t* item_cell = wk.take<int32_t>(c.items);
    double4* rec = wk.take<double4>(c.slots);
    ModeF* pf = wk.take<ModeF>(ldp);
    float* wmat = wk.take<float>(ldp);
    int32_t* list64 = wk.take<int32_t>(ldp);
    uint2* abase = wk.take<uint2>(4 * ldp);

    const int64_t pblocks = (P + 255) / 256;
    const int nb = static_cast<int>(std::min<int64_t>(kBinBboxBlocks, pblocks));
    if (dim == 3) hipLaunchKernelGGL(k_bin_bbox<3>, dim3(nb), dim3(256), 0, s, xyz, P, bbox);
    else hipLaunchKernelGGL(k_bin_bbox<2>, dim3(nb), dim3(256), 0, s, xyz, P, bbox);
    hipLaunchKernelGGL(k_bin_geom, dim3(1), dim3(256), 0, s, bbox, nb, dim, P, static_cast<double>(kBinTarget),
                       c.cells, geom, count);
    const int64_t cblocks = (P + kCountChunk - 1) / kCountChunk;
    if (dim == 3) hipLaunchKernelGGL(k_bin_count<3>, dim3(cblocks), dim3(256), 0, s, xyz, P, geom, count, cellrank);
    else hipLaunchKernelGGL(k_bin_count<2>, dim3(cblocks), dim3(256), 0, s, xyz, P, geom, count, cellrank);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, geom, count, offset);
    hipLaunchKernelGGL(k_bin_items, dim3(static_cast<unsigned>(c.items)), dim3(kItem), 0, s, geom, offset, item_cell,
                       rec);
    if (dim == 3)
        hipLaunchKernelGGL(k_bin_scatter<3>, dim3(pblocks), dim3(256), 0, s, xyz, P, geom, offset, cellrank, rec);
    else
        hipLaunchKernelGGL(k_bin_scatter<2>, dim3(pblocks), dim3(256), 0, s, xyz, P, geom, offset, cellrank, rec);
    hipLaunchKernelGGL(k_bin_modes, dim3((ldp + 255) / 256), dim3(256), 0, s, reinterpret_cast<const double4*>(params),
                       w, n, ldp, dim, geom, pf, wmat, abase);
    hipLaunchKernelGGL(k_bin_flags, dim3(1), dim3(1024), 0, s, pf, n, geom, list64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    // whole 16-mode tiles per slice, and no slice past the last mode
    const int64_t mslice64 = ((n + bin_mode_slices(P, n) - 1) / bin_mode_slices(P, n) + 15) / 16 * 16;
    const int slices = static_cast<int>((n + mslice64 - 1) / mslice64);
    const int mslice = static_cast<int>(mslice64);
    float* part = slices > 1 ? partial : nullptr;
    const dim3 grid(static_cast<unsigned>((c.items + 3) / 4), static_cast<unsigned>(slices));
    TimedScope timed(s);  // the sum and the slice reduction
    if (dim == 3)
        hipLaunchKernelGGL(k_points_binned<3>, grid, dim3(256), 0, s, reinterpret_cast<const double4*>(params), pf,
                           wmat, abase, list64, static_cast<int>(n), geom, item_cell, rec, P, amp, epi, y, k, ind,
                           mslice, part);
    else
        hipLaunchKernelGGL(k_points_binned<2>, grid, dim3(256), 0, s, reinterpret_cast<const double4*>(params), pf,
                           wmat, abase, list64, static_cast<int>(n), geom, item_cell, rec, P, amp, epi, y, k, ind,
                           mslice, part);
    e = hipGetLastError();
    if (e != hipSuccess || slices == 1) return e;
    return launch_points_reduce(partial, slices, P, amp, epi, y, k, ind, s);
}

}  // namespace grf
