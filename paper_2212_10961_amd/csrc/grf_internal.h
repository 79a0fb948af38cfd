// Internal declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "grf.h"

namespace grf {

// ---------------------------------------------------------------- errors
// Sets the thread-local message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail_hip(hipError_t e, const char* what);

#define GRF_HIP(call)                                         \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::grf::fail_hip(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- validation (host)
int check_modes(const grf_modes* m, const char* fn);
int check_grid(const grf_grid* g, int dim, const char* fn);
// Epilogue of a call: required when k or ind is written; ind needs a threshold; ascending.
int check_epi(const grf_epi* e, const float* k, const uint8_t* ind, const char* fn);
// Axis-aligned view of a table (a rotated table's k written to kbuf; see grf_modes).
hipError_t aligned_modes(const grf_modes* m, void* kbuf, hipStream_t s, grf_modes* out);
inline bool is_sep(int m) { return m >= GRF_SEP_BF16 && m <= GRF_SEP_F16_X3; }
inline bool is_hilo(int m) { return m == GRF_SEP_BF16_X3 || m == GRF_SEP_F16_X3; }
inline bool is_bf16(int m) { return m == GRF_SEP_BF16 || m == GRF_SEP_BF16_X3; }

// ---------------------------------------------------------------- kernel timer
// Records an event pair around the main kernel of a call while the timer is enabled.
void timer_mark(hipStream_t s, bool begin);
// While the timer is enabled: the next event pair, for a launch that records its own start
// and stop on the dispatch (hipExtLaunchKernel), which adds no marker packets to the stream.
bool timer_take_pair(hipEvent_t* start, hipEvent_t* stop);
struct TimedScope {
    hipStream_t s;
    bool on;
    explicit TimedScope(hipStream_t st, bool enabled = true) : s(st), on(enabled)
    {
        if (on) timer_mark(s, true);
    }
    ~TimedScope()
    {
        if (on) timer_mark(s, false);
    }
};

// ---------------------------------------------------------------- epilogue
// Applied to each cell's Y before the stores of the sum kernels (Sec. 4.1 scaling, Sec. 3.1
// single truncation): K = exp(mu + Y), facies index #{q : thr[q] < Y}.
struct Epi {
    float mu;
    int nthr;
    float thr[GRF_MAX_THRESHOLDS];
};

Epi make_epi(const grf_epi* e);

// Output pointers are global memory: as global (not flat) stores they count only against the
// vector-memory counter, so later LDS waits do not wait for them.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* global_ptr(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ void epi_store(int64_t c, float yv, const Epi& e, float* __restrict__ y,
                                          float* __restrict__ k, uint8_t* __restrict__ ind)
{
    if (y) global_ptr(y)[c] = yv;
    if (k) global_ptr(k)[c] = expf(e.mu + yv);
    if (ind) {
        int f = 0;
        for (int q = 0; q < e.nthr; ++q) f += (yv > e.thr[q]) ? 1 : 0;
        global_ptr(ind)[c] = static_cast<uint8_t>(f);
    }
}

// Bitruncated (pluri-Gaussian) rule over two fields (Sec. 3.1), a pass of its own after both
// fields are stored: facies rule[i * (ns + 1) + j], i = #{q : t[q] < Y1}, j = #{q : s[q] < Y2},
// value values[facies].  The rule and the values sit in device memory.
struct PluriEpi {
    int nt, ns;
    float t[GRF_MAX_THRESHOLDS];
    float s[GRF_MAX_THRESHOLDS];
    const uint8_t* rule;
    const float* values;
};

// Device copy of a rule's lookup tables (bin -> facies bytes, then the facies values).
constexpr size_t kRuleBytes = 256 + sizeof(float) * GRF_MAX_FACIES;
hipError_t launch_rule_tables(const grf_trunc2& r, void* dst, hipStream_t s);
hipError_t launch_pluri_epilogue(const float* y1, const float* y2, int64_t n, const PluriEpi& pe, uint8_t* facies,
                                 float* value, hipStream_t s);

// ---------------------------------------------------------------- sizes
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Padded mode count used for every per-mode table row (multiple of 64 so that
// mode chunks of the kernels never straddle the end of a row).
inline int64_t padded_modes(int64_t n) { return round_up(n, 64); }

// Bump allocator over a caller workspace.
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(void* p) : base(static_cast<char*>(p)) {}
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += align256(count * sizeof(T));
        return p;
    }
};

// ---------------------------------------------------------------- table formats
enum TableFormat : int {
    TF_REV_F32 = 0,   // float: frac(a x + psi) in revolutions
    TF_REV_F64 = 1,   // double: frac(a x + psi)
    TF_CPLX_F32 = 2,  // float2: (cos, sin)(2 pi frac)
    TF_F16 = 3,       // half2 (re, s*im), s = +1 or -1 (conj)
    TF_F16_HILO = 4,  // two half2 tables: hi and lo parts
    TF_BF16 = 5,
    TF_BF16_HILO = 6,
};

// Per-axis phase table (FP64 range reduction):
//   t[i][j] = frac(a_j x_i + (with_psi ? psi_j : 0)),  a_j = z[axis*n + j] / (2 pi ell),
//   x_i = o + (i + 1/2) h,  psi_j = phi_j / (2 pi).
// Rows are `ldp` entries long; entries j in [n, ldp) are written as zero phase
// (format-specific zero: 0 rev, or (0,0) complex).
struct AxisTableArgs {
    const double* z;
    const double* phi;
    int64_t n;
    int64_t ldp;
    int axis;
    double ell;
    double freq_scale;  // 1 / (2 pi ell): revolutions per unit length per unit of z
    double origin;
    double h;
    int64_t count;  // number of grid points along the axis
    bool with_psi;
    bool conj;      // store (re, -im) for half formats
    bool fast_trig; // cos/sin of the FP64-reduced fraction by the hardware units (FP32);
                    // for tables rounded to one fp16/bf16 (or FP32) pass, else FP64 sincospi
    bool blocked;   // stage-major layout [ldp / 32][count][32] (the separable operands: one
                    // 32-mode stage of every row is contiguous), else row-major [count][ldp]
    int format;
    void* out;      // primary table
    void* out_lo;   // lo table for *_HILO formats
    const double* w;  // per-mode weights folded into complex entries (exp(i 2 pi f) * w_j), or nullptr
};
hipError_t launch_axis_table(const AxisTableArgs& a, hipStream_t s);
hipError_t launch_axis_tables(const AxisTableArgs* d, int nd, hipStream_t s);  // nd <= 6, one launch
int64_t axis_table_blocks(const AxisTableArgs& a);  // 256-thread work blocks one table needs

// Table layout of eval_field_grid for a resolved method (base == nullptr: measure only),
// and the descriptors of the tables it builds (returns how many, <= 3).
struct GridWs {
    void* t[3] = {nullptr, nullptr, nullptr};
    void* tlo[3] = {nullptr, nullptr, nullptr};
    void* partial = nullptr;  // DIRECT_F64 on small grids, FP64; separable mode split, FP32:
                              // per-slice sums
    int slices = 1;           // separable mode split: slices of `pairs` stage pairs each
    int64_t pairs = 0;
    size_t split_bytes = 0;   // bytes of the separable split's sums (the last part of `bytes`)
    size_t bytes = 0;
};
GridWs grid_ws(const grf_modes* m, const grf_grid* g, int method, void* base);
// grad_z[b n + j] = (1/ell_b) sum_a rot_ab grad_k[a n + j] (rot host row-major or nullptr = I).
hipError_t launch_grad_z(const float* gk, int dim, int64_t n, const double* rot, const double* ell, float* gz,
                         hipStream_t s);
// Validated workspace bytes of a grid evaluation: all of it, and the least that it runs in (the
// tables without the mode split's sums; the split is then not taken).
int grid_ws_bytes(const char* fn, const grf_modes* modes, const grf_grid* grid, int method, size_t* bytes,
                  size_t* least);
// eval_field_grid(_tile) after the entry point's name: validation, then tables and sum in `ws`.
int grid_eval(const char* fn, const grf_modes* modes, const grf_grid* grid, int method, int tile,
              const grf_epi* epi, float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes, void* stream);
int grid_table_descs(const grf_modes* m, const grf_grid* g, int method, const GridWs& w, AxisTableArgs* out);

// Rotated tables: out[a * n + j] = sum_b rot[3a + b] z[b * n + j] / ell[b] (device, FP64).
hipError_t launch_rotate_modes(const double* z, int dim, int64_t n, const double* rot, const double* ell, double* out,
                               hipStream_t s);
// Workspace of the axis-aligned copy of a rotated table (0 for axis-aligned tables).
inline size_t rot_ws_bytes(const grf_modes* m)
{
    return m->rotated ? align256(sizeof(double) * size_t(m->dim) * size_t(m->n)) : 0;
}

// Per-mode parameters in revolutions: (a_x, a_y, a_z, psi) as double4, [ldp] rows,
// padded modes get a = 0, psi = 0.
hipError_t launch_mode_params(const double* z, const double* phi, int dim, int64_t n, int64_t ldp,
                              const double* ell, double* out, hipStream_t s);

// ---------------------------------------------------------------- direct kernels
// `w`: device per-mode weights [n] or nullptr (all 1).
hipError_t launch_direct_grid_f32(const float* tx, const float* ty, const float* tz, const double* w, int64_t n,
                                  int64_t ldp, const int64_t* gn, float amp, const Epi& epi,
                                  float* y, float* k, uint8_t* ind, hipStream_t s);
// Mode slices of the FP64 grid sum: grids too small to fill the device split the modes
// into `slices` runs of `mslice` (slices = 1: no split).
struct ModeSlices {
    int slices;
    int64_t mslice;
};
ModeSlices direct_grid_f64_slices(const int64_t* gn, int64_t n);
// `partial` (workspace of direct_grid_f64_slices(gn, n).slices * cells doubles when that is
// > 1, else unused) receives the slices' raw sums before they are added in slice order.
hipError_t launch_direct_grid_f64(const double* tx, const double* ty, const double* tz, const double* w, int64_t n,
                                  int64_t ldp, const int64_t* gn, double amp, const Epi& epi,
                                  double mu64, float* y, float* k, uint8_t* ind, double* y64,
                                  double* k64, double* partial, hipStream_t s);
// `partial` (workspace, points_mode_slices(P, n) * P floats when that is > 1) receives the
// per-slice sums when the modes are split across blocks.
hipError_t launch_direct_points(const double* params, const double* w, int64_t n, int dim, const double* xyz,
                                int64_t P, bool fp64, float amp, const Epi& epi, float* y, float* k,
                                uint8_t* ind, float* partial, hipStream_t s);
constexpr int kPointsPerLane = 8;
int points_mode_slices(int64_t P, int64_t n);
hipError_t launch_epilogue(const float* y, int64_t n, const Epi& epi, float* k, uint8_t* ind,
                           hipStream_t s);
// out[p] = epilogue(amp * sum over slices of partial[slice][p]), slices added in order.
hipError_t launch_points_reduce(const float* partial, int slices, int64_t P, float amp, const Epi& epi, float* y,
                                float* k, uint8_t* ind, hipStream_t s);

// ---------------------------------------------------------------- binned point sum (points.hip)
// Points sorted into cells of their bounding box (sides about equal, each axis cut into a whole
// number of them), each cell's slots padded to whole work items of kBinItemSlots; per (mode,
// work item) the phase at the cell centre is reduced in FP64 and the points' local phases are
// formed in FP32 by a matrix product on the matrix cores.
constexpr int kBinItemSlots = 256;     // points per work item (one wave: 16 groups of 16)
constexpr int kBinTarget = 2048;       // points per cell on average
constexpr int kBinBboxBlocks = 512;    // blocks of the bounding-box pass
constexpr int64_t kBinMinPoints = int64_t(1) << 16;  // GRF_DIRECT_F32 bins from this many points
constexpr int64_t kBinMaxPoints = int64_t(1) << 30;  // (slot indices are 32-bit)
struct BinGeom {
    double lo[3];      // bounding-box corner
    double s[3];       // cell side per axis (each axis of the box holds a whole number of cells)
    double inv_s[3];   // and its reciprocal
    int32_t n[3];      // cells per axis (x fastest)
    int32_t ncell;
    int64_t nslot;     // sorted slots: every cell padded to whole work items
    int64_t nitem;     // nslot / kBinItemSlots
    int32_t n64;       // modes whose local phase is reduced per point in FP64
    int32_t pad_;
};
struct BinCaps {
    int64_t cells, slots, items;
};
inline BinCaps bin_caps(int64_t P)
{
    BinCaps c;
    c.cells = P / (kBinTarget / 2) + 64;
    c.items = (P + (kBinItemSlots - 1) * c.cells + kBinItemSlots - 1) / kBinItemSlots;
    c.slots = c.items * kBinItemSlots;
    return c;
}
// Mode slices of the binned sum (partial sums per slice when > 1).
int bin_mode_slices(int64_t P, int64_t n);
// Workspace of the binned pass for P points and ldp padded modes (the per-slice partial sums
// excluded: bin_mode_slices(P, n) * P floats when that is > 1).
size_t bin_ws_bytes(int64_t P, int64_t ldp);
hipError_t launch_points_binned(const double* params, const double* w, int64_t n, int64_t ldp, int dim,
                                const double* xyz, int64_t P, float amp, const Epi& epi, float* y, float* k,
                                uint8_t* ind, void* ws, float* partial, hipStream_t s);

// ---------------------------------------------------------------- separable (matrix cores)
// Y[z][y][x] = amp Re sum_j P[x,j] Q[y,j],  P = Ex[x,j] Ez[z,j] (3-D) or Ex (2-D),
// Q = exp(2 pi i (a_y y + psi)).
struct SepArgs {
    int method;            // GRF_SEP_*
    int64_t n, ldp;        // modes, padded row length
    int64_t nx, ny, nz;
    const void* px;        // x side, (Re, -Im) pairs [nx][ldp]: half/bf16 pairs, except
                           // 3-D hi+lo where it is float2 (the product with Ez is formed on chip)
    const void* px_lo;     // 2-D X3: lo table
    const void* qy;        // half/bf16 pair table [ny][ldp]
    const void* qy_lo;     // X3: lo table
    const float2* ez;      // 3-D: float2 [nz][ldp]; 2-D: nullptr
    float amp;
    Epi epi;
    float* y;
    float* k;
    uint8_t* ind;
    int tile;              // < 0: size-based default; else tile selector (see sep.hip)
    bool timed = false;    // the call's main kernel: timed by the kernel timer when it is on
    // Mode split (default tile, grids of fewer blocks than CUs): blockIdx.y = slice sums
    // stage pairs [slice pairs, (slice + 1) pairs) into partial[slice][nx ny nz]; a second
    // pass adds the slices in order and applies amp and the epilogue.  nullptr: no split.
    float* partial = nullptr;
    int slices = 1;
    int64_t pairs = 0;
};
hipError_t launch_sep(const SepArgs& a, hipStream_t s);
// Two fields on the same grid (same method, sizes and ldp; the epilogue parameters of `a`
// apply to both) in one launch; b may be nullptr.
hipError_t launch_sep_pair(const SepArgs& a, const SepArgs* b, hipStream_t s);
int sep_tile_count();                // number of tile selectors
void sep_tile_shape(int tile, int* bm, int* bn);
int sep_tile_slices(int tile, int method, bool d3);  // z-slices per block
int sep_default_tile(int method, int64_t nx, int64_t ny, int64_t nz);
// Mode slices of the default tile for one field (1: no split); *pairs = stage pairs per slice.
int sep_mode_slices(int method, int dim, int64_t nx, int64_t ny, int64_t nz, int64_t ldp, int64_t* pairs);

// ---------------------------------------------------------------- batched (persistent) launches
// Generated operands of the 2-D one-pass separable batch tiles.  With E_j(x) = e^{2 pi i a_x x}
// and Q_j(y) = w_j e^{2 pi i (a_y y + psi_j)}, a tile at (x0, y0) of an instance is
//   Y[y0 + s][x0 + r] = A Re sum_j [Q_j(y0 + s) E_j(x0)] R_j(r),   R_j(r) = e^{2 pi i a_x r hx},
// so its x-side operand R is the same for every tile of the instance (a local table of
// kGenRows rows made once per batch call), and only the y side, which carries the tile's
// x0 phase, is generated on chip per tile.
constexpr int kGenRows = 128;  // rows of the local x table (the widest tile)
struct alignas(16) GenMode {
    double ax, ay;  // revolutions per unit length along x and y
    double psi;     // phase of cell (0, 0): psi_j + a_y (oy + hy / 2) + a_x (ox + hx / 2)
    float w;        // weight (0 for padding modes)
    float rc, rs;   // e^{2 pi i frac(a_y hy)}: the step from one row to the next
    float pad_[3];
};
static_assert(sizeof(GenMode) == 48, "three 16-byte loads per mode");
struct GenModeDesc {
    const double* z;    // [2][n]
    const double* phi;  // [n]
    const double* w;    // [n] or nullptr
    int64_t n, ldp;
    double fsx, fsy;    // 1 / (2 pi ell_x), 1 / (2 pi ell_y)
    double ox, oy, hx, hy;
    GenMode* out;       // [ldp]
};
// out[j] of every descriptor (one block row per instance, ldp_max >= every ldp).
hipError_t launch_gen_modes(const GenModeDesc* d, int n_inst, int64_t ldp_max, hipStream_t s);
struct GenArgs {
    const uint32_t* rx;  // local x table: stage-major [ldp / 32][kGenRows][32] (Re, -Im) fp16/bf16 pairs
    const GenMode* md;   // [ldp]
    double hx, hy;
};

// One descriptor per instance; work items [item0, item0 + tiles_x * tiles_y * nz) belong to it.
struct SepBatchItem {
    SepArgs a;
    GenArgs g;        // used when the launch generates its operands (2-D one-pass forms)
    int64_t item0;
    int32_t tiles_x, tiles_y;
    int32_t variant;  // 0: 128x128 tiles, 1: 64x64 tiles
    int32_t pad_;
};
// Work queues of the separable persistent launch: queue q holds the work items
// [start, start + count) and counts them on counters[q * kQueueStride].  Each block starts on
// the queue of the accelerator complex (XCD, with its own L2) it runs on, so that the tiles
// of one instance, which share operand rows, run side by side under one L2; once its queue
// is drained it takes work from the next queues in turn.
constexpr int kMaxQueues = 8;     // XCDs of the device
constexpr int kQueueStride = 32;  // counters 256 B apart
struct BatchQueue {
    int64_t start, count;
};
hipError_t launch_sep_batch(int method, bool d3, const SepBatchItem* items, int n_inst, const BatchQueue* queues,
                            int nq, unsigned long long* counters, int grid, hipStream_t s);
int sep_batch_blocks_per_cu(int method, bool d3);
// The 2-D one-pass forms (SEP_F16, SEP_BF16) generate their operands on chip in the batch.
inline bool sep_batch_generates(int method, bool d3)
{
    return !d3 && (method == GRF_SEP_F16 || method == GRF_SEP_BF16);
}

struct DirectBatchItem {
    const float* tx;
    const float* ty;
    const float* tz;
    const double* w;  // per-mode weights or nullptr
    float* y;         // outputs of the instance, each may be nullptr
    float* k;
    uint8_t* ind;
    Epi epi;
    int64_t ldp;
    int64_t nq;       // ny * nz
    int64_t item0;
    int32_t n, nx, ny, nxt;  // nxt: 64-cell tiles along x
    float amp;
    int32_t pad_;
};
hipError_t launch_direct_batch(const DirectBatchItem* items, int n_inst, int64_t total,
                               unsigned long long* counter, int grid, hipStream_t s);
int direct_batch_blocks_per_cu();
constexpr int kDirectTile = 64;  // cells per tile side of the direct grid kernel

// Batched per-axis tables: one launch over many AxisTableArgs (device array).  blk[b]
// (device, total_blocks entries) = (descriptor << 40) | work block within that table, for
// work blocks 0 .. axis_table_blocks(descriptor) - 1 of every descriptor.
hipError_t launch_axis_tables_batched(const AxisTableArgs* descs, const uint64_t* blk, int64_t total_blocks,
                                      hipStream_t s);
// p[i * stride] = v for i < n (n <= 64).
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, int stride, hipStream_t s);

// ---------------------------------------------------------------- adjoint
// Separable dense adjoint on a grid, x in chunks of kBwdSepK cells: per mode j,
// S_j = sum_c g_c e^{i theta_jc} = sum_q [sum_x g[q][x] Ex[x][j]] Ey[y_q][j] Ez[z_q][j] over the
// rows q = (y, z), the bracket (and its x-weighted twin) as a bf16 hi+lo matrix product.
constexpr int kBwdSepK = 128;
struct BwdSep {
    uint16_t* ga_hi;       // qp x kBwdSepK bf16 hi / lo of dL/dY rows z nyp + y (fragment-major)
    uint16_t* ga_lo;
    uint16_t* ex_hi;       // [4 ldp][kBwdSepK] rows 4 j + (Re Ex, Im Ex, x Re Ex, x Im Ex)
    uint16_t* ex_lo;
    const float2* ey;      // [nyp][ldp] e^{2 pi i (a_y y + psi)} (rows past ny: finite, unused)
    const float2* ez;      // [nz][ldp] e^{2 pi i a_z z} (one row of 1 in 2-D)
    const double* zx;      // x components of the (axis-aligned) wavevector table, [n]
    double fsx;            // 1 / (2 pi ell_x)
    int64_t ny, nyp, nz;   // y extent, padded to a multiple of 32, z extent (1 in 2-D)
    int64_t qp;            // rows nyp nz
    int64_t chunks;        // row chunks (partial sums)
};
int64_t bwd_sep_chunks(int64_t ldp, int64_t qp);

struct BwdArgs {
    const double* params;  // [ldp] double4 (a_x, a_y, a_z, psi) in revolutions
    int64_t n, ldp;
    int dim;
    const double* xyz;     // points [P][dim] or nullptr for grid
    const int64_t* gn;     // grid dims (host) when xyz == nullptr
    const double* go;      // grid origin (host)
    const double* gh;      // grid spacing (host)
    int64_t P;
    const float* gy;
    const float* ysaved;
    float amp, sigma;
    const double* ell;     // host
    const double* z;       // device modes z (for grad_ell)
    float* gphi;
    float* gk;
    float* gsigma;
    float* gell;
    const double* w;       // device per-mode weights or nullptr
    const double* rot;     // host row-major 3 x 3 when the table is rotated (z, ell are the
                           // original table's; params hold k = rot diag(1/ell) z), else nullptr
    const float* tx;       // grid path: FP32 revolution tables (psi in ty), or nullptr
    const float* ty;
    const float* tz;
    float* partial;        // workspace [nchunks][5][ldp]
    float* scal_partial;   // workspace [nblocks]
    int64_t nchunks;
    const BwdSep* sep;     // grid path: separable form (host struct), or nullptr
};
int64_t bwd_chunks(int64_t P);
// floats of scalar-partial workspace: 4 per reduce block plus 1024 dot partials
inline int64_t bwd_scal_floats(int64_t n) { return 4 * ((n + 255) / 256) + 1024; }
hipError_t launch_backward(const BwdArgs& a, hipStream_t s);

// ---------------------------------------------------------------- conditioning (kriging)
enum KrigeKind : int { KR_GAUSS = 0, KR_EXP = 1, KR_M32 = 2, KR_M52 = 3 };
struct KrigeModel {
    int kind;           // KrigeKind
    double s2;          // sigma^2
    double nugget_abs;  // nugget * sigma^2 on the diagonal
    double mt[9];       // M^T row-major, M = R diag(1/ell) (dim 2: zero third row/column)
};
struct KrigeTarget {
    bool grid;
    int dim;
    int64_t count;      // cells or points
    int64_t n[3];       // grid
    double o[3], h[3];
    const double* xyz;  // points [count][dim]
};
hipError_t launch_cov_matrix(const double* x, int64_t m, int dim, const KrigeModel& km, double* C, int64_t lda,
                             hipStream_t s);
// Blocked Cholesky A = L L^T (64-wide blocks; A's lower triangle is consumed) with the forward
// substitution L z = r: L below the diagonal blocks goes, transposed, to A's upper triangle;
// the inverses of the diagonal factors to `dinv` (ceil(m / 64) blocks of 64 x 64 doubles); r
// (m doubles) is updated in place and z (m doubles) receives every block of z but the last.
hipError_t launch_cholesky(double* A, int64_t m, int64_t lda, double* dinv, double* r, double* z, int32_t* info,
                           hipStream_t s);
// Backward substitution L^T x = z with the output of launch_cholesky (z is overwritten).
hipError_t launch_chol_back(const double* A, int64_t m, int64_t lda, const double* dinv, const double* r, double* z,
                            double* x, hipStream_t s);
hipError_t launch_residual(const float* d, const float* y, int64_t m, double* r, hipStream_t s);
hipError_t launch_krige_stage(const double* x, const double* alpha, int64_t m, int dim, const KrigeModel& km,
                              float4* out, hipStream_t s);
hipError_t launch_krige_apply(const float4* obs, const double* xobs, int64_t m, const KrigeModel& km,
                              const KrigeTarget& tg, float* y, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, hipStream_t s);

}  // namespace grf
