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

// ---------------------------------------------------------------- epilogue
struct Epi {
    float mu;
    int nthr;
    float thr[GRF_MAX_THRESHOLDS];
};

Epi make_epi(const grf_epi* e);

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
    double origin;
    double h;
    int64_t count;  // number of grid points along the axis
    bool with_psi;
    bool conj;      // store (re, -im) for half formats
    int format;
    void* out;      // primary table
    void* out_lo;   // lo table for *_HILO formats
};
hipError_t launch_axis_table(const AxisTableArgs& a, hipStream_t s);

// Per-mode parameters in revolutions: (a_x, a_y, a_z, psi) as double4, [ldp] rows,
// padded modes get a = 0, psi = 0.
hipError_t launch_mode_params(const double* z, const double* phi, int dim, int64_t n, int64_t ldp,
                              const double* ell, double* out, hipStream_t s);

// ---------------------------------------------------------------- direct kernels
hipError_t launch_direct_grid_f32(const float* tx, const float* ty, const float* tz, int64_t n,
                                  int64_t ldp, const int64_t* gn, float amp, const Epi& epi,
                                  float* y, float* k, uint8_t* ind, hipStream_t s);
hipError_t launch_direct_grid_f64(const double* tx, const double* ty, const double* tz, int64_t n,
                                  int64_t ldp, const int64_t* gn, double amp, const Epi& epi,
                                  double mu64, float* y, float* k, uint8_t* ind, double* y64,
                                  double* k64, hipStream_t s);
hipError_t launch_direct_points(const double* params, int64_t n, int dim, const double* xyz,
                                int64_t P, bool fp64, float amp, const Epi& epi, float* y, float* k,
                                uint8_t* ind, hipStream_t s);
hipError_t launch_epilogue(const float* y, int64_t n, const Epi& epi, float* k, uint8_t* ind,
                           hipStream_t s);

// ---------------------------------------------------------------- separable (matrix cores)
// Y[z][y][x] = amp Re sum_j P[x,j] Q[y,j],  P = Ex[x,j] Ez[z,j] (3-D) or Ex (2-D),
// Q = exp(2 pi i (a_y y + psi)).
struct SepArgs {
    int method;            // GRF_SEP_*
    int64_t n, ldp;        // modes, padded row length
    int64_t nx, ny, nz;
    const void* px;        // 2-D: half/bf16 pair table [nx][ldp] (conj); 3-D: float2 [nx][ldp]
    const void* px_lo;     // 2-D X3: lo table
    const void* qy;        // half/bf16 pair table [ny][ldp]
    const void* qy_lo;     // X3: lo table
    const float2* ez;      // 3-D: float2 [nz][ldp]; 2-D: nullptr
    float amp;
    Epi epi;
    float* y;
    float* k;
    uint8_t* ind;
    int tile;              // 0 = default; else tile selector (see sep.hip)
};
hipError_t launch_sep(const SepArgs& a, hipStream_t s);
int sep_tile_count();                // number of tile selectors
void sep_tile_shape(int tile, int* bm, int* bn);

// ---------------------------------------------------------------- adjoint
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
    float* partial;        // workspace [nchunks][5][ldp]
    float* scal_partial;   // workspace [nblocks]
    int64_t nchunks;
};
int64_t bwd_chunks(int64_t P);
// floats of scalar-partial workspace: 4 per reduce block plus 1024 dot partials
inline int64_t bwd_scal_floats(int64_t n) { return 4 * ((n + 255) / 256) + 1024; }
hipError_t launch_backward(const BwdArgs& a, hipStream_t s);

}  // namespace grf
