/*
 * grf.h -- C ABI of the MI355X (gfx950) spectral Gaussian-random-field library.
 *
 * The library evaluates the random-phase form of the discrete spectral sum of
 * Icardi et al. (2022), Sec. 4.1 eq. DiscreteFT,
 *
 *     Y(x) = sqrt(2 sigma^2 / N) * sum_{j<N} cos(k_j . x + phi_j),   k_{j,a} = z_{j,a} / ell_a,
 *
 * at structured-grid cell centres or at arbitrary points, with wavevectors z_j drawn
 * from the normalised spectral density of the covariance (App. A) and anisotropic
 * correlation lengths by per-axis rescaling of frequency space (Sec. 4.1), followed
 * by the log-normal scaling K = exp(mu + Y) or the truncation rule of Sec. 3.1.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: GRF_OK (0) or a negative GRF_E* code.
 *    No function throws, aborts or exits.  On failure grf_last_error() returns a
 *    message for the calling thread.
 *  - Argument validation happens on the host before anything is enqueued: an
 *    invalid call enqueues no work and leaves outputs untouched.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary process memory.  All buffers are owned by the caller.
 *    The library allocates device memory only inside a grf_plan (batched path).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Device
 *    work is enqueued asynchronously on it; the library never synchronises the
 *    device except inside grf_plan_create/destroy and the autotuner.
 *  - Grid cells are ordered with the x index fastest: c = i + nx (j + ny k).
 *    Cell centres are origin_a + (i_a + 1/2) h_a.
 *  - Mode tables are axis-major: z[a * n + j] for axis a < dim, mode j < n.
 *  - Calls on different streams, or from different threads, are independent.
 */
#ifndef GRF_H
#define GRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRF_VERSION 10100 /* 1.1.0: rotated and weighted tables, bitruncated rule, kriging */

/* status codes */
#define GRF_OK 0
#define GRF_EINVAL (-1)       /* bad spec, shape, method or null required pointer */
#define GRF_ENOMEM (-2)       /* workspace too small, or plan allocation failed */
#define GRF_EDEVICE (-3)      /* HIP runtime error (message carries hipGetErrorString) */
#define GRF_EUNSUPPORTED (-4) /* valid but unsupported combination (e.g. separable on points) */

/* covariance families (App. A) */
#define GRF_COV_GAUSSIAN 0    /* C(r) = sigma^2 exp(-|r/ell|^2), eq. gauSpe */
#define GRF_COV_EXPONENTIAL 1 /* C(r) = sigma^2 exp(-|r/ell|),   eq. expSpe */
#define GRF_COV_MATERN 2      /* eq. matSpe with 2*nu a positive integer <= 64 */

/* evaluation methods */
#define GRF_AUTO (-1)       /* separable FP16 on grids with >= 2^16 cells, else DIRECT_F32 */
#define GRF_DIRECT_F32 0    /* one cos per mode and cell, FP64 per-axis phase reduction */
#define GRF_DIRECT_F64 1    /* FP64 throughout (small problems, reference-grade) */
#define GRF_SEP_BF16 2      /* matrix-core contraction, bf16 tables, one pass */
#define GRF_SEP_F16 3       /* matrix-core contraction, fp16 tables, one pass */
#define GRF_SEP_BF16_X3 4   /* bf16 hi+lo split tables, three passes */
#define GRF_SEP_F16_X3 5    /* fp16 hi+lo split tables, three passes */
/* point sums only (eval_field_points, eval_pluri_points): the two forms GRF_DIRECT_F32 picks from */
#define GRF_DIRECT_F32_BINNED 6    /* points binned in cells, FP64 phase per (mode, cell), FP32 offsets */
#define GRF_DIRECT_F32_POINTWISE 7 /* FP64 phase per (mode, point) */

#define GRF_MAX_THRESHOLDS 15
#define GRF_MAX_FACIES 64

/* Generator options (App. B dictionary: correlation, Kmean, Ksigma, Lcorr, nu, nfreq,
 * disableY/disableZ as dim).  make_modes reads dim, cov, n_modes, seed and nu (the
 * standardised table does not depend on the scalars); grf_modes_init reads dim, n_modes,
 * sigma2, ell and len_convention; mu is the caller's grf_epi.mu. */
typedef struct grf_spec {
    int32_t dim;            /* 2 or 3 */
    int32_t cov;            /* GRF_COV_* */
    double sigma2;          /* variance of Y (of ln K), >= 0 */
    double mu;              /* mean of ln K (copied by the caller into grf_epi.mu) */
    double ell[3];          /* correlation lengths per axis, > 0 (ell[2] ignored for dim 2) */
    int64_t n_modes;        /* N >= 1 */
    uint64_t seed;          /* Philox4x32-10 key */
    int32_t len_convention; /* 0: ell as above; 1: ell given as the paper's length lambda:
                               Gaussian ell = 2 lambda / sqrt(pi) (eq. gauSpe writes the
                               correlation as exp(-(pi/4)(r/lambda)^2)); the exponential and
                               Matern forms take lambda as ell unchanged */
    double nu;              /* Matern smoothness; 2*nu must be an integer in [1, 64] */
} grf_spec;

/* A mode table in device memory plus the scalars that enter the field.
 * Anisotropy: k_j = z_j / ell per axis (Sec. 4.1), or with rotated = 1 the general map
 * k_j = rot diag(1/ell) z_j (the extension to rotations and general transformation
 * matrices named in Sec. 4.1 and in the conclusions, Sec. 6).  With an orthonormal rot the
 * covariance's principal axes are the columns of rot, with correlation lengths ell.
 * Evaluations of a rotated table need dim * n * 8 more workspace bytes (included in every
 * *_ws_size); the batched path does not take rotated tables (GRF_EUNSUPPORTED). */
typedef struct grf_modes {
    int32_t dim;        /* 2 or 3 */
    int32_t pad_;
    int64_t n;          /* number of modes N >= 1 */
    const double* z;    /* device, [dim][n]: standardised wavevectors */
    const double* phi;  /* device, [n]: phases in radians */
    double sigma;       /* standard deviation, amplitude = sigma * sqrt(2 / N) */
    double ell[3];      /* correlation lengths (> 0) */
    int32_t rotated;    /* 0 or 1 */
    int32_t pad2_;
    double rot[9];      /* row-major 3 x 3 (dim 2 uses the upper-left 2 x 2 block); finite */
    const double* w;    /* device, [n] per-mode weights, or NULL (all 1):
                           Y = sigma sqrt(2/N) sum_j w_j cos(k_j . x + phi_j) */
} grf_modes;

/* Structured grid: centres origin + (i + 1/2) h, x index fastest; n[2] = 1 for dim 2. */
typedef struct grf_grid {
    int64_t n[3];
    double origin[3];
    double h[3];
} grf_grid;

/* Epilogue applied to Y before the store (Sec. 4.1 scaling, Sec. 3.1 truncation rule). */
typedef struct grf_epi {
    float mu;                                /* K = exp(mu + Y) (written when k != NULL) */
    int32_t n_thresholds;                    /* facies index = #{i : t_i < Y} (when ind != NULL);  */
    float thresholds[GRF_MAX_THRESHOLDS];    /* one threshold t gives I = [Y > t] (strict) */
} grf_epi;

/* Library version (GRF_VERSION of the build). */
int grf_version(void);

/* Message for the last failed call on this thread ("" if none).  Never NULL. */
const char* grf_last_error(void);

/*
 * make_modes -- draw a mode table on the host (App. A spectral densities; phases for
 * Sec. 4.1 eq. DiscreteFT in its random-phase reading).
 *   spec    host; validated (dim, cov, n_modes >= 1, nu for Matern).
 *   z_out   host, [dim][n_modes] doubles, written.
 *   phi_out host, [n_modes] doubles in [0, 2 pi), written.
 * Philox4x32-10 keyed by spec->seed, counter (j lo, j hi, slot, 0); Box-Muller normals.
 * Gaussian z = sqrt(2) g; exponential z = g / |h0|; Matern z = g sqrt(2nu / chi2_{2nu}).
 * Deterministic in (dim, cov, nu, n_modes, seed); a prefix of a longer table equals the
 * shorter table.  Does not touch the GPU.
 */
int make_modes(const grf_spec* spec, double* z_out, double* phi_out);

/*
 * grf_modes_init -- the grf_modes descriptor of a table drawn for `spec`: dim, n = n_modes,
 * sigma = sqrt(sigma2), ell per axis after the len_convention conversion (ell[a] = 1 for
 * a >= dim), axis-aligned (rotated = 0, rot = I), no weights (w = NULL).
 *   spec  host; validated (dim, cov, n_modes >= 1, sigma2 finite and >= 0, ell[a < dim]
 *         finite and > 0, len_convention 0 or 1).
 *   z, phi  the table's device arrays ([dim][n_modes], [n_modes]); stored, not read.
 *   out   host, written only on success.  Pure host code; does not touch the GPU.
 */
int grf_modes_init(const grf_spec* spec, const double* z, const double* phi, grf_modes* out);

/*
 * make_modes_lattice -- the fixed-frequency, Gaussian-weight form of Sec. 4.1 eq. DiscreteFT
 * (read as the real sum sum_j c_j [W_j cos(k_j . x) + W'_j sin(k_j . x)], W, W' independent
 * N(0,1), c_j^2 = sigma^2 S(u_j) / sum_i S(u_i), S the standardised spectral density of App. A):
 * frequencies on the half-space lattice of N = m^dim / 2 points with spacing du
 * (standardised units; k = u / ell): mode j = i0 + (m/2)(i1 + m i2) has u_0 = du (i0 + 1/2),
 * u_a = du (i_a - m/2 + 1/2) for a > 0.  (W_j, W'_j) is the Box-Muller pair of draw slot 1
 * of Philox counter j.  Written as a weighted table: z = u, phi_j = -atan2(W'_j, W_j) mod 2 pi,
 * w_j = sqrt(N/2 * p_j * (W_j^2 + W'_j^2)), so that grf_modes{z, phi, sigma, ell, w}
 * evaluates the sum exactly.
 *   spec     host: dim, cov (nu for Matern), seed; spec->n_modes must equal m^dim / 2.
 *   m        even, >= 2;  du > 0.
 *   z_out [dim][N], phi_out [N], w_out [N]: host arrays, written.
 */
int make_modes_lattice(const grf_spec* spec, int32_t m, double du, double* z_out, double* phi_out, double* w_out);

/*
 * snap_periodic -- the "periodic" option of App. B: every wavevector is moved to the nearest
 * point of the lattice of a box with periods L_a, k_a = 2 pi m_a / L_a with
 * m_a = round(k_a L_a / (2 pi)) (halves away from zero), along each axis with
 * period[a] > 0 (other axes untouched), where k = rot diag(1/ell) z (rot = NULL: identity;
 * else row-major 3 x 3, dim 2 uses the upper-left block, orthonormal to 1e-9).  The result
 * is returned standardised, z_out = diag(ell) rot^T k, so that a table with these ell and
 * rot evaluates the snapped k; the field then repeats with period L_a along axis a.
 * Host arrays: z, z_out [dim][n] (may alias), ell [dim] > 0, period [dim].  No GPU work.
 */
int snap_periodic(int dim, int64_t n, const double* z, const double* ell, const double* rot, const double* period,
                  double* z_out);

/* Device workspace (bytes) that eval_field_grid takes for this problem and method, including
 * the sums of the separable mode split where it applies (see eval_field_grid). */
int eval_field_grid_ws_size(const grf_modes* modes, const grf_grid* grid, int method, size_t* bytes);

/*
 * eval_field_grid -- Y, K and/or facies index at every cell centre of a structured grid.
 *   modes, grid, epi  host structs (modes->z / phi point to device memory).
 *   method            GRF_DIRECT_F32 | GRF_DIRECT_F64 | GRF_SEP_* | GRF_AUTO.
 *   y, k              device float[C] or NULL; ind device uint8[C] or NULL (C = cells).
 *                     At least one output must be non-NULL.  epi may be NULL when
 *                     k and ind are NULL.
 *   ws, ws_bytes      device workspace of eval_field_grid_ws_size bytes: the per-axis
 *                     tables; for DIRECT_F64 on grids too small to fill the device (under
 *                     131,072 cells) the FP64 partial sums of its mode slices; for the
 *                     separable methods on grids of fewer default tiles than the device
 *                     has CUs, the FP32 sums of the mode slices that the contraction is split
 *                     into (at most 32 MiB; the slices are added in order by a second pass
 *                     that applies the epilogue).  A workspace smaller than that but large
 *                     enough for the tables runs the contraction unsplit (the same field up
 *                     to FP32 summation order); below that GRF_ENOMEM.  Contents on entry
 *                     are ignored.
 * Separable methods require dim 3 grids with nx, ny >= 1 (any size; ragged tiles
 * are masked) or dim 2 grids.  Phases are range-reduced per axis in FP64.
 */
int eval_field_grid(const grf_modes* modes, const grf_grid* grid, int method, const grf_epi* epi,
                    float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes, void* stream);

/*
 * eval_field_grid_noalloc -- eval_field_grid for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace (per-axis tables, partial sums) goes to a fixed scratch array of
 * GRF_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on until the
 * process ends, instead of a caller workspace.
 *   Arguments as eval_field_grid without ws / ws_bytes; outputs are still the caller's.
 *   A problem whose tables exceed the scratch size is GRF_ENOMEM, with nothing enqueued;
 *   the separable mode split is taken when its sums fit as well.  Allocates nothing (no hipMalloc, hipFree or
 *   allocating library call); the first call on a device looks up that device's copy.
 * Every call on one device shares that device's array: calls that overlap on one GPU (other
 * streams or threads, before the previous call's kernels have finished) race on it.  Calls
 * in order on one stream are safe.  The array's contents on entry are never read.
 */
#define GRF_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int eval_field_grid_noalloc(const grf_modes* modes, const grf_grid* grid, int method, const grf_epi* epi,
                            float* y, float* k, uint8_t* ind, void* stream);

/*
 * eval_field_grid_tile -- eval_field_grid with an explicit tile shape for the separable
 * methods (tuning and tests).  tile = -1 is the size-based default (what eval_field_grid
 * uses); 0 .. grf_sep_tile_count()-1 selects a shape.  Any selector gives the same field up
 * to the rounding of the fp16/bf16 operands' FP32 accumulation order.  A selector >= 0 runs
 * unsplit (no mode split).  A selector >= 0 with a direct method, or one out of range, is
 * GRF_EINVAL.  Other arguments as eval_field_grid.
 */
int eval_field_grid_tile(const grf_modes* modes, const grf_grid* grid, int method, int tile, const grf_epi* epi,
                         float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes, void* stream);

/* Number of separable tile selectors. */
int grf_sep_tile_count(void);

/* Block shape of a separable tile selector for a method (GRF_SEP_*) and dim (2 or 3):
 * rows (y cells) x cols (x cells) per block, and the z-slices one block covers. */
int grf_sep_tile_shape(int tile, int method, int dim, int32_t* rows, int32_t* cols, int32_t* slices);

/* FP64 outputs of the plain method (Sec. 4.1 eq. DiscreteFT), DIRECT_F64 only:
 * y64 / k64 device double[C] or NULL (at least one non-NULL); mu is used for k64. */
int eval_field_grid_f64(const grf_modes* modes, const grf_grid* grid, double mu, double* y64,
                        double* k64, void* ws, size_t ws_bytes, void* stream);

/* Device workspace (bytes) that eval_field_points needs. */
int eval_field_points_ws_size(const grf_modes* modes, int64_t n_points, int method, size_t* bytes);

/*
 * eval_field_points -- the field at P arbitrary points (unstructured cell centres,
 * Sec. 4.1: the direct sum applies to any mesh).
 *   xyz      device double[P][dim] (row-major).
 *   method   GRF_DIRECT_F32: cos and sum in FP32 with FP64 phase reduction, in one of two forms
 *              GRF_DIRECT_F32_BINNED (what GRF_DIRECT_F32 uses from 65,536 points): points are
 *                sorted into cells of the bounding box of their finite coordinates (sides
 *                about equal, a whole number of cells per axis, about 2,048 points per cell,
 *                slots padded to work items of 256), the phase at the cell centre is reduced in
 *                FP64 per mode and work item and each point adds its offset's phase, formed on
 *                the matrix cores with FP32 accuracy; modes whose offset phase can reach 4
 *                revolutions within a cell take the per-point FP64 reduction instead.
 *                At most 2^30 points (GRF_EUNSUPPORTED above).  A point's value depends on the
 *                other points only through the cell geometry, not on their order
 *                (deterministic); a point with a non-finite coordinate gets NaN;
 *              GRF_DIRECT_F32_POINTWISE: phase a.x + psi reduced in FP64 per mode and point;
 *            GRF_DIRECT_F64: FP64 throughout.  Separable methods -> GRF_EUNSUPPORTED.
 *   y, k, ind, epi, ws: as eval_field_grid (outputs in input order).  P = 0 is a no-op.
 */
int eval_field_points(const grf_modes* modes, const double* xyz, int64_t n_points, int method,
                      const grf_epi* epi, float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes,
                      void* stream);

/*
 * epilogue_apply -- stand-alone epilogue over an existing field (memory-bound form):
 * k[c] = exp(epi->mu + y[c]) if k != NULL; ind[c] = #{i : t_i < y[c]} if ind != NULL.
 * y, k: device float[n]; ind: device uint8[n].  n = 0 is a no-op.
 */
int epilogue_apply(const float* y, int64_t n, const grf_epi* epi, float* k, uint8_t* ind,
                   void* stream);

/*
 * Bitruncated (pluri-Gaussian) truncation rule, Sec. 3.1 and App. B ("bitruncated",
 * "thresholds", "thresholds2", "values"): two independent fields Y1, Y2 are thresholded
 * separately, cell c lies in bin (i, j) with i = #{a : t_a < Y1_c} and j = #{b : s_b < Y2_c}
 * (strict: Y == t falls in the lower bin), and the rule merges the (n_t + 1) x (n_s + 1)
 * bins into facies: facies_c = rule[i * (n_s + 1) + j]; value_c = values[facies_c].
 * With n_s = 0 and rule[i] = i this is the single truncation of grf_epi.
 */
typedef struct grf_trunc2 {
    int32_t n_t;                        /* thresholds on Y1, ascending, 0 .. GRF_MAX_THRESHOLDS */
    float t[GRF_MAX_THRESHOLDS];
    int32_t n_s;                        /* thresholds on Y2, ascending, 0 .. GRF_MAX_THRESHOLDS */
    float s[GRF_MAX_THRESHOLDS];
    uint8_t rule[(GRF_MAX_THRESHOLDS + 1) * (GRF_MAX_THRESHOLDS + 1)]; /* first (n_t+1)(n_s+1) used */
    int32_t n_values;                   /* 0 .. GRF_MAX_FACIES; every used rule entry must be
                                           < n_values when a value output is requested */
    float values[GRF_MAX_FACIES];
} grf_trunc2;

/* Workspace of eval_pluri_grid when the caller keeps neither field (y1 == y2 == NULL): both
 * fields' tables (and, where eval_field_grid would split the modes, both fields' slice sums),
 * the rule tables and the fields.  Each field buffer the caller passes makes the need C * 4
 * bytes (rounded up to 256) smaller. */
int eval_pluri_grid_ws_size(const grf_modes* m1, const grf_modes* m2, const grf_grid* grid, int method,
                            size_t* bytes);

/*
 * eval_pluri_grid -- a pluri-Gaussian facies field on a structured grid: Y1 from m1 and Y2
 * from m2 by `method` (as eval_field_grid), then the bitruncated rule over the two stored
 * fields.  m1 and m2 must have the same dim (independent tables: different seeds).
 *   facies  device uint8[C] or NULL;  value device float[C] or NULL (one of them required).
 *   y1, y2  device float[C] or NULL: keep the fields; a field not kept lives in the workspace.
 * The facies are decided in FP32 on each path's Y; they match the FP64 definition except
 * in cells whose Y1 or Y2 lies within that path's error of a threshold.
 */
int eval_pluri_grid(const grf_modes* m1, const grf_modes* m2, const grf_grid* grid, int method,
                    const grf_trunc2* rule, uint8_t* facies, float* value, float* y1, float* y2, void* ws,
                    size_t ws_bytes, void* stream);

/* The same at P arbitrary points (xyz device double[P][dim]); the workspace size is for
 * y1 == y2 == NULL. */
int eval_pluri_points_ws_size(const grf_modes* m1, const grf_modes* m2, int64_t n_points, int method,
                              size_t* bytes);
int eval_pluri_points(const grf_modes* m1, const grf_modes* m2, const double* xyz, int64_t n_points, int method,
                      const grf_trunc2* rule, uint8_t* facies, float* value, float* y1, float* y2, void* ws,
                      size_t ws_bytes, void* stream);

/* Stand-alone bitruncated rule over two existing fields y1, y2 (device float[n]);
 * facies device uint8[n] / value device float[n], either may be NULL (not both);
 * ws: device workspace of at least GRF_PLURI_APPLY_WS_BYTES bytes (the rule's tables). */
#define GRF_PLURI_APPLY_WS_BYTES 512
int pluri_apply(const float* y1, const float* y2, int64_t n, const grf_trunc2* rule, uint8_t* facies,
                float* value, void* ws, size_t ws_bytes, void* stream);

/*
 * Gradients of a scalar loss L through Y at P points, given g = dL/dY (field_backward).
 * With theta_jp = k_j . x_p + phi_j and A = sigma sqrt(2/N) (chain rule through
 * Sec. 4.1 eq. DiscreteFT, k = z / ell):
 *   grad_phi[j]      = -A sum_p g_p sin theta_jp
 *   grad_k[a*n + j]  = -A sum_p g_p x_{p,a} sin theta_jp
 *   grad_sigma[0]    = sum_p g_p Y_p / sigma        (Y recomputed unless y_saved given)
 *   grad_ell[a]      = -(1/ell_a) sum_j k_{j,a} grad_k[a*n + j]
 *   xyz     device double[P][dim];  grad_y device float[P];  y_saved device float[P] or NULL.
 *   outputs device float arrays (any may be NULL); overwritten, not accumulated.
 *   ws      device workspace of field_backward_ws_size bytes.
 * Sines are recomputed (no stored cosines); sums over points are reduced in a fixed
 * order (deterministic).  P = 0 writes zeros.
 */
int field_backward_ws_size(const grf_modes* modes, int64_t n_points, size_t* bytes);
int field_backward(const grf_modes* modes, const double* xyz, int64_t n_points, const float* grad_y,
                   const float* y_saved, float* grad_phi, float* grad_k, float* grad_sigma,
                   float* grad_ell, void* ws, size_t ws_bytes, void* stream);

/*
 * grad_z_from_k -- the chain rule from the wavevector gradient to the standard draws z of the
 * table, k_j = rot diag(1/ell) z_j (Sec. 4.1; rot = identity for axis-aligned tables):
 *   grad_z[b*n + j] = (1/ell_b) sum_a rot[a][b] grad_k[a*n + j]   (FP64 sum, FP32 result).
 *   modes    as for field_backward (dim, n, ell, rot / rotated are read).
 *   grad_k   device float[dim][n] (field_backward's grad_k); grad_z device float[dim][n],
 *            overwritten, not aliasing grad_k (GRF_EINVAL).  n = 0: nothing is enqueued.
 */
int grad_z_from_k(const grf_modes* modes, const float* grad_k, float* grad_z, void* stream);

/* The same gradients for a dense dL/dY over every cell of a structured grid.
 * grad_y device float[C] (x fastest). */
int field_backward_grid_ws_size(const grf_modes* modes, const grf_grid* grid, size_t* bytes);
int field_backward_grid(const grf_modes* modes, const grf_grid* grid, const float* grad_y,
                        const float* y_saved, float* grad_phi, float* grad_k, float* grad_sigma,
                        float* grad_ell, void* ws, size_t ws_bytes, void* stream);

/*
 * field_backward_grid_method -- the same with the method chosen:
 *   GRF_DIRECT_F32   per mode and cell from FP32 revolution tables (one sine per mode-cell);
 *   GRF_SEP_BF16_X3  separable form: the per-mode sums factor over the axes like the forward
 *                    sum (eq. DiscreteFT with k.x split per axis), S_j = sum_{y,z}
 *                    [sum_x g Ex] Ey Ez, the bracket a bf16 hi+lo matrix product (relative
 *                    error ~2^-16) reduced with Ey Ez in FP32; x runs in chunks of 128
 *                    cells, one after another;
 *   GRF_AUTO         the separable form (what field_backward_grid does).
 * The workspace of field_backward_grid_ws_size fits every method.
 */
int field_backward_grid_method(const grf_modes* modes, const grf_grid* grid, int method, const float* grad_y,
                               const float* y_saved, float* grad_phi, float* grad_k, float* grad_sigma,
                               float* grad_ell, void* ws, size_t ws_bytes, void* stream);

/*
 * Conditioning on observations by kriging the residuals (the paper lists conditioning on
 * data as future work, Sec. 6): with observations d_i at x_i (i < M) and a realisation Y,
 *   alpha = (C(X, X) + nugget sigma^2 I)^-1 (d - Y(X)),   Y_c(x) = Y(x) + sum_i alpha_i C(x - x_i),
 * where C(dx) = sigma^2 rho(|M^T dx|) is the model covariance of the table's field
 * (M = diag(1/ell), or rot diag(1/ell) for rotated tables; rho of App. A).  Y_c honours the
 * data (exactly for nugget 0, up to the forward path's error) and, over realisations, has the
 * simple-kriging conditional covariance.
 */
typedef struct grf_krige {
    int32_t cov;     /* GRF_COV_GAUSSIAN, GRF_COV_EXPONENTIAL, or GRF_COV_MATERN with nu 1/2, 3/2, 5/2 */
    int32_t pad_;
    double nu;       /* Matern smoothness (ignored otherwise) */
    double nugget;   /* >= 0: nugget * sigma^2 is added to the diagonal of C(X, X) */
} grf_krige;

/* Workspace of krige_weights: the FP64 M x M matrix, the inverses of its 64 x 64 diagonal
 * factors, two FP64 vectors of the substitutions, and the point evaluation of Y. */
int krige_weights_ws_size(const grf_modes* modes, int64_t n_obs, size_t* bytes);

/*
 * krige_weights -- alpha for M observations (M >= 1, at most 1,048,560).
 *   xobs   device double[M][dim];  dobs device float[M] (observed values of Y, i.e. ln K - mu).
 *   alpha  device double[M], written.
 *   info   device int32 or NULL: 0, or the 1-based index of the first non-positive pivot of
 *          the Cholesky factorisation (C(X, X) + nugget not positive definite: alpha is NaN).
 * Y(X) is evaluated by the FP32 direct point sum of `modes`; the system is factorised in FP64.
 */
int krige_weights(const grf_modes* modes, const grf_krige* kp, const double* xobs, const float* dobs, int64_t n_obs,
                  double* alpha, int32_t* info, void* ws, size_t ws_bytes, void* stream);

/* Workspace of krige_apply_grid / krige_apply_points: 16 bytes per observation. */
int krige_apply_ws_size(int64_t n_obs, size_t* bytes);

/*
 * krige_apply_grid / krige_apply_points -- y += sum_i alpha_i C(x - x_i) at every cell centre
 * of `grid` (y device float[C], x fastest) or at points xyz (device double[P][dim], y float[P]).
 * Run after eval_field_grid / eval_field_points of the same table for Y_c.  Lags are formed in
 * FP64 from the first observation and summed in FP32.
 */
int krige_apply_grid(const grf_modes* modes, const grf_krige* kp, const double* xobs, const double* alpha,
                     int64_t n_obs, const grf_grid* grid, float* y, void* ws, size_t ws_bytes, void* stream);
int krige_apply_points(const grf_modes* modes, const grf_krige* kp, const double* xobs, const double* alpha,
                       int64_t n_obs, const double* xyz, int64_t n_points, float* y, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * Batched ensembles of independent realisations on grids of uneven size, evaluated
 * in one persistent launch (plus the per-axis table build) captured in a hipGraph.
 */
typedef struct grf_batch_item {
    grf_modes modes; /* per-instance mode table (device) and scalars */
    grf_grid grid;   /* dim 2 or 3 grid */
    grf_epi epi;     /* per-instance epilogue (Sec. 4.1 scaling, Sec. 3.1 truncation rule):
                        read for k (mu) and ind (thresholds, at least one when ind != NULL) */
    float* y;        /* device float[cells of this grid] or NULL */
    float* k;        /* device float[cells]: K = exp(mu + Y), or NULL */
    uint8_t* ind;    /* device uint8[cells]: facies index #{i : t_i < Y}, or NULL */
} grf_batch_item;   /* at least one of y, k, ind per item */

typedef struct grf_plan grf_plan;

/* Plan flags */
#define GRF_PLAN_GRAPH 1    /* capture the launch sequence in a hipGraph and replay it */
#define GRF_PLAN_AUTOTUNE 2 /* time candidate tile shapes on first use (cached per size class) */

/*
 * grf_plan_create -- a plan owns device memory for the batch's tables and descriptors,
 * the autotuned tile choices and the captured graph, keyed by the batch signature.
 *   method  GRF_DIRECT_F32 or a GRF_SEP_* method (GRF_AUTO -> GRF_SEP_F16).
 *   flags   GRF_PLAN_* bits.
 *   tune_cache_path  host string or NULL: a text file where tuned tile choices are read
 *                    from and appended to.
 */
int grf_plan_create(grf_plan** plan, int method, int flags, const char* tune_cache_path);
int grf_plan_destroy(grf_plan* plan);

/*
 * eval_field_batch -- evaluate n items.  items is a host array; each item's outputs
 * receive what eval_field_grid(method, &item.epi, y, k, ind) would write (bitwise for the
 * direct method and the hi+lo forms with the same tile shape; the 2-D one-pass forms
 * generate their operands on chip and agree within the method's rounding).  The first call
 * with a new batch signature (sizes, scalars, table, weight and output pointers, epilogue,
 * method) builds descriptors, tunes if asked and captures the graph; later calls with the
 * same signature replay it, reading the tables' current contents.  Calls on one plan must
 * not overlap (they share the plan's device memory).
 */
int eval_field_batch(grf_plan* plan, const grf_batch_item* items, int32_t n, void* stream);

/* Statistics of the last eval_field_batch call on this plan (for benchmarks):
 * tile_m/tile_n chosen for the separable path (0 for direct), replayed = 1 if the graph
 * was replayed, work_items = tiles in the persistent queue. */
int grf_plan_info(const grf_plan* plan, int32_t* tile_m, int32_t* tile_n, int32_t* replayed,
                  int64_t* work_items);

/*
 * Kernel timer (instrumentation for benchmarks).  While enabled, every call records a
 * pair of HIP events on its stream around its main kernel: the sum kernel of
 * eval_field_grid / eval_field_points, the epilogue kernel of epilogue_apply, the main
 * adjoint kernel of field_backward(_grid) and the persistent kernel of eval_field_batch.
 * The separable contraction of eval_field_grid (and of eval_pluri_grid) carries the pair on
 * its own dispatch (hipExtLaunchKernel start/stop events), so it measures that kernel alone.
 *   grf_kernel_timer_enable(1) clears the record and starts recording; (0) stops.
 *   grf_kernel_timer_read waits for the recorded events and returns the summed kernel
 *   time (ms) and the number of timed launches.  Events are created on first use and
 *   reused; recording is process-wide and guarded by a mutex.
 */
int grf_kernel_timer_enable(int enable);
int grf_kernel_timer_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GRF_H */
