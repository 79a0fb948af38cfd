/*
 * grf_oracle.c -- plain FP64 CPU reference for the spectral Gaussian-random-field
 * path (Icardi, Pescimoro, Municchi, Hidalgo 2022, "Computational framework for
 * complex flow and transport in heterogeneous porous media", Sec. 4.1 and App. A/B).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * Everything here is the plain definition, written out in double precision:
 *
 *   Y(x) = sqrt(2 sigma^2 / N) * sum_{j<N} cos(k_j . x + phi_j),   k_{j,a} = z_{j,a} / ell_a
 *
 * (the random-phase form of the discrete spectral sum, Sec. 4.1 eq. DiscreteFT;
 * frequencies rescaled per axis for anisotropy, Sec. 4.1), with z_j drawn from the
 * normalised spectral density of the covariance (App. A, eqs. gauSpe, expSpe, matSpe)
 * and phi_j uniform on [0, 2 pi).  The sum over modes is sequential in j; no
 * blocking, no range reduction beyond what libm's cos does, no fusion.
 *
 * Readings of the paper taken here (each listed in the design notes):
 *  - exactly N modes, amplitude sqrt(2 sigma^2/N) (the paper's j=0..N_f sum has no
 *    stated normalisation);
 *  - angular wavevectors, C(r) = int S(k) e^{i k.r} dk (the App. A pairs are
 *    consistent only under that convention);
 *  - Gaussian correlation exp(-r^2/ell^2); the paper's lambda maps to
 *    ell = 2 lambda / sqrt(pi) (App. A, eq. gauSpe);
 *  - exponential correlation exp(-r/ell) (App. A, eq. expSpe);
 *  - Matern with 2 nu a positive integer (App. A, eq. matSpe), sampled as a
 *    multivariate Student t with 2 nu degrees of freedom;
 *  - grid cell centres origin + (i + 1/2) h, x index fastest.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), key = seed, counter = (mode index lo,
 * mode index hi, draw slot, 0).  Each call yields two 64-bit words
 * (w0 = out1:out0, w1 = out3:out2).  Slot 0 gives the phase, slots 1-2 the d
 * spatial normals, slots 3.. the mixing normals (exponential / Matern radial part).
 * Uniforms on (0,1): ((w >> 11) + 1/2) * 2^-53.  Normals: Box-Muller.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops below will use (1 without OpenMP). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of the OpenMP loops below (timing of the oracle at a given core count). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ RNG */

static uint32_t orc_mulhi32(uint32_t a, uint32_t b, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *lo = (uint32_t)p;
    return (uint32_t)(p >> 32);
}

/* One Philox4x32 block: 10 rounds of the S-box/P-box network of Salmon et al.,
 * multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t lo0, lo1;
        uint32_t hi0 = orc_mulhi32(0xD2511F53u, c0, &lo0);
        uint32_t hi1 = orc_mulhi32(0xCD9E8D57u, c2, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The two 64-bit words of draw slot `slot` of mode `j` under `seed`. */
void orc_words(uint64_t seed, int64_t j, uint32_t slot, uint64_t w[2])
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)j & 0xffffffffu), (uint32_t)((uint64_t)j >> 32), slot, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    w[0] = ((uint64_t)o[1] << 32) | o[0];
    w[1] = ((uint64_t)o[3] << 32) | o[2];
}

static double orc_unit(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* Two standard normals from one draw slot (Box-Muller). */
static void orc_normal_pair(uint64_t seed, int64_t j, uint32_t slot, double g[2])
{
    uint64_t w[2];
    orc_words(seed, j, slot, w);
    double u1 = orc_unit(w[0]);
    double u2 = orc_unit(w[1]);
    double r = sqrt(-2.0 * log(u1));
    g[0] = r * cos(2.0 * ORC_PI * u2);
    g[1] = r * sin(2.0 * ORC_PI * u2);
}

/*
 * Draw N modes for covariance `cov` (0 Gaussian, 1 exponential, 2 Matern) in
 * `dim` dimensions.  z is [dim][n] (axis-major), phi is [n].
 *   Gaussian  (eq. gauSpe, ell convention):  z = sqrt(2) g            (density of k=z/ell is exp(-|k ell|^2/4))
 *   Exponential (eq. expSpe):               z = g / |h0|             (multivariate Cauchy)
 *   Matern, 2nu = m integer (eq. matSpe):   z = g * sqrt(m / sum_{i<m} h_i^2)  (multivariate t, m dof)
 * Returns 0, or -1 on bad arguments.
 */
int orc_sample_modes(int dim, int cov, double nu, int64_t n, uint64_t seed, double* z, double* phi)
{
    if (dim < 1 || dim > 3 || n < 1 || !z || !phi) return -1;
    int m = 0;
    if (cov == 2) {
        double twonu = 2.0 * nu;
        m = (int)llround(twonu);
        if (m < 1 || fabs(twonu - m) > 1e-12 || m > 64) return -1;
    } else if (cov != 0 && cov != 1) {
        return -1;
    }
    for (int64_t j = 0; j < n; ++j) {
        uint64_t w[2];
        orc_words(seed, j, 0u, w);
        phi[j] = 2.0 * ORC_PI * orc_unit(w[0]);

        double g[4];
        orc_normal_pair(seed, j, 1u, g);
        orc_normal_pair(seed, j, 2u, g + 2);

        double scale;
        if (cov == 0) {
            scale = sqrt(2.0);
        } else if (cov == 1) {
            double h[2];
            orc_normal_pair(seed, j, 3u, h);
            scale = 1.0 / fabs(h[0]);
        } else {
            double chi2 = 0.0;
            for (int i = 0; i < m; i += 2) {
                double h[2];
                orc_normal_pair(seed, j, 3u + (uint32_t)(i / 2), h);
                chi2 += h[0] * h[0];
                if (i + 1 < m) chi2 += h[1] * h[1];
            }
            scale = sqrt((double)m / chi2);
        }
        for (int a = 0; a < dim; ++a) z[(int64_t)a * n + j] = g[a] * scale;
    }
    return 0;
}

/* ------------------------------------------------------------------ field */

/* Y at P points x[P][dim] (row-major), from modes z[dim][n], phi[n]. */
void orc_field_points(int dim, int64_t n, const double* z, const double* phi, double sigma,
                      const double* ell, int64_t P, const double* x, double* y)
{
    double amp = sigma * sqrt(2.0 / (double)n);
    double* k = (double*)malloc(sizeof(double) * (size_t)(dim * n));
    for (int a = 0; a < dim; ++a)
        for (int64_t j = 0; j < n; ++j) k[a * n + j] = z[a * n + j] / ell[a];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        const double* xp = x + p * dim;
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double th = phi[j];
            for (int a = 0; a < dim; ++a) th += k[a * n + j] * xp[a];
            s += cos(th);
        }
        y[p] = amp * s;
    }
    free(k);
}

/* Centre of grid cell with linear index c (x fastest): x_a = o_a + (i_a + 1/2) h_a. */
static void orc_cell_centre(int dim, const int64_t* gn, const double* o, const double* h, int64_t c,
                            double* xc)
{
    int64_t rem = c;
    for (int a = 0; a < dim; ++a) {
        int64_t i = rem % gn[a];
        rem /= gn[a];
        xc[a] = o[a] + ((double)i + 0.5) * h[a];
    }
}

/* Y at a list of grid cells (linear indices), for sampled checks at full size. */
void orc_field_cells(int dim, int64_t n, const double* z, const double* phi, double sigma,
                     const double* ell, const int64_t* gn, const double* o, const double* h,
                     int64_t ncells, const int64_t* cells, double* y)
{
    double* x = (double*)malloc(sizeof(double) * (size_t)(ncells * dim));
    for (int64_t q = 0; q < ncells; ++q) orc_cell_centre(dim, gn, o, h, cells[q], x + q * dim);
    orc_field_points(dim, n, z, phi, sigma, ell, ncells, x, y);
    free(x);
}

/* Y on the whole grid gn[0] x ... x gn[dim-1], x index fastest. */
void orc_field_grid(int dim, int64_t n, const double* z, const double* phi, double sigma,
                    const double* ell, const int64_t* gn, const double* o, const double* h, double* y)
{
    int64_t C = 1;
    for (int a = 0; a < dim; ++a) C *= gn[a];
    double* x = (double*)malloc(sizeof(double) * (size_t)(C * dim));
    for (int64_t c = 0; c < C; ++c) orc_cell_centre(dim, gn, o, h, c, x + c * dim);
    orc_field_points(dim, n, z, phi, sigma, ell, C, x, y);
    free(x);
}

/*
 * The same field through the product-of-exponentials identity
 *   Y = amp * Re sum_j e^{i phi_j} prod_a e^{i k_{j,a} x_a},
 * evaluated per cell in double complex arithmetic written out as (re, im) pairs.
 * Validation of the algebra the separable (matrix-core) form rests on.
 */
void orc_field_grid_separable(int dim, int64_t n, const double* z, const double* phi, double sigma,
                              const double* ell, const int64_t* gn, const double* o, const double* h,
                              double* y)
{
    double amp = sigma * sqrt(2.0 / (double)n);
    int64_t C = 1;
    for (int a = 0; a < dim; ++a) C *= gn[a];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < C; ++c) {
        double xc[3];
        orc_cell_centre(dim, gn, o, h, c, xc);
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double re = cos(phi[j]), im = sin(phi[j]);
            for (int a = 0; a < dim; ++a) {
                double t = z[a * n + j] / ell[a] * xc[a];
                double er = cos(t), ei = sin(t);
                double nr = re * er - im * ei;
                double ni = re * ei + im * er;
                re = nr;
                im = ni;
            }
            s += re;
        }
        y[c] = amp * s;
    }
}

/* ------------------------------------------------------------------ epilogues */

/* Log-normal permeability K = exp(mu + Y) (Sec. 4.1: the field scaled to mean mu). */
void orc_lognormal(int64_t C, const double* y, double mu, double* k)
{
    for (int64_t c = 0; c < C; ++c) k[c] = exp(mu + y[c]);
}

/* Truncation rule (Sec. 3.1): facies index = number of thresholds strictly below Y.
 * With one threshold t this is the indicator [Y > t]. */
void orc_facies(int64_t C, const double* y, int nthr, const double* thr, uint8_t* out)
{
    for (int64_t c = 0; c < C; ++c) {
        int f = 0;
        for (int i = 0; i < nthr; ++i)
            if (y[c] > thr[i]) ++f;
        out[c] = (uint8_t)f;
    }
}

/* ------------------------------------------------------------------ gradients */

/*
 * Gradients of a scalar loss L through Y at P points, given g[p] = dL/dY_p.
 * With theta_jp = k_j . x_p + phi_j and amp = sigma sqrt(2/N):
 *   dL/dphi_j   = -amp sum_p g_p sin theta_jp
 *   dL/dk_{a,j} = -amp sum_p g_p x_{p,a} sin theta_jp
 *   dL/dsigma   = sum_p g_p Y_p / sigma
 *   dL/dell_a   = sum_j dL/dk_{a,j} * (-z_{a,j} / ell_a^2)       (k = z / ell, z fixed)
 * dk is [dim][n]; dell is [dim].  Sums over p run in order, per mode.
 */
void orc_grad_points(int dim, int64_t n, const double* z, const double* phi, double sigma,
                     const double* ell, int64_t P, const double* x, const double* g,
                     double* dphi, double* dk, double* dsigma, double* dell)
{
    double amp = sigma * sqrt(2.0 / (double)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    orc_field_points(dim, n, z, phi, sigma, ell, P, x, y);
    double ds = 0.0;
    for (int64_t p = 0; p < P; ++p) ds += g[p] * y[p];
    *dsigma = ds / sigma;
    free(y);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0, u[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < P; ++p) {
            const double* xp = x + p * dim;
            double th = phi[j];
            for (int a = 0; a < dim; ++a) th += z[a * n + j] / ell[a] * xp[a];
            double sn = sin(th);
            s += g[p] * sn;
            for (int a = 0; a < dim; ++a) u[a] += g[p] * xp[a] * sn;
        }
        dphi[j] = -amp * s;
        for (int a = 0; a < dim; ++a) dk[a * n + j] = -amp * u[a];
    }
    for (int a = 0; a < dim; ++a) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc += dk[a * n + j] * (-z[a * n + j] / (ell[a] * ell[a]));
        dell[a] = acc;
    }
}

/* ------------------------------------------------------------------ pluri-Gaussian (bitruncated) */

/*
 * Bitruncated rule (Sec. 3.1, truncation-rule figure): two independent fields Y1, Y2
 * are thresholded separately; cell c lies in bin (i, j) with i = #{a : t_a < Y1_c} and
 * j = #{b : s_b < Y2_c} (strict inequalities, so Y == t falls in the lower bin), and the
 * rule maps the (nt + 1) x (ns + 1) bins to facies: facies_c = rule[i * (ns + 1) + j].
 * With ns = 0 this is the single truncation of orc_facies composed with rule[i].
 * When values != NULL, val_c = values[facies_c] (the "values" option of App. B).
 */
void orc_pluri(int64_t C, const double* y1, const double* y2, int nt, const double* t, int ns,
               const double* s, const uint8_t* rule, const double* values, uint8_t* out, double* val)
{
    for (int64_t c = 0; c < C; ++c) {
        int i = 0, j = 0;
        for (int a = 0; a < nt; ++a)
            if (y1[c] > t[a]) ++i;
        for (int b = 0; b < ns; ++b)
            if (y2[c] > s[b]) ++j;
        const uint8_t f = rule[i * (ns + 1) + j];
        out[c] = f;
        if (values && val) val[c] = values[f];
    }
}

/* Normal CDF of N(0, v) at x; +-infinity are handled by erfc. */
static double orc_normal_cdf(double x, double v) { return 0.5 * erfc(-x / sqrt(2.0 * v)); }

/*
 * Proportion of each facies when Y1 ~ N(0, v1) and Y2 ~ N(0, v2) are independent
 * (Sec. 3.1): bin (i, j) has probability [G1(t_i) - G1(t_{i-1})] [G2(s_j) - G2(s_{j-1})]
 * with t_{-1} = -inf and t_nt = +inf (likewise s); bins of the same facies add up.
 * p[0 .. nfac-1] is overwritten; rule entries must be < nfac.
 */
void orc_pluri_proportions(int nt, const double* t, double v1, int ns, const double* s, double v2,
                           const uint8_t* rule, int nfac, double* p)
{
    for (int f = 0; f < nfac; ++f) p[f] = 0.0;
    for (int i = 0; i <= nt; ++i) {
        const double lo1 = i == 0 ? -INFINITY : t[i - 1], hi1 = i == nt ? INFINITY : t[i];
        const double p1 = orc_normal_cdf(hi1, v1) - orc_normal_cdf(lo1, v1);
        for (int j = 0; j <= ns; ++j) {
            const double lo2 = j == 0 ? -INFINITY : s[j - 1], hi2 = j == ns ? INFINITY : s[j];
            const double p2 = orc_normal_cdf(hi2, v2) - orc_normal_cdf(lo2, v2);
            p[rule[i * (ns + 1) + j]] += p1 * p2;
        }
    }
}

/* ------------------------------------------------------------------ general anisotropy */

/*
 * The field with a general linear map of frequency space (Sec. 4.1: the per-axis rescaling
 * "can be extended by including rotations, or more general transformation matrices"):
 *   k_j = M z_j  (M is dim x dim, row-major; M = R diag(1/ell) rotates the principal
 *   axes of the covariance onto the columns of R),
 *   Y(x) = sqrt(2 sigma^2/N) sum_j cos(k_j . x + phi_j).
 * With M = diag(1/ell) this is orc_field_points.
 */
void orc_field_points_mat(int dim, int64_t n, const double* z, const double* phi, double sigma,
                          const double* M, int64_t P, const double* x, double* y)
{
    double amp = sigma * sqrt(2.0 / (double)n);
    double* k = (double*)malloc(sizeof(double) * (size_t)(dim * n));
    for (int a = 0; a < dim; ++a)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int b = 0; b < dim; ++b) v += M[a * dim + b] * z[b * n + j];
            k[a * n + j] = v;
        }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        const double* xp = x + p * dim;
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double th = phi[j];
            for (int a = 0; a < dim; ++a) th += k[a * n + j] * xp[a];
            s += cos(th);
        }
        y[p] = amp * s;
    }
    free(k);
}

/*
 * Periodic option (App. B "periodic"): each wavevector is moved to the nearest point of
 * the lattice of a box with periods L_a, k_a = 2 pi m_a / L_a with m_a = round(k_a L_a / 2 pi),
 * for every axis with L_a > 0 (axes with L_a <= 0 are left alone).  k = R diag(1/ell) z
 * before snapping (R = identity when rot == NULL, row-major dim x dim, orthonormal), and the
 * snapped table is returned in the same standardised form: z' = diag(ell) R^T k'.
 * The field then satisfies Y(x + L_a e_a) = Y(x).
 */
void orc_snap_periodic(int dim, int64_t n, const double* z, const double* ell, const double* rot,
                       const double* period, double* z_out)
{
    for (int64_t j = 0; j < n; ++j) {
        double zs[3], k[3];
        for (int b = 0; b < dim; ++b) zs[b] = z[b * n + j] / ell[b];
        for (int a = 0; a < dim; ++a) {
            double v = 0.0;
            for (int b = 0; b < dim; ++b) v += (rot ? rot[a * dim + b] : (a == b ? 1.0 : 0.0)) * zs[b];
            if (period[a] > 0.0) v = 2.0 * ORC_PI * round(v * period[a] / (2.0 * ORC_PI)) / period[a];
            k[a] = v;
        }
        for (int b = 0; b < dim; ++b) {
            double v = 0.0;
            for (int a = 0; a < dim; ++a) v += (rot ? rot[a * dim + b] : (a == b ? 1.0 : 0.0)) * k[a];
            z_out[b * n + j] = v * ell[b];
        }
    }
}

/*
 * Gradients through the rotated field k_j = R diag(1/ell) z_j (R row-major, orthonormal,
 * dim x dim), given g[p] = dL/dY_p at points x:
 *   dL/dphi_j, dL/dk_{a,j}, dL/dsigma as in orc_grad_points (k is the wavevector itself);
 *   dL/dell_b = sum_j sum_a dL/dk_{a,j} R_ab (-z_{b,j} / ell_b^2)   (z and R fixed).
 */
void orc_grad_points_rot(int dim, int64_t n, const double* z, const double* phi, double sigma,
                         const double* ell, const double* rot, int64_t P, const double* x, const double* g,
                         double* dphi, double* dk, double* dsigma, double* dell)
{
    double M[9];
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) M[a * dim + b] = rot[a * dim + b] / ell[b];
    double amp = sigma * sqrt(2.0 / (double)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    orc_field_points_mat(dim, n, z, phi, sigma, M, P, x, y);
    double ds = 0.0;
    for (int64_t p = 0; p < P; ++p) ds += g[p] * y[p];
    *dsigma = ds / sigma;
    free(y);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        double k[3];
        for (int a = 0; a < dim; ++a) {
            k[a] = 0.0;
            for (int b = 0; b < dim; ++b) k[a] += M[a * dim + b] * z[b * n + j];
        }
        double s = 0.0, u[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < P; ++p) {
            const double* xp = x + p * dim;
            double th = phi[j];
            for (int a = 0; a < dim; ++a) th += k[a] * xp[a];
            double sn = sin(th);
            s += g[p] * sn;
            for (int a = 0; a < dim; ++a) u[a] += g[p] * xp[a] * sn;
        }
        dphi[j] = -amp * s;
        for (int a = 0; a < dim; ++a) dk[a * n + j] = -amp * u[a];
    }
    for (int b = 0; b < dim; ++b) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int a = 0; a < dim; ++a)
                acc += dk[a * n + j] * rot[a * dim + b] * (-z[b * n + j] / (ell[b] * ell[b]));
        dell[b] = acc;
    }
}

/* ------------------------------------------------------------------ fixed-frequency estimator */

/* Standardised spectral shape (ell = 1, angular frequency) of the covariance, up to a
 * constant (App. A): Gaussian exp(-|u|^2/4), exponential (1 + |u|^2)^(-(d+1)/2), Matern
 * (1 + |u|^2 / (2 nu))^(-(2 nu + d)/2). */
static double orc_spectral_shape(int dim, int cov, double nu, const double* u)
{
    double r2 = 0.0;
    for (int a = 0; a < dim; ++a) r2 += u[a] * u[a];
    if (cov == 0) return exp(-r2 / 4.0);
    if (cov == 1) return pow(1.0 + r2, -0.5 * (dim + 1));
    return pow(1.0 + r2 / (2.0 * nu), -0.5 * (2.0 * nu + dim));
}

/*
 * The discrete spectral sum of Sec. 4.1 eq. DiscreteFT with fixed frequencies and Gaussian
 * weights, in its real reading
 *   Y(x) = sum_j c_j [W_j cos(k_j . x) + W'_j sin(k_j . x)],  c_j = sigma sqrt(p_j),
 *   p_j = S(u_j) / sum_i S(u_i),  k_j = u_j / ell,  W, W' independent N(0, 1),
 * over the half-space lattice u_j of m^dim / 2 points (m even, spacing du): mode
 * j = i0 + (m/2) (i1 + m i2) has u_0 = du (i0 + 1/2), u_a = du (i_a - m/2 + 1/2) for a > 0.
 * (W_j, W'_j) is the Box-Muller pair of draw slot 1 of counter j.  Written in the
 * random-phase form sigma sqrt(2/N) sum_j w_j cos(k_j . x + phi_j):
 *   w_j = sqrt(p_j (W_j^2 + W'_j^2) N / 2),  phi_j = -atan2(W'_j, W_j) mod 2 pi.
 * Outputs z [dim][N] (= u), phi [N], w [N]; W, Wp [N] when not NULL.  Returns N, or -1.
 */
int64_t orc_lattice_modes(int dim, int cov, double nu, int m, double du, uint64_t seed, double* z, double* phi,
                          double* w, double* W, double* Wp)
{
    if ((dim != 2 && dim != 3) || m < 2 || (m % 2) != 0 || !(du > 0.0) || cov < 0 || cov > 2) return -1;
    int64_t n = (int64_t)(m / 2) * m;
    if (dim == 3) n *= m;
    double* S = (double*)malloc(sizeof(double) * (size_t)n);
    double tot = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t r = j;
        int64_t i0 = r % (m / 2);
        r /= (m / 2);
        int64_t i1 = r % m;
        int64_t i2 = r / m;
        double u[3] = {du * ((double)i0 + 0.5), du * ((double)i1 - m / 2 + 0.5), du * ((double)i2 - m / 2 + 0.5)};
        for (int a = 0; a < dim; ++a) z[a * n + j] = u[a];
        S[j] = orc_spectral_shape(dim, cov, nu, u);
        tot += S[j];
    }
    for (int64_t j = 0; j < n; ++j) {
        double g[2];
        orc_normal_pair(seed, j, 1u, g);
        double a = -atan2(g[1], g[0]);
        if (a < 0.0) a += 2.0 * ORC_PI;
        phi[j] = a;
        w[j] = sqrt(S[j] / tot * (g[0] * g[0] + g[1] * g[1]) * (double)n / 2.0);
        if (W) W[j] = g[0];
        if (Wp) Wp[j] = g[1];
    }
    free(S);
    return n;
}

/* Weighted random-phase sum Y(x) = sigma sqrt(2/N) sum_j w_j cos(k_j . x + phi_j), k = z / ell. */
void orc_field_points_w(int dim, int64_t n, const double* z, const double* phi, const double* w, double sigma,
                        const double* ell, int64_t P, const double* x, double* y)
{
    double amp = sigma * sqrt(2.0 / (double)n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        const double* xp = x + p * dim;
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double th = phi[j];
            for (int a = 0; a < dim; ++a) th += z[a * n + j] / ell[a] * xp[a];
            s += w[j] * cos(th);
        }
        y[p] = amp * s;
    }
}

/*
 * Gradients through the weighted random-phase sum of orc_field_points_w (the fixed-frequency
 * form of Sec. 4.1 eq. DiscreteFT), given g[p] = dL/dY_p.  With theta_jp = k_j . x_p + phi_j,
 * k = z / ell and amp = sigma sqrt(2/N), the weights w held fixed:
 *   dL/dphi_j   = -amp w_j sum_p g_p sin theta_jp
 *   dL/dk_{a,j} = -amp w_j sum_p g_p x_{p,a} sin theta_jp
 *   dL/dsigma   = sum_p g_p Y_p / sigma                         (Y of the weighted sum)
 *   dL/dell_a   = sum_j dL/dk_{a,j} * (-z_{a,j} / ell_a^2)
 */
void orc_grad_points_w(int dim, int64_t n, const double* z, const double* phi, const double* w, double sigma,
                       const double* ell, int64_t P, const double* x, const double* g,
                       double* dphi, double* dk, double* dsigma, double* dell)
{
    double amp = sigma * sqrt(2.0 / (double)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    orc_field_points_w(dim, n, z, phi, w, sigma, ell, P, x, y);
    double ds = 0.0;
    for (int64_t p = 0; p < P; ++p) ds += g[p] * y[p];
    *dsigma = ds / sigma;
    free(y);

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0, u[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < P; ++p) {
            const double* xp = x + p * dim;
            double th = phi[j];
            for (int a = 0; a < dim; ++a) th += z[a * n + j] / ell[a] * xp[a];
            double sn = sin(th);
            s += g[p] * sn;
            for (int a = 0; a < dim; ++a) u[a] += g[p] * xp[a] * sn;
        }
        dphi[j] = -amp * w[j] * s;
        for (int a = 0; a < dim; ++a) dk[a * n + j] = -amp * w[j] * u[a];
    }
    for (int a = 0; a < dim; ++a) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc += dk[a * n + j] * (-z[a * n + j] / (ell[a] * ell[a]));
        dell[a] = acc;
    }
}
