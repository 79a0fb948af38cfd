// make_modes: host-side spectral sampler for the mode table.
//
// Wavevectors follow the normalised spectral densities of App. A (eqs. gauSpe,
// expSpe, matSpe) with per-axis rescaling k = z / ell (Sec. 4.1); phases are
// uniform on [0, 2 pi) for the random-phase form of Sec. 4.1 eq. DiscreteFT.
//
// Random numbers come from Philox4x32-10 (Salmon et al., SC'11): key = seed,
// counter = (mode lo, mode hi, slot, 0); every block yields two 64-bit words
// (out1:out0, out3:out2).  Slot 0 -> phase, slots 1-2 -> the d spatial normals,
// slots 3.. -> radial mixing normals.  Uniform on (0,1): ((w >> 11) + 1/2) 2^-53;
// normals by Box-Muller (pairs: r cos, r sin).
#include <cmath>
#include <cstdint>

#include "grf_internal.h"

namespace {

struct Philox {
    uint32_t key0, key1;

    static inline void round(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0,
                             uint32_t k1)
    {
        const uint64_t m0 = 0xD2511F53ull * x0;
        const uint64_t m1 = 0xCD9E8D57ull * x2;
        const uint32_t y0 = static_cast<uint32_t>(m1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = static_cast<uint32_t>(m0 >> 32) ^ x3 ^ k1;
        x1 = static_cast<uint32_t>(m1);
        x3 = static_cast<uint32_t>(m0);
        x0 = y0;
        x2 = y2;
    }

    // Two 64-bit words for counter (lo, hi, slot, 0).
    void block(uint64_t ctr, uint32_t slot, uint64_t& w0, uint64_t& w1) const
    {
        uint32_t x0 = static_cast<uint32_t>(ctr), x1 = static_cast<uint32_t>(ctr >> 32);
        uint32_t x2 = slot, x3 = 0;
        uint32_t k0 = key0, k1 = key1;
        round(x0, x1, x2, x3, k0, k1);
        for (int r = 1; r < 10; ++r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
            round(x0, x1, x2, x3, k0, k1);
        }
        w0 = (static_cast<uint64_t>(x1) << 32) | x0;
        w1 = (static_cast<uint64_t>(x3) << 32) | x2;
    }
};

inline double to_unit(uint64_t w) { return (static_cast<double>(w >> 11) + 0.5) * 0x1.0p-53; }

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline void box_muller(const Philox& g, uint64_t j, uint32_t slot, double out[2])
{
    uint64_t w0, w1;
    g.block(j, slot, w0, w1);
    const double rad = std::sqrt(-2.0 * std::log(to_unit(w0)));
    const double ang = kTwoPi * to_unit(w1);
    out[0] = rad * std::cos(ang);
    out[1] = rad * std::sin(ang);
}

}  // namespace

extern "C" int make_modes(const grf_spec* spec, double* z_out, double* phi_out)
{
    using grf::fail;
    if (!spec) return fail(GRF_EINVAL, "make_modes: spec is NULL");
    if (spec->dim != 2 && spec->dim != 3) return fail(GRF_EINVAL, "make_modes: dim must be 2 or 3 (got %d)", spec->dim);
    if (spec->n_modes < 1) return fail(GRF_EINVAL, "make_modes: n_modes must be >= 1");
    if (!z_out || !phi_out) return fail(GRF_EINVAL, "make_modes: output pointer is NULL");
    int dof = 0;
    switch (spec->cov) {
    case GRF_COV_GAUSSIAN:
    case GRF_COV_EXPONENTIAL:
        break;
    case GRF_COV_MATERN: {
        const double m = 2.0 * spec->nu;
        dof = static_cast<int>(std::lround(m));
        if (!(m > 0.0) || std::fabs(m - dof) > 1e-12 || dof < 1 || dof > 64)
            return fail(GRF_EINVAL, "make_modes: Matern needs 2*nu an integer in [1, 64] (nu = %g)", spec->nu);
        break;
    }
    default:
        return fail(GRF_EINVAL, "make_modes: unknown covariance %d", spec->cov);
    }

    const Philox gen{static_cast<uint32_t>(spec->seed), static_cast<uint32_t>(spec->seed >> 32)};
    const int64_t n = spec->n_modes;
    const int dim = spec->dim;
    for (int64_t j = 0; j < n; ++j) {
        const uint64_t jj = static_cast<uint64_t>(j);
        uint64_t w0, w1;
        gen.block(jj, 0u, w0, w1);
        phi_out[j] = kTwoPi * to_unit(w0);

        double g[4];
        box_muller(gen, jj, 1u, g);
        box_muller(gen, jj, 2u, g + 2);

        double radial;
        if (spec->cov == GRF_COV_GAUSSIAN) {
            radial = std::sqrt(2.0);  // k ~ N(0, 2/ell^2): correlation exp(-r^2/ell^2)
        } else if (spec->cov == GRF_COV_EXPONENTIAL) {
            double h[2];
            box_muller(gen, jj, 3u, h);
            radial = 1.0 / std::fabs(h[0]);  // multivariate Cauchy
        } else {
            double chi2 = 0.0;
            for (int i = 0; i < dof; i += 2) {
                double h[2];
                box_muller(gen, jj, 3u + static_cast<uint32_t>(i / 2), h);
                chi2 += h[0] * h[0];
                if (i + 1 < dof) chi2 += h[1] * h[1];
            }
            radial = std::sqrt(static_cast<double>(dof) / chi2);  // multivariate t, 2 nu dof
        }
        for (int a = 0; a < dim; ++a) z_out[static_cast<int64_t>(a) * n + j] = g[a] * radial;
    }
    return GRF_OK;
}

extern "C" int snap_periodic(int dim, int64_t n, const double* z, const double* ell, const double* rot,
                             const double* period, double* z_out)
{
    using grf::fail;
    if (dim != 2 && dim != 3) return fail(GRF_EINVAL, "snap_periodic: dim must be 2 or 3 (got %d)", dim);
    if (n < 0) return fail(GRF_EINVAL, "snap_periodic: n < 0");
    if (!z || !ell || !period || !z_out) return fail(GRF_EINVAL, "snap_periodic: NULL argument");
    for (int a = 0; a < dim; ++a) {
        if (!(ell[a] > 0.0) || !std::isfinite(ell[a])) return fail(GRF_EINVAL, "snap_periodic: ell[%d] must be > 0", a);
        if (!std::isfinite(period[a])) return fail(GRF_EINVAL, "snap_periodic: period[%d] must be finite", a);
    }
    double R[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) R[a][b] = rot ? rot[3 * a + b] : (a == b ? 1.0 : 0.0);
    if (rot) {  // orthonormal: rot rot^T = I on the used block
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                double d = 0.0;
                for (int c = 0; c < dim; ++c) d += R[a][c] * R[b][c];
                if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-9))
                    return fail(GRF_EINVAL, "snap_periodic: rot must be orthonormal");
            }
    }
    for (int64_t j = 0; j < n; ++j) {
        double u[3], k[3];
        for (int b = 0; b < dim; ++b) u[b] = z[static_cast<int64_t>(b) * n + j] / ell[b];
        for (int a = 0; a < dim; ++a) {
            double v = 0.0;
            for (int b = 0; b < dim; ++b) v += R[a][b] * u[b];
            if (period[a] > 0.0) v = kTwoPi * std::round(v * period[a] / kTwoPi) / period[a];
            k[a] = v;
        }
        for (int b = 0; b < dim; ++b) {
            double v = 0.0;
            for (int a = 0; a < dim; ++a) v += R[a][b] * k[a];
            z_out[static_cast<int64_t>(b) * n + j] = v * ell[b];
        }
    }
    return GRF_OK;
}

namespace {

// Standardised spectral shape (ell = 1, angular frequency, up to a constant) of App. A:
// Gaussian exp(-|u|^2 / 4), exponential (1 + |u|^2)^(-(d+1)/2), Matern with 2 nu = dof
// (1 + |u|^2 / dof)^(-(dof + d)/2).
double spectral_shape(int cov, int dim, int dof, double r2)
{
    if (cov == GRF_COV_GAUSSIAN) return std::exp(-0.25 * r2);
    if (cov == GRF_COV_EXPONENTIAL) return std::pow(1.0 + r2, -0.5 * (dim + 1));
    return std::pow(1.0 + r2 / dof, -0.5 * (dof + dim));
}

}  // namespace

extern "C" int make_modes_lattice(const grf_spec* spec, int32_t m, double du, double* z_out, double* phi_out,
                                  double* w_out)
{
    using grf::fail;
    if (!spec) return fail(GRF_EINVAL, "make_modes_lattice: spec is NULL");
    const int dim = spec->dim;
    if (dim != 2 && dim != 3) return fail(GRF_EINVAL, "make_modes_lattice: dim must be 2 or 3 (got %d)", dim);
    if (m < 2 || (m & 1) || m > (1 << 20)) return fail(GRF_EINVAL, "make_modes_lattice: m must be even, 2 .. 2^20");
    if (!(du > 0.0) || !std::isfinite(du)) return fail(GRF_EINVAL, "make_modes_lattice: du must be finite and > 0");
    if (!z_out || !phi_out || !w_out) return fail(GRF_EINVAL, "make_modes_lattice: output pointer is NULL");
    const int64_t half = m / 2;
    const int64_t n = dim == 3 ? half * m * m : half * m;
    if (spec->n_modes != n)
        return fail(GRF_EINVAL, "make_modes_lattice: n_modes must be m^dim / 2 = %lld", static_cast<long long>(n));
    int dof = 0;
    switch (spec->cov) {
    case GRF_COV_GAUSSIAN:
    case GRF_COV_EXPONENTIAL: break;
    case GRF_COV_MATERN: {
        const double t = 2.0 * spec->nu;
        dof = static_cast<int>(std::lround(t));
        if (!(t > 0.0) || std::fabs(t - dof) > 1e-12 || dof < 1 || dof > 64)
            return fail(GRF_EINVAL, "make_modes_lattice: Matern needs 2*nu an integer in [1, 64] (nu = %g)", spec->nu);
        break;
    }
    default: return fail(GRF_EINVAL, "make_modes_lattice: unknown covariance %d", spec->cov);
    }

    // lattice coordinates and the normalisation of p_j = S(u_j) / sum S (w_out holds S first)
    double total = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i0 = j % half, rest = j / half;
        const int64_t i1 = rest % m, i2 = rest / m;
        const double u0 = du * (static_cast<double>(i0) + 0.5);
        const double u1 = du * (static_cast<double>(i1 - half) + 0.5);
        const double u2 = dim == 3 ? du * (static_cast<double>(i2 - half) + 0.5) : 0.0;
        z_out[j] = u0;
        z_out[n + j] = u1;
        if (dim == 3) z_out[2 * n + j] = u2;
        const double s = spectral_shape(spec->cov, dim, dof, u0 * u0 + u1 * u1 + u2 * u2);
        w_out[j] = s;
        total += s;
    }
    const Philox gen{static_cast<uint32_t>(spec->seed), static_cast<uint32_t>(spec->seed >> 32)};
    for (int64_t j = 0; j < n; ++j) {
        double g[2];
        box_muller(gen, static_cast<uint64_t>(j), 1u, g);  // (W_j, W'_j)
        double ph = -std::atan2(g[1], g[0]);
        if (ph < 0.0) ph += kTwoPi;
        phi_out[j] = ph;
        w_out[j] = std::sqrt(w_out[j] / total * (g[0] * g[0] + g[1] * g[1]) * 0.5 * static_cast<double>(n));
    }
    return GRF_OK;
}

extern "C" int grf_modes_init(const grf_spec* spec, const double* z, const double* phi, grf_modes* out)
{
    using grf::fail;
    if (!spec || !out) return fail(GRF_EINVAL, "grf_modes_init: spec or out is NULL");
    if (spec->dim != 2 && spec->dim != 3)
        return fail(GRF_EINVAL, "grf_modes_init: dim must be 2 or 3 (got %d)", spec->dim);
    if (spec->n_modes < 1) return fail(GRF_EINVAL, "grf_modes_init: n_modes must be >= 1");
    if (spec->cov < GRF_COV_GAUSSIAN || spec->cov > GRF_COV_MATERN)
        return fail(GRF_EINVAL, "grf_modes_init: unknown covariance %d", spec->cov);
    if (!(spec->sigma2 >= 0.0) || !std::isfinite(spec->sigma2))
        return fail(GRF_EINVAL, "grf_modes_init: sigma2 must be finite and >= 0");
    if (spec->len_convention != 0 && spec->len_convention != 1)
        return fail(GRF_EINVAL, "grf_modes_init: len_convention must be 0 or 1 (got %d)", spec->len_convention);
    for (int a = 0; a < spec->dim; ++a)
        if (!(spec->ell[a] > 0.0) || !std::isfinite(spec->ell[a]))
            return fail(GRF_EINVAL, "grf_modes_init: ell[%d] must be finite and > 0", a);
    if (!z || !phi) return fail(GRF_EINVAL, "grf_modes_init: z or phi is NULL");
    // The Gaussian correlation written with the integral scale lambda, exp(-(pi/4)(r/lambda)^2)
    // (eq. gauSpe), is exp(-r^2/ell^2) with ell = 2 lambda / sqrt(pi); the exponential and
    // Matern forms use lambda as the length itself.
    const double scale = (spec->len_convention == 1 && spec->cov == GRF_COV_GAUSSIAN) ? 2.0 / std::sqrt(M_PI) : 1.0;
    grf_modes m{};
    m.dim = spec->dim;
    m.n = spec->n_modes;
    m.z = z;
    m.phi = phi;
    m.sigma = std::sqrt(spec->sigma2);
    for (int a = 0; a < 3; ++a) m.ell[a] = a < spec->dim ? scale * spec->ell[a] : 1.0;
    m.rotated = 0;
    m.rot[0] = m.rot[4] = m.rot[8] = 1.0;
    m.w = nullptr;
    *out = m;
    return GRF_OK;
}
