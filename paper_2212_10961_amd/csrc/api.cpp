// C-ABI entry points: validation, workspace layout and dispatch to the kernels.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "grf_internal.h"

namespace grf {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

namespace {
struct KernelTimer {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t used = 0;             // events recorded since enable
};
KernelTimer& ktimer()
{
    static KernelTimer t;
    return t;
}
}  // namespace

void timer_mark(hipStream_t s, bool begin)
{
    KernelTimer& t = ktimer();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on) return;
    if (begin && (t.used & 1)) return;   // unmatched begin: ignore
    if (!begin && !(t.used & 1)) return; // stop without start
    if (t.used == t.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        t.ev.push_back(e);
    }
    if (hipEventRecord(t.ev[t.used], s) == hipSuccess) ++t.used;
}

bool timer_take_pair(hipEvent_t* start, hipEvent_t* stop)
{
    KernelTimer& t = ktimer();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on || (t.used & 1)) return false;
    while (t.ev.size() < t.used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        t.ev.push_back(e);
    }
    *start = t.ev[t.used];
    *stop = t.ev[t.used + 1];
    t.used += 2;
    return true;
}

int fail_hip(hipError_t e, const char* what)
{
    return fail(GRF_EDEVICE, "HIP error in %s: %s", what, hipGetErrorString(e));
}

Epi make_epi(const grf_epi* e)
{
    Epi r{};
    if (e) {
        r.mu = e->mu;
        r.nthr = e->n_thresholds;
        for (int i = 0; i < GRF_MAX_THRESHOLDS; ++i) r.thr[i] = i < e->n_thresholds ? e->thresholds[i] : 0.f;
    }
    return r;
}

int check_modes(const grf_modes* m, const char* fn)
{
    if (!m) return fail(GRF_EINVAL, "%s: modes is NULL", fn);
    if (m->dim != 2 && m->dim != 3) return fail(GRF_EINVAL, "%s: dim must be 2 or 3 (got %d)", fn, m->dim);
    if (m->n < 1) return fail(GRF_EINVAL, "%s: number of modes must be >= 1", fn);
    if (m->n > (int64_t(1) << 31)) return fail(GRF_EINVAL, "%s: too many modes", fn);
    if (!m->z || !m->phi) return fail(GRF_EINVAL, "%s: modes z/phi pointer is NULL", fn);
    if (!(m->sigma >= 0.0) || !std::isfinite(m->sigma)) return fail(GRF_EINVAL, "%s: sigma must be finite and >= 0", fn);
    for (int a = 0; a < m->dim; ++a)
        if (!(m->ell[a] > 0.0) || !std::isfinite(m->ell[a]))
            return fail(GRF_EINVAL, "%s: ell[%d] must be finite and > 0", fn, a);
    if (m->rotated != 0 && m->rotated != 1) return fail(GRF_EINVAL, "%s: rotated must be 0 or 1", fn);
    if (m->rotated)
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(m->rot[i])) return fail(GRF_EINVAL, "%s: rot must be finite", fn);
    return GRF_OK;
}

// Axis-aligned view of a table: a rotated table's wavevectors k = R diag(1/ell) z go to
// `kbuf` (rot_ws_bytes(m) bytes of device workspace) and are evaluated as z' = k, ell' = 1.
hipError_t aligned_modes(const grf_modes* m, void* kbuf, hipStream_t s, grf_modes* out)
{
    *out = *m;
    if (!m->rotated) return hipSuccess;
    const hipError_t e = launch_rotate_modes(m->z, m->dim, m->n, m->rot, m->ell, static_cast<double*>(kbuf), s);
    out->z = static_cast<const double*>(kbuf);
    out->ell[0] = out->ell[1] = out->ell[2] = 1.0;
    out->rotated = 0;
    return e;
}

int check_grid(const grf_grid* g, int dim, const char* fn)
{
    if (!g) return fail(GRF_EINVAL, "%s: grid is NULL", fn);
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1) return fail(GRF_EINVAL, "%s: grid n[%d] must be >= 1", fn, a);
        if (a < dim && (!std::isfinite(g->h[a]) || !std::isfinite(g->origin[a])))
            return fail(GRF_EINVAL, "%s: grid origin/h must be finite", fn);
    }
    if (dim == 2 && g->n[2] != 1) return fail(GRF_EINVAL, "%s: dim 2 grid needs n[2] == 1", fn);
    if (g->n[0] > (1 << 24) || g->n[1] > (1 << 24) || g->n[2] > (1 << 24))
        return fail(GRF_EINVAL, "%s: grid side too large", fn);
    const int64_t cells = g->n[0] * g->n[1] * g->n[2];
    if (cells > (int64_t(1) << 40)) return fail(GRF_EINVAL, "%s: grid too large", fn);
    return GRF_OK;
}

int check_epi(const grf_epi* e, const float* k, const uint8_t* ind, const char* fn)
{
    if ((k || ind) && !e) return fail(GRF_EINVAL, "%s: epi is NULL but k or ind requested", fn);
    if (e && (e->n_thresholds < 0 || e->n_thresholds > GRF_MAX_THRESHOLDS))
        return fail(GRF_EINVAL, "%s: n_thresholds must be in [0, %d]", fn, GRF_MAX_THRESHOLDS);
    if (ind && e && e->n_thresholds < 1) return fail(GRF_EINVAL, "%s: ind requested with no thresholds", fn);
    if (e)
        for (int i = 1; i < e->n_thresholds; ++i)
            if (!(e->thresholds[i] >= e->thresholds[i - 1]))
                return fail(GRF_EINVAL, "%s: thresholds must be ascending", fn);
    return GRF_OK;
}


// The point-sum form GRF_DIRECT_F32 resolves to: binned for many points, else per point.
static int resolve_points_f32(int method, int64_t P)
{
    if (method != GRF_DIRECT_F32) return method;
    return (P >= kBinMinPoints && P <= kBinMaxPoints) ? GRF_DIRECT_F32_BINNED : GRF_DIRECT_F32_POINTWISE;
}

// Workspace of eval_field_points: per-mode parameters, the binned pass's sort and offsets, plus
// the per-slice partial sums when an FP32 form splits the modes across blocks.
static size_t points_ws_bytes(int64_t n, int64_t P, int method)
{
    method = resolve_points_f32(method, P);
    size_t b = align256(sizeof(double) * 4 * size_t(padded_modes(n)));
    int slices = 1;
    if (method == GRF_DIRECT_F32_POINTWISE) slices = points_mode_slices(P, n);
    if (method == GRF_DIRECT_F32_BINNED) {
        b += bin_ws_bytes(P, padded_modes(n));
        slices = bin_mode_slices(P, n);
    }
    if (slices > 1) b += align256(sizeof(float) * size_t(slices) * size_t(P));
    return b;
}

static int resolve_grid_method(int method, const grf_grid* g)
{
    if (method == GRF_AUTO) {
        const int64_t cells = g->n[0] * g->n[1] * g->n[2];
        return cells >= (int64_t(1) << 16) ? GRF_SEP_F16 : GRF_DIRECT_F32;
    }
    return method;
}

GridWs grid_ws(const grf_modes* m, const grf_grid* g, int method, void* base)
{
    GridWs w;
    Carve c(base);
    const int64_t ldp = padded_modes(m->n);
    const int dim = m->dim;
    if (method == GRF_DIRECT_F32) {
        for (int a = 0; a < 3; ++a) w.t[a] = c.take<float>(size_t(g->n[a]) * ldp);
    } else if (method == GRF_DIRECT_F64) {
        for (int a = 0; a < 3; ++a) w.t[a] = c.take<double>(size_t(g->n[a]) * ldp);
        const ModeSlices ms = direct_grid_f64_slices(g->n, m->n);
        if (ms.slices > 1) w.partial = c.take<double>(size_t(ms.slices) * size_t(g->n[0] * g->n[1] * g->n[2]));
    } else if (is_sep(method)) {
        const bool hilo = is_hilo(method);
        if (dim == 2) {
            w.t[0] = c.take<uint32_t>(size_t(g->n[0]) * ldp);
            if (hilo) w.tlo[0] = c.take<uint32_t>(size_t(g->n[0]) * ldp);
        } else {
            // Ex feeds the on-the-fly product Ex * Ez[z]: half pairs for one pass, float2 for hi+lo
            if (hilo) w.t[0] = c.take<float2>(size_t(g->n[0]) * ldp);
            else w.t[0] = c.take<uint32_t>(size_t(g->n[0]) * ldp);
            w.t[2] = c.take<float2>(size_t(g->n[2]) * ldp);
        }
        w.t[1] = c.take<uint32_t>(size_t(g->n[1]) * ldp);
        if (hilo) w.tlo[1] = c.take<uint32_t>(size_t(g->n[1]) * ldp);
        // grids of few tiles: the modes split over slices whose sums are added afterwards
        w.slices = sep_mode_slices(method, dim, g->n[0], g->n[1], g->n[2], ldp, &w.pairs);
        if (w.slices > 1) {
            const size_t before = c.used;
            w.partial = c.take<float>(size_t(w.slices) * size_t(g->n[0] * g->n[1] * g->n[2]));
            w.split_bytes = c.used - before;
        }
    }
    w.bytes = c.used;
    return w;
}

int grid_ws_bytes(const char* fn, const grf_modes* modes, const grf_grid* grid, int method, size_t* bytes,
                  size_t* least)
{
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if ((rc = check_grid(grid, modes->dim, fn))) return rc;
    if (!bytes || !least) return fail(GRF_EINVAL, "%s: bytes is NULL", fn);
    method = resolve_grid_method(method, grid);
    if (method < GRF_DIRECT_F32 || method > GRF_SEP_F16_X3) return fail(GRF_EINVAL, "%s: unknown method %d", fn, method);
    const GridWs w = grid_ws(modes, grid, method, nullptr);
    *bytes = rot_ws_bytes(modes) + w.bytes;
    *least = *bytes - w.split_bytes;
    return GRF_OK;
}

int grid_table_descs(const grf_modes* m, const grf_grid* g, int method, const GridWs& w, AxisTableArgs* out)
{
    const int64_t ldp = padded_modes(m->n);
    int nd = 0;
    for (int a = 0; a < 3; ++a) {
        AxisTableArgs t{};
        t.z = m->z;
        t.phi = m->phi;
        t.n = m->n;
        t.ldp = ldp;
        t.axis = a;
        t.ell = a < m->dim ? m->ell[a] : 1.0;
        t.freq_scale = 1.0 / (6.283185307179586476925286766559 * t.ell);
        t.origin = g->origin[a];
        t.h = g->h[a];
        t.count = g->n[a];
        t.with_psi = (a == 1);
        t.conj = false;
        t.out = w.t[a];
        t.out_lo = w.tlo[a];
        t.w = nullptr;
        if (a >= m->dim) t.z = nullptr;  // axis absent: zero phase
        if (method == GRF_DIRECT_F32) {
            t.format = TF_REV_F32;
        } else if (method == GRF_DIRECT_F64) {
            t.format = TF_REV_F64;
        } else {
            const bool hilo = is_hilo(method), bf = is_bf16(method);
            // single-pass operands are rounded to fp16/bf16 (2^-11 or 2^-8): the hardware
            // sin/cos of the FP64-reduced fraction (|err| ~1e-7) is far below that
            t.fast_trig = !hilo;
            if (a == 1 || (a == 0 && m->dim == 2)) {
                t.format = bf ? (hilo ? TF_BF16_HILO : TF_BF16) : (hilo ? TF_F16_HILO : TF_F16);
                t.conj = (a == 0);
                t.blocked = true;
                if (a == 1) t.w = m->w;  // per-mode weights ride on the y operand (with the phase)
            } else if (a == 0) {  // 3-D x axis: (Re, -Im) Ex for the product with Ez
                t.format = hilo ? TF_CPLX_F32 : (bf ? TF_BF16 : TF_F16);
                t.conj = true;
                t.blocked = true;
            } else if (a == 2 && m->dim == 3) {
                // the one-pass fp16 form multiplies in packed fp16; the others in FP32
                t.format = (!hilo && !bf) ? TF_F16 : TF_CPLX_F32;
            } else {
                continue;  // dim 2: no z table for the separable form
            }
        }
        out[nd++] = t;
    }
    return nd;
}

static hipError_t build_tables(const grf_modes* m, const grf_grid* g, int method, const GridWs& w,
                               hipStream_t s)
{
    AxisTableArgs d[3];
    const int nd = grid_table_descs(m, g, method, w, d);
    return launch_axis_tables(d, nd, s);
}

}  // namespace grf

using namespace grf;

extern "C" {

int grf_version(void) { return GRF_VERSION; }

int grf_kernel_timer_enable(int enable)
{
    KernelTimer& t = ktimer();
    std::lock_guard<std::mutex> lk(t.mu);
    t.on = enable != 0;
    if (t.on) t.used = 0;
    return GRF_OK;
}

int grf_kernel_timer_read(double* total_ms, int64_t* launches)
{
    if (!total_ms || !launches) return fail(GRF_EINVAL, "grf_kernel_timer_read: NULL output");
    KernelTimer& t = ktimer();
    std::lock_guard<std::mutex> lk(t.mu);
    double sum = 0.0;
    const size_t pairs = t.used / 2;
    for (size_t i = 0; i < pairs; ++i) {
        GRF_HIP(hipEventSynchronize(t.ev[2 * i + 1]));
        float ms = 0.f;
        GRF_HIP(hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = static_cast<int64_t>(pairs);
    return GRF_OK;
}

const char* grf_last_error(void) { return g_err; }

int eval_field_grid_ws_size(const grf_modes* modes, const grf_grid* grid, int method, size_t* bytes)
{
    size_t least = 0;
    return grf::grid_ws_bytes("eval_field_grid_ws_size", modes, grid, method, bytes, &least);
}

}  // extern "C"

namespace grf {

// Tables and sum of one grid evaluation with a prepared epilogue; the caller has validated
// the modes, grid, method (resolved), tile and outputs, and `ws` holds grid_ws(...) bytes.
// Arguments of the separable kernel for one field whose tables are laid out as `w`.
static SepArgs sep_args(const grf_modes* modes, const grf_grid* grid, int method, int tile, const Epi& e, float* y,
                        float* k, uint8_t* ind, const GridWs& w)
{
    SepArgs a{};
    a.method = method;
    a.n = modes->n;
    a.ldp = padded_modes(modes->n);
    a.nx = grid->n[0];
    a.ny = grid->n[1];
    a.nz = grid->n[2];
    a.px = w.t[0];
    a.px_lo = w.tlo[0];
    a.qy = w.t[1];
    a.qy_lo = w.tlo[1];
    a.ez = modes->dim == 3 ? static_cast<const float2*>(w.t[2]) : nullptr;
    a.amp = static_cast<float>(modes->sigma * std::sqrt(2.0 / static_cast<double>(modes->n)));
    a.epi = e;
    a.y = y;
    a.k = k;
    a.ind = ind;
    a.tile = tile;  // -1: size-based default
    if (tile < 0 && w.partial) {  // the mode split of the default tile (grid_ws decides)
        a.partial = static_cast<float*>(w.partial);
        a.slices = w.slices;
        a.pairs = w.pairs;
    }
    return a;
}

static int grid_launch(const grf_modes* modes, const grf_grid* grid, int method, int tile, const Epi& e, float* y,
                       float* k, uint8_t* ind, void* ws, hipStream_t s, bool allow_split = true)
{
    GridWs w = grid_ws(modes, grid, method, ws);
    if (!allow_split && w.split_bytes) w.partial = nullptr;  // the workspace holds the tables only
    const float amp = static_cast<float>(modes->sigma * std::sqrt(2.0 / static_cast<double>(modes->n)));
    const int64_t ldp = padded_modes(modes->n);

    GRF_HIP(build_tables(modes, grid, method, w, s));
    if (is_sep(method)) {
        SepArgs a = sep_args(modes, grid, method, tile, e, y, k, ind, w);
        a.timed = true;
        GRF_HIP(launch_sep(a, s));
        return GRF_OK;
    }
    TimedScope timed(s);
    if (method == GRF_DIRECT_F32) {
        GRF_HIP(launch_direct_grid_f32(static_cast<const float*>(w.t[0]), static_cast<const float*>(w.t[1]),
                                       static_cast<const float*>(w.t[2]), modes->w, modes->n, ldp, grid->n, amp, e,
                                       y, k, ind, s));
    } else if (method == GRF_DIRECT_F64) {
        const double amp64 = modes->sigma * std::sqrt(2.0 / static_cast<double>(modes->n));
        GRF_HIP(launch_direct_grid_f64(static_cast<const double*>(w.t[0]), static_cast<const double*>(w.t[1]),
                                       static_cast<const double*>(w.t[2]), modes->w, modes->n, ldp, grid->n, amp64, e,
                                       0.0, y, k, ind, nullptr, nullptr, static_cast<double*>(w.partial), s));
    }
    return GRF_OK;
}

static int check_grid_method(const char* fn, const grf_grid* grid, int* method, int tile)
{
    *method = resolve_grid_method(*method, grid);
    if (*method < GRF_DIRECT_F32 || *method > GRF_SEP_F16_X3)
        return fail(GRF_EINVAL, "%s: unknown method %d", fn, *method);
    if (tile < -1 || tile >= sep_tile_count())
        return fail(GRF_EINVAL, "%s: tile selector %d outside [-1, %d)", fn, tile, sep_tile_count());
    if (tile >= 0 && !is_sep(*method)) return fail(GRF_EINVAL, "%s: tile selectors apply to separable methods", fn);
    return GRF_OK;
}

int grid_eval(const char* fn, const grf_modes* modes, const grf_grid* grid, int method, int tile,
                     const grf_epi* epi, float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes, void* stream)
{
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if ((rc = check_grid(grid, modes->dim, fn))) return rc;
    if (!y && !k && !ind) return fail(GRF_EINVAL, "%s: no output requested", fn);
    if ((rc = check_epi(epi, k, ind, fn))) return rc;
    if ((rc = check_grid_method(fn, grid, &method, tile))) return rc;
    const size_t rb = rot_ws_bytes(modes);
    const GridWs gw = grid_ws(modes, grid, method, nullptr);
    // A workspace without room for the mode split's sums (eval_field_grid_ws_size counts them)
    // runs the unsplit contraction.
    const size_t need = rb + gw.bytes - gw.split_bytes;
    if (ws_bytes < need || (!ws && need))
        return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    grf_modes am;
    GRF_HIP(aligned_modes(modes, ws, s, &am));
    return grid_launch(&am, grid, method, tile, make_epi(epi), y, k, ind, static_cast<char*>(ws) + rb, s,
                       ws_bytes >= rb + gw.bytes);
}

// ---------------------------------------------------------------- bitruncated (pluri-Gaussian) rule

static int check_trunc2(const grf_trunc2* r, bool want_value, const char* fn)
{
    if (!r) return fail(GRF_EINVAL, "%s: rule is NULL", fn);
    if (r->n_t < 0 || r->n_t > GRF_MAX_THRESHOLDS || r->n_s < 0 || r->n_s > GRF_MAX_THRESHOLDS)
        return fail(GRF_EINVAL, "%s: threshold counts must be in [0, %d]", fn, GRF_MAX_THRESHOLDS);
    for (int i = 1; i < r->n_t; ++i)
        if (!(r->t[i] >= r->t[i - 1])) return fail(GRF_EINVAL, "%s: thresholds t must be ascending", fn);
    for (int i = 1; i < r->n_s; ++i)
        if (!(r->s[i] >= r->s[i - 1])) return fail(GRF_EINVAL, "%s: thresholds s must be ascending", fn);
    if (r->n_values < 0 || r->n_values > GRF_MAX_FACIES)
        return fail(GRF_EINVAL, "%s: n_values must be in [0, %d]", fn, GRF_MAX_FACIES);
    if (want_value) {
        const int bins = (r->n_t + 1) * (r->n_s + 1);
        for (int b = 0; b < bins; ++b)
            if (r->rule[b] >= r->n_values)
                return fail(GRF_EINVAL, "%s: rule entry %d names facies %d but only %d values are given", fn, b,
                            r->rule[b], r->n_values);
    }
    return GRF_OK;
}

static_assert(kRuleBytes <= GRF_PLURI_APPLY_WS_BYTES, "pluri_apply workspace holds the rule tables");

// `tables` is device memory holding the rule's lookup tables (launch_rule_tables).
static PluriEpi make_pluri(const grf_trunc2* r, const void* tables)
{
    PluriEpi e{};
    e.nt = r->n_t;
    for (int i = 0; i < r->n_t; ++i) e.t[i] = r->t[i];
    e.ns = r->n_s;
    for (int i = 0; i < r->n_s; ++i) e.s[i] = r->s[i];
    e.rule = static_cast<const uint8_t*>(tables);
    e.values = reinterpret_cast<const float*>(static_cast<const uint8_t*>(tables) + 256);
    return e;
}

static int check_pair(const grf_modes* m1, const grf_modes* m2, const char* fn)
{
    int rc;
    if ((rc = check_modes(m1, fn)) || (rc = check_modes(m2, fn))) return rc;
    if (m1->dim != m2->dim) return fail(GRF_EINVAL, "%s: both fields must have the same dim", fn);
    return GRF_OK;
}

// Workspace of the bitruncated grid: the rule's tables, each field the caller does not keep,
// and the larger of the two fields' table layouts (the two evaluations run one after the other).
static size_t pluri_grid_ws(const grf_modes* m1, const grf_modes* m2, const grf_grid* g, int method, bool own_y1,
                            bool own_y2)
{
    const int64_t C = g->n[0] * g->n[1] * g->n[2];
    // separable forms: both fields' tables at once (one table launch, one contraction launch)
    const size_t b1 = grid_ws(m1, g, method, nullptr).bytes, b2 = grid_ws(m2, g, method, nullptr).bytes;
    const size_t t = is_sep(method) ? b1 + b2 : std::max(b1, b2);
    const size_t f = align256(sizeof(float) * size_t(C));
    return align256(kRuleBytes) + rot_ws_bytes(m1) + rot_ws_bytes(m2) + (own_y1 ? f : 0) + (own_y2 ? f : 0) + t;
}

}  // namespace grf

extern "C" {

int eval_pluri_grid_ws_size(const grf_modes* m1, const grf_modes* m2, const grf_grid* grid, int method,
                            size_t* bytes)
{
    const char* fn = "eval_pluri_grid_ws_size";
    int rc;
    if ((rc = check_pair(m1, m2, fn))) return rc;
    if ((rc = check_grid(grid, m1->dim, fn))) return rc;
    if (!bytes) return fail(GRF_EINVAL, "%s: bytes is NULL", fn);
    if ((rc = check_grid_method(fn, grid, &method, -1))) return rc;
    *bytes = pluri_grid_ws(m1, m2, grid, method, true, true);
    return GRF_OK;
}

int eval_pluri_grid(const grf_modes* m1, const grf_modes* m2, const grf_grid* grid, int method,
                    const grf_trunc2* rule, uint8_t* facies, float* value, float* y1, float* y2, void* ws,
                    size_t ws_bytes, void* stream)
{
    const char* fn = "eval_pluri_grid";
    int rc;
    if ((rc = check_pair(m1, m2, fn))) return rc;
    if ((rc = check_grid(grid, m1->dim, fn))) return rc;
    if (!facies && !value) return fail(GRF_EINVAL, "%s: facies or value output required", fn);
    if ((rc = check_trunc2(rule, value != nullptr, fn))) return rc;
    if ((rc = check_grid_method(fn, grid, &method, -1))) return rc;
    const size_t need = pluri_grid_ws(m1, m2, grid, method, y1 == nullptr, y2 == nullptr);
    if (!ws || ws_bytes < need) return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t C = grid->n[0] * grid->n[1] * grid->n[2];
    Carve c(ws);
    uint8_t* rt = c.take<uint8_t>(kRuleBytes);
    void* k1 = c.base + c.used;
    c.used += rot_ws_bytes(m1);
    void* k2 = c.base + c.used;
    c.used += rot_ws_bytes(m2);
    float* f1 = y1 ? y1 : c.take<float>(size_t(C));
    float* f2 = y2 ? y2 : c.take<float>(size_t(C));
    void* tabs = c.base + c.used;
    grf_modes a1, a2;
    GRF_HIP(aligned_modes(m1, k1, s, &a1));
    GRF_HIP(aligned_modes(m2, k2, s, &a2));
    GRF_HIP(launch_rule_tables(*rule, rt, s));
    if (is_sep(method)) {
        // both fields: one launch of the six (2-D: four) tables, one of the contraction
        const GridWs w1 = grid_ws(&a1, grid, method, tabs);
        const GridWs w2 = grid_ws(&a2, grid, method, static_cast<char*>(tabs) + w1.bytes);
        AxisTableArgs d[6];
        const int nd1 = grid_table_descs(&a1, grid, method, w1, d);
        const int nd2 = grid_table_descs(&a2, grid, method, w2, d + nd1);
        GRF_HIP(launch_axis_tables(d, nd1 + nd2, s));
        const SepArgs s2 = sep_args(&a2, grid, method, -1, Epi{}, f2, nullptr, nullptr, w2);
        SepArgs s1 = sep_args(&a1, grid, method, -1, Epi{}, f1, nullptr, nullptr, w1);
        s1.timed = true;
        GRF_HIP(launch_sep_pair(s1, &s2, s));
    } else {
        if ((rc = grid_launch(&a1, grid, method, -1, Epi{}, f1, nullptr, nullptr, tabs, s))) return rc;
        if ((rc = grid_launch(&a2, grid, method, -1, Epi{}, f2, nullptr, nullptr, tabs, s))) return rc;
    }
    GRF_HIP(launch_pluri_epilogue(f1, f2, C, make_pluri(rule, rt), facies, value, s));
    return GRF_OK;
}

int pluri_apply(const float* y1, const float* y2, int64_t n, const grf_trunc2* rule, uint8_t* facies, float* value,
                void* ws, size_t ws_bytes, void* stream)
{
    const char* fn = "pluri_apply";
    if (n < 0) return fail(GRF_EINVAL, "%s: n < 0", fn);
    int rc;
    if ((rc = check_trunc2(rule, value != nullptr, fn))) return rc;
    if (n == 0) return GRF_OK;
    if (!facies && !value) return fail(GRF_EINVAL, "%s: facies or value output required", fn);
    if (!y1 || !y2) return fail(GRF_EINVAL, "%s: y1 and y2 are required", fn);
    if (!ws || ws_bytes < GRF_PLURI_APPLY_WS_BYTES)
        return fail(GRF_ENOMEM, "%s: workspace of %d bytes needed, %zu given", fn, GRF_PLURI_APPLY_WS_BYTES, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    GRF_HIP(launch_rule_tables(*rule, ws, s));
    TimedScope timed(s);
    GRF_HIP(launch_pluri_epilogue(y1, y2, n, make_pluri(rule, ws), facies, value, s));
    return GRF_OK;
}

}  // extern "C"

namespace grf {

// Per-mode parameters and the point sum with a prepared epilogue (validated by the caller;
// `ws` holds points_ws_bytes(...)).
static int points_launch(const grf_modes* modes, const double* xyz, int64_t n_points, int method, const Epi& e,
                         float* y, float* k, uint8_t* ind, void* ws, hipStream_t s, bool timed = true)
{
    const int64_t ldp = padded_modes(modes->n);
    method = resolve_points_f32(method, n_points);
    Carve c(ws);
    double* params = c.take<double>(4 * ldp);
    GRF_HIP(launch_mode_params(modes->z, modes->phi, modes->dim, modes->n, ldp, modes->ell, params, s));
    const float amp = static_cast<float>(modes->sigma * std::sqrt(2.0 / static_cast<double>(modes->n)));
    if (method == GRF_DIRECT_F32_BINNED) {
        char* bins = c.take<char>(bin_ws_bytes(n_points, ldp));
        float* partial = c.take<float>(size_t(bin_mode_slices(n_points, modes->n)) * n_points);
        GRF_HIP(launch_points_binned(params, modes->w, modes->n, ldp, modes->dim, xyz, n_points, amp, e, y, k, ind,
                                     bins, partial, s));
        return GRF_OK;
    }
    float* partial = method == GRF_DIRECT_F32_POINTWISE
                         ? c.take<float>(size_t(points_mode_slices(n_points, modes->n)) * n_points)
                         : nullptr;
    TimedScope scope(s, timed);
    GRF_HIP(launch_direct_points(params, modes->w, modes->n, modes->dim, xyz, n_points, method == GRF_DIRECT_F64, amp,
                                 e, y, k, ind, partial, s));
    return GRF_OK;
}

static int check_points_method(const char* fn, int* method, int64_t n_points)
{
    if (*method == GRF_AUTO) *method = GRF_DIRECT_F32;
    if (is_sep(*method)) return fail(GRF_EUNSUPPORTED, "%s: separable methods need a structured grid", fn);
    if (*method != GRF_DIRECT_F32 && *method != GRF_DIRECT_F64 && *method != GRF_DIRECT_F32_BINNED &&
        *method != GRF_DIRECT_F32_POINTWISE)
        return fail(GRF_EINVAL, "%s: unknown method %d", fn, *method);
    if (*method == GRF_DIRECT_F32_BINNED && n_points > kBinMaxPoints)
        return fail(GRF_EUNSUPPORTED, "%s: the binned form takes at most %lld points", fn,
                    static_cast<long long>(kBinMaxPoints));
    return GRF_OK;
}

}  // namespace grf

extern "C" {

int eval_pluri_points_ws_size(const grf_modes* m1, const grf_modes* m2, int64_t n_points, int method,
                              size_t* bytes)
{
    const char* fn = "eval_pluri_points_ws_size";
    int rc;
    if ((rc = check_pair(m1, m2, fn))) return rc;
    if (!bytes) return fail(GRF_EINVAL, "%s: bytes is NULL", fn);
    if (n_points < 0) return fail(GRF_EINVAL, "%s: n_points < 0", fn);
    if ((rc = check_points_method(fn, &method, n_points))) return rc;
    *bytes = align256(kRuleBytes) + rot_ws_bytes(m1) + rot_ws_bytes(m2) + 2 * align256(sizeof(float) * size_t(n_points)) +
             std::max(points_ws_bytes(m1->n, n_points, method), points_ws_bytes(m2->n, n_points, method));
    return GRF_OK;
}

int eval_pluri_points(const grf_modes* m1, const grf_modes* m2, const double* xyz, int64_t n_points, int method,
                      const grf_trunc2* rule, uint8_t* facies, float* value, float* y1, float* y2, void* ws,
                      size_t ws_bytes, void* stream)
{
    const char* fn = "eval_pluri_points";
    int rc;
    if ((rc = check_pair(m1, m2, fn))) return rc;
    if (n_points < 0) return fail(GRF_EINVAL, "%s: n_points < 0", fn);
    if (n_points > (int64_t(1) << 40)) return fail(GRF_EINVAL, "%s: too many points", fn);
    if ((rc = check_points_method(fn, &method, n_points))) return rc;
    if ((rc = check_trunc2(rule, value != nullptr, fn))) return rc;
    if (n_points == 0) return GRF_OK;
    if (!facies && !value) return fail(GRF_EINVAL, "%s: facies or value output required", fn);
    if (!xyz) return fail(GRF_EINVAL, "%s: xyz is NULL", fn);
    const size_t fb = align256(sizeof(float) * size_t(n_points));
    const size_t need = align256(kRuleBytes) + rot_ws_bytes(m1) + rot_ws_bytes(m2) + (y1 ? 0 : fb) + (y2 ? 0 : fb) +
                        std::max(points_ws_bytes(m1->n, n_points, method), points_ws_bytes(m2->n, n_points, method));
    if (!ws || ws_bytes < need) return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carve c(ws);
    uint8_t* rt = c.take<uint8_t>(kRuleBytes);
    void* k1 = c.base + c.used;
    c.used += rot_ws_bytes(m1);
    void* k2 = c.base + c.used;
    c.used += rot_ws_bytes(m2);
    float* f1 = y1 ? y1 : c.take<float>(size_t(n_points));
    float* f2 = y2 ? y2 : c.take<float>(size_t(n_points));
    void* rest = c.base + c.used;
    grf_modes a1, a2;
    GRF_HIP(aligned_modes(m1, k1, s, &a1));
    GRF_HIP(aligned_modes(m2, k2, s, &a2));
    GRF_HIP(launch_rule_tables(*rule, rt, s));
    if ((rc = points_launch(&a1, xyz, n_points, method, Epi{}, f1, nullptr, nullptr, rest, s))) return rc;
    if ((rc = points_launch(&a2, xyz, n_points, method, Epi{}, f2, nullptr, nullptr, rest, s))) return rc;
    GRF_HIP(launch_pluri_epilogue(f1, f2, n_points, make_pluri(rule, rt), facies, value, s));
    return GRF_OK;
}

}  // extern "C"

extern "C" {

int eval_field_grid(const grf_modes* modes, const grf_grid* grid, int method, const grf_epi* epi,
                    float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes, void* stream)
{
    return grid_eval("eval_field_grid", modes, grid, method, -1, epi, y, k, ind, ws, ws_bytes, stream);
}

int eval_field_grid_tile(const grf_modes* modes, const grf_grid* grid, int method, int tile, const grf_epi* epi,
                         float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes, void* stream)
{
    return grid_eval("eval_field_grid_tile", modes, grid, method, tile, epi, y, k, ind, ws, ws_bytes, stream);
}

int grf_sep_tile_count(void) { return sep_tile_count(); }

int grf_sep_tile_shape(int tile, int method, int dim, int32_t* rows, int32_t* cols, int32_t* slices)
{
    const char* fn = "grf_sep_tile_shape";
    if (tile < 0 || tile >= sep_tile_count()) return fail(GRF_EINVAL, "%s: tile %d outside [0, %d)", fn, tile, sep_tile_count());
    if (!is_sep(method)) return fail(GRF_EINVAL, "%s: method %d is not separable", fn, method);
    if (dim != 2 && dim != 3) return fail(GRF_EINVAL, "%s: dim must be 2 or 3", fn);
    if (!rows || !cols || !slices) return fail(GRF_EINVAL, "%s: NULL output", fn);
    int bm = 0, bn = 0;
    sep_tile_shape(tile, &bm, &bn);
    *rows = bm;
    *cols = bn;
    *slices = sep_tile_slices(tile, method, dim == 3);
    return GRF_OK;
}

int eval_field_grid_f64(const grf_modes* modes, const grf_grid* grid, double mu, double* y64, double* k64,
                        void* ws, size_t ws_bytes, void* stream)
{
    const char* fn = "eval_field_grid_f64";
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if ((rc = check_grid(grid, modes->dim, fn))) return rc;
    if (!y64 && !k64) return fail(GRF_EINVAL, "%s: no output requested", fn);
    if (!std::isfinite(mu)) return fail(GRF_EINVAL, "%s: mu must be finite", fn);
    const size_t rb = rot_ws_bytes(modes);
    const size_t need = rb + grid_ws(modes, grid, GRF_DIRECT_F64, nullptr).bytes;
    if (ws_bytes < need || !ws)
        return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    grf_modes am;
    GRF_HIP(aligned_modes(modes, ws, s, &am));
    const GridWs w = grid_ws(&am, grid, GRF_DIRECT_F64, static_cast<char*>(ws) + rb);
    GRF_HIP(build_tables(&am, grid, GRF_DIRECT_F64, w, s));
    const double amp64 = modes->sigma * std::sqrt(2.0 / static_cast<double>(modes->n));
    GRF_HIP(launch_direct_grid_f64(static_cast<const double*>(w.t[0]), static_cast<const double*>(w.t[1]),
                                   static_cast<const double*>(w.t[2]), modes->w, modes->n, padded_modes(modes->n),
                                   grid->n, amp64, Epi{}, mu, nullptr, nullptr, nullptr, y64, k64,
                                   static_cast<double*>(w.partial), s));
    return GRF_OK;
}

int eval_field_points_ws_size(const grf_modes* modes, int64_t n_points, int method, size_t* bytes)
{
    int rc;
    if ((rc = check_modes(modes, "eval_field_points_ws_size"))) return rc;
    if (!bytes) return fail(GRF_EINVAL, "eval_field_points_ws_size: bytes is NULL");
    if (n_points < 0) return fail(GRF_EINVAL, "eval_field_points_ws_size: n_points < 0");
    if ((rc = check_points_method("eval_field_points_ws_size", &method, n_points))) return rc;
    *bytes = rot_ws_bytes(modes) + points_ws_bytes(modes->n, n_points, method);
    return GRF_OK;
}

int eval_field_points(const grf_modes* modes, const double* xyz, int64_t n_points, int method,
                      const grf_epi* epi, float* y, float* k, uint8_t* ind, void* ws, size_t ws_bytes,
                      void* stream)
{
    const char* fn = "eval_field_points";
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if (n_points < 0) return fail(GRF_EINVAL, "%s: n_points < 0", fn);
    if (n_points > (int64_t(1) << 40)) return fail(GRF_EINVAL, "%s: too many points", fn);
    if ((rc = check_points_method(fn, &method, n_points))) return rc;
    if ((rc = check_epi(epi, k, ind, fn))) return rc;
    if (n_points == 0) return GRF_OK;
    if (!y && !k && !ind) return fail(GRF_EINVAL, "%s: no output requested", fn);
    if (!xyz) return fail(GRF_EINVAL, "%s: xyz is NULL", fn);
    const size_t rb = rot_ws_bytes(modes);
    const size_t need = rb + points_ws_bytes(modes->n, n_points, method);
    if (!ws || ws_bytes < need) return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    grf_modes am;
    GRF_HIP(aligned_modes(modes, ws, s, &am));
    return points_launch(&am, xyz, n_points, method, make_epi(epi), y, k, ind, static_cast<char*>(ws) + rb, s);
}

}  // extern "C"

// ---------------------------------------------------------------- conditioning (kriging)
namespace grf {

constexpr int64_t kMaxObs = 65535 * 16;

static int make_krige_model(const grf_modes* m, const grf_krige* kp, const char* fn, KrigeModel* km)
{
    if (!kp) return fail(GRF_EINVAL, "%s: kriging parameters are NULL", fn);
    KrigeModel r{};
    if (kp->cov == GRF_COV_GAUSSIAN) r.kind = KR_GAUSS;
    else if (kp->cov == GRF_COV_EXPONENTIAL) r.kind = KR_EXP;
    else if (kp->cov == GRF_COV_MATERN) {
        if (std::fabs(kp->nu - 0.5) < 1e-12) r.kind = KR_EXP;
        else if (std::fabs(kp->nu - 1.5) < 1e-12) r.kind = KR_M32;
        else if (std::fabs(kp->nu - 2.5) < 1e-12) r.kind = KR_M52;
        else return fail(GRF_EUNSUPPORTED, "%s: Matern kriging needs nu = 1/2, 3/2 or 5/2 (got %g)", fn, kp->nu);
    } else {
        return fail(GRF_EINVAL, "%s: unknown covariance %d", fn, kp->cov);
    }
    if (!(kp->nugget >= 0.0) || !std::isfinite(kp->nugget)) return fail(GRF_EINVAL, "%s: nugget must be >= 0", fn);
    r.s2 = m->sigma * m->sigma;
    r.nugget_abs = kp->nugget * r.s2;
    // M^T with M = R diag(1/ell): (M^T)[b][a] = R[a][b] / ell_b
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            double v = 0.0;
            if (a < m->dim && b < m->dim) v = (m->rotated ? m->rot[3 * a + b] : (a == b ? 1.0 : 0.0)) / m->ell[b];
            r.mt[3 * b + a] = v;
        }
    *km = r;
    return GRF_OK;
}

static size_t krige_ws(const grf_modes* m, int64_t M)
{
    const size_t nblk = size_t((M + 63) / 64);
    return align256(sizeof(double) * size_t(M) * size_t(M)) + 2 * align256(sizeof(double) * size_t(M)) +
           align256(sizeof(float) * size_t(M)) + align256(sizeof(double) * nblk * 64 * 64) + rot_ws_bytes(m) +
           points_ws_bytes(m->n, M, GRF_DIRECT_F32);
}

}  // namespace grf

extern "C" {

int krige_weights_ws_size(const grf_modes* modes, int64_t n_obs, size_t* bytes)
{
    const char* fn = "krige_weights_ws_size";
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if (!bytes) return fail(GRF_EINVAL, "%s: bytes is NULL", fn);
    if (n_obs < 1 || n_obs > kMaxObs) return fail(GRF_EINVAL, "%s: n_obs must be in [1, %lld]", fn, (long long)kMaxObs);
    *bytes = krige_ws(modes, n_obs);
    return GRF_OK;
}

int krige_weights(const grf_modes* modes, const grf_krige* kp, const double* xobs, const float* dobs, int64_t n_obs,
                  double* alpha, int32_t* info, void* ws, size_t ws_bytes, void* stream)
{
    const char* fn = "krige_weights";
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    KrigeModel km;
    if ((rc = make_krige_model(modes, kp, fn, &km))) return rc;
    if (n_obs < 1 || n_obs > kMaxObs) return fail(GRF_EINVAL, "%s: n_obs must be in [1, %lld]", fn, (long long)kMaxObs);
    if (!xobs || !dobs || !alpha) return fail(GRF_EINVAL, "%s: xobs, dobs and alpha are required", fn);
    if (!(modes->sigma > 0.0)) return fail(GRF_EINVAL, "%s: sigma must be > 0", fn);
    const size_t need = krige_ws(modes, n_obs);
    if (!ws || ws_bytes < need) return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = n_obs;
    Carve c(ws);
    double* C = c.take<double>(size_t(M) * size_t(M));
    double* resid = c.take<double>(size_t(M));
    double* zf = c.take<double>(size_t(M));
    float* yu = c.take<float>(size_t(M));
    double* dinv = c.take<double>(size_t((M + 63) / 64) * 64 * 64);
    void* kbuf = c.base + c.used;
    c.used += rot_ws_bytes(modes);
    void* pws = c.base + c.used;
    if (info) GRF_HIP(launch_fill_i32(info, 0, s));
    grf_modes am;
    GRF_HIP(aligned_modes(modes, kbuf, s, &am));
    if ((rc = points_launch(&am, xobs, M, GRF_DIRECT_F32, Epi{}, yu, nullptr, nullptr, pws, s, false))) return rc;
    GRF_HIP(launch_residual(dobs, yu, M, resid, s));
    GRF_HIP(launch_cov_matrix(xobs, M, modes->dim, km, C, M, s));
    TimedScope timed(s);
    GRF_HIP(launch_cholesky(C, M, M, dinv, resid, zf, info, s));
    GRF_HIP(launch_chol_back(C, M, M, dinv, resid, zf, alpha, s));
    return GRF_OK;
}

int krige_apply_ws_size(int64_t n_obs, size_t* bytes)
{
    if (!bytes) return fail(GRF_EINVAL, "krige_apply_ws_size: bytes is NULL");
    if (n_obs < 1 || n_obs > kMaxObs) return fail(GRF_EINVAL, "krige_apply_ws_size: n_obs out of range");
    *bytes = align256(sizeof(float) * 4 * size_t(n_obs));
    return GRF_OK;
}

static int krige_apply(const char* fn, const grf_modes* modes, const grf_krige* kp, const double* xobs,
                       const double* alpha, int64_t n_obs, const KrigeTarget& tg, float* y, void* ws, size_t ws_bytes,
                       void* stream)
{
    int rc;
    KrigeModel km;
    if ((rc = make_krige_model(modes, kp, fn, &km))) return rc;
    if (n_obs < 1 || n_obs > kMaxObs) return fail(GRF_EINVAL, "%s: n_obs must be in [1, %lld]", fn, (long long)kMaxObs);
    if (!xobs || !alpha || !y) return fail(GRF_EINVAL, "%s: xobs, alpha and y are required", fn);
    const size_t need = align256(sizeof(float) * 4 * size_t(n_obs));
    if (!ws || ws_bytes < need) return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float4* staged = static_cast<float4*>(ws);
    GRF_HIP(launch_krige_stage(xobs, alpha, n_obs, modes->dim, km, staged, s));
    TimedScope timed(s);
    GRF_HIP(launch_krige_apply(staged, xobs, n_obs, km, tg, y, s));
    return GRF_OK;
}

int krige_apply_grid(const grf_modes* modes, const grf_krige* kp, const double* xobs, const double* alpha,
                     int64_t n_obs, const grf_grid* grid, float* y, void* ws, size_t ws_bytes, void* stream)
{
    const char* fn = "krige_apply_grid";
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if ((rc = check_grid(grid, modes->dim, fn))) return rc;
    KrigeTarget tg{};
    tg.grid = true;
    tg.dim = modes->dim;
    tg.count = grid->n[0] * grid->n[1] * grid->n[2];
    for (int a = 0; a < 3; ++a) {
        tg.n[a] = grid->n[a];
        tg.o[a] = grid->origin[a];
        tg.h[a] = grid->h[a];
    }
    return krige_apply(fn, modes, kp, xobs, alpha, n_obs, tg, y, ws, ws_bytes, stream);
}

int krige_apply_points(const grf_modes* modes, const grf_krige* kp, const double* xobs, const double* alpha,
                       int64_t n_obs, const double* xyz, int64_t n_points, float* y, void* ws, size_t ws_bytes,
                       void* stream)
{
    const char* fn = "krige_apply_points";
    int rc;
    if ((rc = check_modes(modes, fn))) return rc;
    if (n_points < 0 || n_points > (int64_t(1) << 40)) return fail(GRF_EINVAL, "%s: n_points out of range", fn);
    if (n_points == 0) return GRF_OK;
    if (!xyz) return fail(GRF_EINVAL, "%s: xyz is NULL", fn);
    KrigeTarget tg{};
    tg.grid = false;
    tg.dim = modes->dim;
    tg.count = n_points;
    tg.xyz = xyz;
    return krige_apply(fn, modes, kp, xobs, alpha, n_obs, tg, y, ws, ws_bytes, stream);
}

int epilogue_apply(const float* y, int64_t n, const grf_epi* epi, float* k, uint8_t* ind, void* stream)
{
    const char* fn = "epilogue_apply";
    if (n < 0) return fail(GRF_EINVAL, "%s: n < 0", fn);
    if (!epi) return fail(GRF_EINVAL, "%s: epi is NULL", fn);
    int rc;
    if ((rc = check_epi(epi, k, ind, fn))) return rc;
    if (n == 0) return GRF_OK;
    if (!k && !ind) return fail(GRF_EINVAL, "%s: no output requested", fn);
    if (!y) return fail(GRF_EINVAL, "%s: y is NULL", fn);
    TimedScope timed(static_cast<hipStream_t>(stream));
    GRF_HIP(launch_epilogue(y, n, make_epi(epi), k, ind, static_cast<hipStream_t>(stream)));
    return GRF_OK;
}

int field_backward_ws_size(const grf_modes* modes, int64_t n_points, size_t* bytes)
{
    int rc;
    if ((rc = check_modes(modes, "field_backward_ws_size"))) return rc;
    if (!bytes) return fail(GRF_EINVAL, "field_backward_ws_size: bytes is NULL");
    if (n_points < 0) return fail(GRF_EINVAL, "field_backward_ws_size: n_points < 0");
    const int64_t ldp = padded_modes(modes->n);
    const int64_t nch = bwd_chunks(n_points);
    *bytes = rot_ws_bytes(modes) + align256(sizeof(double) * 4 * ldp) + align256(sizeof(float) * 5 * ldp * nch) +
             align256(sizeof(float) * bwd_scal_floats(modes->n));
    return GRF_OK;
}

// The separable dense adjoint takes x in chunks of kBwdSepK cells (the K axis of one
// operand); each chunk's row-chunk sums get their own partial slots.
static bool bwd_sep_ok(const grf_grid* g) { return g->n[0] >= 1; }
static int64_t bwd_sep_xchunks(const grf_grid* g) { return (g->n[0] + kBwdSepK - 1) / kBwdSepK; }

static int64_t round_up32(int64_t v) { return (v + 31) / 32 * 32; }

// Rows of the separable adjoint's operand: y padded to a multiple of 32 per z-slice.
static int64_t bwd_sep_rows(const grf_grid* g) { return round_up32(g->n[1]) * g->n[2]; }

// Workspace of the separable path: mode parameters, partial sums, scalars, the operands and
// the y and z tables.
static size_t bwd_sep_ws(const grf_modes* m, const grf_grid* g)
{
    const int64_t ldp = padded_modes(m->n), qp = bwd_sep_rows(g);
    const int64_t nz = m->dim == 3 ? g->n[2] : 1;
    const int64_t nch = bwd_sep_chunks(ldp, qp) * bwd_sep_xchunks(g);
    return rot_ws_bytes(m) + align256(sizeof(double) * 4 * ldp) + align256(sizeof(float) * 5 * ldp * nch) +
           align256(sizeof(float) * bwd_scal_floats(m->n)) + 2 * align256(sizeof(uint16_t) * qp * kBwdSepK) +
           2 * align256(sizeof(uint16_t) * 4 * ldp * kBwdSepK) + align256(sizeof(float2) * round_up32(g->n[1]) * ldp) +
           align256(sizeof(float2) * nz * ldp);
}

static int backward_common(const char* fn, const grf_modes* modes, const double* xyz, const grf_grid* grid,
                           int64_t P, const float* grad_y, const float* y_saved, float* grad_phi,
                           float* grad_k, float* grad_sigma, float* grad_ell, void* ws, size_t ws_bytes,
                           void* stream, int method = GRF_AUTO)
{
    size_t need = 0;
    int rc = grid ? field_backward_grid_ws_size(modes, grid, &need) : field_backward_ws_size(modes, P, &need);
    if (rc) return rc;
    const bool sep = grid && method != GRF_DIRECT_F32 && bwd_sep_ok(grid);
    if (!grad_phi && !grad_k && !grad_sigma && !grad_ell) return fail(GRF_EINVAL, "%s: no output requested", fn);
    if (P > 0 && !grad_y) return fail(GRF_EINVAL, "%s: grad_y is NULL", fn);
    if (P > 0 && !xyz && !grid) return fail(GRF_EINVAL, "%s: xyz is NULL", fn);
    if (!ws || ws_bytes < need) return fail(GRF_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t ldp = padded_modes(modes->n);
    Carve c(ws);
    void* kbuf = c.base;
    c.used += rot_ws_bytes(modes);
    double* params = c.take<double>(4 * ldp);
    const int64_t qp = grid ? bwd_sep_rows(grid) : 0;
    const int64_t nch = sep ? bwd_sep_chunks(ldp, qp) * bwd_sep_xchunks(grid) : bwd_chunks(P);
    float* partial = c.take<float>(5 * ldp * nch);
    float* scal = c.take<float>(bwd_scal_floats(modes->n));
    grf_modes am;  // sums run on k itself; grad_ell maps back through the original table
    GRF_HIP(aligned_modes(modes, kbuf, s, &am));
    GRF_HIP(launch_mode_params(am.z, am.phi, am.dim, am.n, ldp, am.ell, params, s));
    GridWs tabs;
    BwdSep bs{};
    if (sep) {
        // bf16 hi + lo operands, then complex FP32 y and z tables (FP64 phases, psi in y)
        const int64_t nz = modes->dim == 3 ? grid->n[2] : 1;
        bs.ga_hi = c.take<uint16_t>(qp * kBwdSepK);
        bs.ga_lo = c.take<uint16_t>(qp * kBwdSepK);
        bs.ex_hi = c.take<uint16_t>(4 * ldp * kBwdSepK);
        bs.ex_lo = c.take<uint16_t>(4 * ldp * kBwdSepK);
        float2* ey = c.take<float2>(round_up32(grid->n[1]) * ldp);
        float2* ez = c.take<float2>(nz * ldp);
        AxisTableArgs d[2];
        for (int k = 0; k < 2; ++k) {
            const int a = k + 1;
            AxisTableArgs& t = d[k];
            t = AxisTableArgs{};
            t.z = a < am.dim ? am.z : nullptr;  // 2-D: no z axis, one row of zero phase
            t.phi = am.phi;
            t.n = am.n;
            t.ldp = ldp;
            t.axis = a;
            t.ell = a < am.dim ? am.ell[a] : 1.0;
            t.freq_scale = 1.0 / (6.283185307179586476925286766559 * t.ell);
            t.origin = grid->origin[a];
            t.h = grid->h[a];
            t.count = a == 1 ? round_up32(grid->n[1]) : nz;  // y rows up to the padded extent
            t.with_psi = a == 1;
            t.format = TF_CPLX_F32;
            t.out = a == 1 ? static_cast<void*>(ey) : static_cast<void*>(ez);
        }
        GRF_HIP(launch_axis_tables(d, 2, s));
        bs.ey = ey;
        bs.ez = ez;
        bs.zx = am.z;
        bs.fsx = 1.0 / (6.283185307179586476925286766559 * am.ell[0]);
        bs.ny = grid->n[1];
        bs.nyp = round_up32(grid->n[1]);
        bs.nz = nz;
        bs.qp = qp;
        bs.chunks = bwd_sep_chunks(ldp, qp);  // per x chunk
    } else if (grid) {  // per-axis FP32 revolution tables of the direct method
        tabs = grid_ws(&am, grid, GRF_DIRECT_F32, c.base + c.used);
        GRF_HIP(build_tables(&am, grid, GRF_DIRECT_F32, tabs, s));
    }
    BwdArgs a{};
    a.tx = static_cast<const float*>(tabs.t[0]);
    a.ty = static_cast<const float*>(tabs.t[1]);
    a.tz = static_cast<const float*>(tabs.t[2]);
    a.params = params;
    a.n = modes->n;
    a.ldp = ldp;
    a.dim = modes->dim;
    a.xyz = xyz;
    a.gn = grid ? grid->n : nullptr;
    a.go = grid ? grid->origin : nullptr;
    a.gh = grid ? grid->h : nullptr;
    a.P = P;
    a.gy = grad_y;
    a.ysaved = y_saved;
    a.amp = static_cast<float>(modes->sigma * std::sqrt(2.0 / static_cast<double>(modes->n)));
    a.sigma = static_cast<float>(modes->sigma);
    a.ell = modes->ell;
    a.z = modes->z;
    a.w = modes->w;
    a.rot = modes->rotated ? modes->rot : nullptr;
    a.gphi = grad_phi;
    a.gk = grad_k;
    a.gsigma = grad_sigma;
    a.gell = grad_ell;
    a.partial = partial;
    a.scal_partial = scal;
    a.nchunks = nch;
    a.sep = sep ? &bs : nullptr;
    GRF_HIP(launch_backward(a, s));
    return GRF_OK;
}

int field_backward(const grf_modes* modes, const double* xyz, int64_t n_points, const float* grad_y,
                   const float* y_saved, float* grad_phi, float* grad_k, float* grad_sigma, float* grad_ell,
                   void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_modes(modes, "field_backward");
    if (rc) return rc;
    if (n_points < 0) return fail(GRF_EINVAL, "field_backward: n_points < 0");
    if (modes->sigma <= 0.0 && grad_sigma) return fail(GRF_EINVAL, "field_backward: sigma must be > 0 for grad_sigma");
    return backward_common("field_backward", modes, xyz, nullptr, n_points, grad_y, y_saved, grad_phi, grad_k,
                           grad_sigma, grad_ell, ws, ws_bytes, stream);
}

int grad_z_from_k(const grf_modes* modes, const float* grad_k, float* grad_z, void* stream)
{
    int rc = check_modes(modes, "grad_z_from_k");
    if (rc) return rc;
    if (modes->n > 0 && (!grad_k || !grad_z)) return fail(GRF_EINVAL, "grad_z_from_k: grad_k and grad_z are required");
    if (modes->n > 0 && grad_k == grad_z) return fail(GRF_EINVAL, "grad_z_from_k: grad_z must not alias grad_k");
    GRF_HIP(launch_grad_z(grad_k, modes->dim, modes->n, modes->rotated ? modes->rot : nullptr, modes->ell, grad_z,
                          static_cast<hipStream_t>(stream)));
    return GRF_OK;
}

int field_backward_grid_ws_size(const grf_modes* modes, const grf_grid* grid, size_t* bytes)
{
    int rc;
    if ((rc = check_modes(modes, "field_backward_grid_ws_size"))) return rc;
    if ((rc = check_grid(grid, modes->dim, "field_backward_grid_ws_size"))) return rc;
    if ((rc = field_backward_ws_size(modes, grid->n[0] * grid->n[1] * grid->n[2], bytes))) return rc;
    *bytes += grid_ws(modes, grid, GRF_DIRECT_F32, nullptr).bytes;  // revolution tables
    if (bwd_sep_ok(grid)) *bytes = std::max(*bytes, bwd_sep_ws(modes, grid));  // either method fits
    return GRF_OK;
}

int field_backward_grid(const grf_modes* modes, const grf_grid* grid, const float* grad_y, const float* y_saved,
                        float* grad_phi, float* grad_k, float* grad_sigma, float* grad_ell, void* ws,
                        size_t ws_bytes, void* stream)
{
    int rc = check_modes(modes, "field_backward_grid");
    if (rc) return rc;
    if ((rc = check_grid(grid, modes->dim, "field_backward_grid"))) return rc;
    if (modes->sigma <= 0.0 && grad_sigma) return fail(GRF_EINVAL, "field_backward_grid: sigma must be > 0 for grad_sigma");
    return backward_common("field_backward_grid", modes, nullptr, grid, grid->n[0] * grid->n[1] * grid->n[2],
                           grad_y, y_saved, grad_phi, grad_k, grad_sigma, grad_ell, ws, ws_bytes, stream);
}

int field_backward_grid_method(const grf_modes* modes, const grf_grid* grid, int method, const float* grad_y,
                               const float* y_saved, float* grad_phi, float* grad_k, float* grad_sigma,
                               float* grad_ell, void* ws, size_t ws_bytes, void* stream)
{
    const char* fn = "field_backward_grid_method";
    int rc = check_modes(modes, fn);
    if (rc) return rc;
    if ((rc = check_grid(grid, modes->dim, fn))) return rc;
    if (method != GRF_AUTO && method != GRF_DIRECT_F32 && method != GRF_SEP_BF16_X3)
        return fail(GRF_EINVAL, "%s: method must be GRF_AUTO, GRF_DIRECT_F32 or GRF_SEP_BF16_X3", fn);
    if (modes->sigma <= 0.0 && grad_sigma) return fail(GRF_EINVAL, "%s: sigma must be > 0 for grad_sigma", fn);
    return backward_common(fn, modes, nullptr, grid, grid->n[0] * grid->n[1] * grid->n[2], grad_y, y_saved, grad_phi,
                           grad_k, grad_sigma, grad_ell, ws, ws_bytes, stream, method);
}

}  // extern "C"
