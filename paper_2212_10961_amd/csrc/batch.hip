// Batched ensembles of independent realisations on grids of uneven size.
//
// A plan turns a batch into three launches: a counter reset, one batched per-axis table
// build over every instance (the FP64 range reduction), and one persistent kernel whose
// blocks pull (instance, tile, slice) work items from an atomic counter.  The sequence is
// captured once in a hipGraph per batch signature and replayed afterwards.  For the
// separable methods each instance's tile shape (128x128 or 64x64) comes from its size
// class; with GRF_PLAN_AUTOTUNE the plan times both shapes on instances of each class the
// first time it meets the class and caches the winner (optionally in a text file).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "grf_internal.h"

using namespace grf;

struct grf_plan {
    int method = GRF_SEP_F16;
    int flags = 0;
    std::string cache_path;
    std::map<std::string, int> tuned;  // size-class key -> tile variant

    std::vector<uint64_t> sig;  // signature of the built batch
    bool built = false;
    bool d3 = false;
    int n_inst = 0;
    int n_desc = 0;
    int64_t total_items = 0;
    int64_t table_blocks = 0;
    int grid = 0;
    int32_t tile_m = 0, tile_n = 0;
    int32_t replayed = 0;

    void* d_tables = nullptr;
    size_t cap_tables = 0;
    void* d_items = nullptr;
    size_t cap_items = 0;
    AxisTableArgs* d_tdesc = nullptr;
    uint64_t* d_tblk = nullptr;  // per work block: (descriptor << 40) | local block
    size_t cap_tdesc = 0;
    GenModeDesc* d_gmd = nullptr;             // generated forms: per-instance mode-table descriptors
    size_t cap_gmd = 0;
    int64_t ldp_max = 0;
    unsigned long long* d_counter = nullptr;  // kMaxQueues counters, kQueueStride apart
    BatchQueue* d_queues = nullptr;           // in the same allocation, after the counters
    int nq = 1;

    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int size_bucket(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= v && b < 40) ++b;
    return b;
}

std::string class_key(int method, int64_t ldp, const grf_grid& g)
{
    std::ostringstream o;
    o << "sep method=" << method << " ldp=" << ldp << " bx=" << size_bucket(g.n[0]) << " by=" << size_bucket(g.n[1]);
    return o.str();
}

// Tile shape by size: 128x128 tiles once a slice spans several of them, else 64x64.
int default_variant(const grf_grid& g)
{
    return (g.n[0] >= 192 && g.n[1] >= 192) ? 0 : 1;
}

void load_cache(grf_plan* p)
{
    if (p->cache_path.empty()) return;
    std::ifstream f(p->cache_path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t at = line.rfind(' ');
        if (line.rfind("sep ", 0) != 0 || at == std::string::npos) continue;
        const int v = std::atoi(line.c_str() + at + 1);
        if (v == 0 || v == 1) p->tuned[line.substr(0, at)] = v;
    }
}

void save_cache_line(const grf_plan* p, const std::string& key, int v)
{
    if (p->cache_path.empty()) return;
    std::ofstream f(p->cache_path, std::ios::app);
    if (f) f << key << ' ' << v << '\n';
}

template <class T>
hipError_t ensure(T*& ptr, size_t& cap, size_t bytes)
{
    if (bytes <= cap && ptr) return hipSuccess;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes > 0 ? bytes : 256);
    if (e != hipSuccess) return e;
    ptr = static_cast<T*>(q);
    cap = bytes;
    return hipSuccess;
}

void push_bits(std::vector<uint64_t>& s, double d)
{
    uint64_t u;
    std::memcpy(&u, &d, sizeof(u));
    s.push_back(u);
}

std::vector<uint64_t> signature(const grf_plan* p, const grf_batch_item* items, int32_t n)
{
    std::vector<uint64_t> s;
    s.reserve(static_cast<size_t>(n) * 26 + 2);
    s.push_back(static_cast<uint64_t>(p->method));
    s.push_back(static_cast<uint64_t>(n));
    for (int32_t i = 0; i < n; ++i) {
        const grf_batch_item& it = items[i];
        s.push_back(static_cast<uint64_t>(it.modes.dim));
        s.push_back(static_cast<uint64_t>(it.modes.n));
        s.push_back(reinterpret_cast<uint64_t>(it.modes.z));
        s.push_back(reinterpret_cast<uint64_t>(it.modes.phi));
        push_bits(s, it.modes.sigma);
        for (int a = 0; a < 3; ++a) {
            push_bits(s, it.modes.ell[a]);
            s.push_back(static_cast<uint64_t>(it.grid.n[a]));
            push_bits(s, it.grid.origin[a]);
            push_bits(s, it.grid.h[a]);
        }
        s.push_back(reinterpret_cast<uint64_t>(it.modes.w));
        s.push_back(static_cast<uint64_t>(it.modes.rotated));
        s.push_back(reinterpret_cast<uint64_t>(it.y));
        s.push_back(reinterpret_cast<uint64_t>(it.k));
        s.push_back(reinterpret_cast<uint64_t>(it.ind));
        // the epilogue is baked into the captured descriptors: every field that enters it
        uint32_t mu;
        std::memcpy(&mu, &it.epi.mu, sizeof(mu));
        s.push_back((static_cast<uint64_t>(static_cast<uint32_t>(it.epi.n_thresholds)) << 32) | mu);
        for (int q = 0; q < it.epi.n_thresholds && q < GRF_MAX_THRESHOLDS; ++q) {
            uint32_t t;
            std::memcpy(&t, &it.epi.thresholds[q], sizeof(t));
            s.push_back(t);
        }
    }
    return s;
}

void destroy_graph(grf_plan* p)
{
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// The three launches of one batch evaluation.
hipError_t enqueue(grf_plan* p, hipStream_t s, const void* items, int n_items_desc, int64_t total)
{
    const bool sep = is_sep(p->method);
    hipError_t e = launch_fill_u64(p->d_counter, 0ull, sep ? p->nq : 1, kQueueStride, s);
    if (e != hipSuccess) return e;
    if (p->table_blocks > 0) {
        e = launch_axis_tables_batched(p->d_tdesc, p->d_tblk, p->table_blocks, s);
        if (e != hipSuccess) return e;
    }
    if (p->d_gmd && p->ldp_max > 0) {
        e = launch_gen_modes(p->d_gmd, p->n_inst, p->ldp_max, s);
        if (e != hipSuccess) return e;
    }
    if (sep)
        return launch_sep_batch(p->method, p->d3, static_cast<const SepBatchItem*>(items), n_items_desc, p->d_queues,
                                p->nq, p->d_counter, p->grid, s);
    return launch_direct_batch(static_cast<const DirectBatchItem*>(items), n_items_desc, total, p->d_counter, p->grid,
                               s);
}

constexpr size_t kCounterBytes = sizeof(unsigned long long) * kQueueStride * kMaxQueues;

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

}  // namespace

// Build descriptors, tables layout, tuning and (optionally) the graph for a new signature.
static int build_plan(grf_plan* p, const grf_batch_item* items, int32_t n, hipStream_t s)
{
    const char* fn = "eval_field_batch";
    GRF_HIP(hipStreamSynchronize(s));  // buffers below may still be in use by earlier calls
    if (p->cap) GRF_HIP(hipStreamSynchronize(p->cap));
    destroy_graph(p);
    p->built = false;

    const bool sep = is_sep(p->method);
    p->d3 = items[0].modes.dim == 3;
    const bool gen = sep && sep_batch_generates(p->method, p->d3);  // operands made on chip

    // ---- table layout and descriptors (same tables as eval_field_grid would build); for the
    // generated forms, each instance's local x table and mode table instead
    std::vector<GridWs> ws(n);
    std::vector<size_t> toff(n);
    size_t tbytes = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t ldp = padded_modes(items[i].modes.n);
        toff[i] = tbytes;
        if (gen) {
            tbytes += align256(sizeof(uint32_t) * size_t(kGenRows) * size_t(ldp)) + align256(sizeof(GenMode) * size_t(ldp));
        } else {
            ws[i] = grid_ws(&items[i].modes, &items[i].grid, p->method, nullptr);
            tbytes += ws[i].bytes - ws[i].split_bytes;  // tables only: batch tiles do not split the modes
        }
    }
    GRF_HIP(ensure(p->d_tables, p->cap_tables, tbytes));
    std::vector<AxisTableArgs> td;
    std::vector<uint64_t> blk;
    std::vector<GenModeDesc> gmd;
    std::vector<const uint32_t*> rx_of(n);
    std::vector<const GenMode*> md_of(n);
    p->ldp_max = 0;
    if (gen) {
        int64_t total = 0;
        for (int32_t i = 0; i < n; ++i) {
            const grf_modes& m = items[i].modes;
            const grf_grid& gr = items[i].grid;
            const int64_t ldp = padded_modes(m.n);
            char* base = static_cast<char*>(p->d_tables) + toff[i];
            AxisTableArgs t{};
            t.z = m.z;
            t.phi = m.phi;
            t.n = m.n;
            t.ldp = ldp;
            t.axis = 0;
            t.ell = m.ell[0];
            t.freq_scale = 1.0 / (6.283185307179586476925286766559 * m.ell[0]);
            t.origin = -0.5 * gr.h[0];  // entry r at x = r hx: R_j(r) = e^{2 pi i a_x r hx}
            t.h = gr.h[0];
            t.count = kGenRows;
            t.with_psi = false;
            t.conj = true;
            t.fast_trig = true;  // one fp16/bf16 rounding of the operand
            t.blocked = true;
            t.format = is_bf16(p->method) ? TF_BF16 : TF_F16;
            t.out = base;
            t.out_lo = nullptr;
            t.w = nullptr;
            rx_of[i] = static_cast<const uint32_t*>(t.out);
            td.push_back(t);
            total += axis_table_blocks(t);
            GenModeDesc g{};
            g.z = m.z;
            g.phi = m.phi;
            g.w = m.w;
            g.n = m.n;
            g.ldp = ldp;
            g.fsx = t.freq_scale;
            g.fsy = 1.0 / (6.283185307179586476925286766559 * m.ell[1]);
            g.ox = gr.origin[0];
            g.oy = gr.origin[1];
            g.hx = gr.h[0];
            g.hy = gr.h[1];
            g.out = reinterpret_cast<GenMode*>(base + align256(sizeof(uint32_t) * size_t(kGenRows) * size_t(ldp)));
            md_of[i] = g.out;
            gmd.push_back(g);
            p->ldp_max = std::max(p->ldp_max, ldp);
        }
        if (total > 0x7fffffff) return fail(GRF_EINVAL, "%s: batch tables too large for one launch", fn);
        for (size_t di = 0; di < td.size(); ++di) {
            const int64_t nb = axis_table_blocks(td[di]);
            for (int64_t w = 0; w < nb; ++w) blk.push_back((static_cast<uint64_t>(di) << 40) | static_cast<uint64_t>(w));
        }
        GRF_HIP(ensure(p->d_gmd, p->cap_gmd, gmd.size() * sizeof(GenModeDesc)));
        GRF_HIP(hipMemcpy(p->d_gmd, gmd.data(), gmd.size() * sizeof(GenModeDesc), hipMemcpyHostToDevice));
    }
    if (!gen) {
        int64_t total = 0;
        for (int32_t i = 0; i < n; ++i) {
            AxisTableArgs d[3];
            const int nd = grid_table_descs(&items[i].modes, &items[i].grid, p->method, ws[i], d);
            for (int k = 0; k < nd; ++k) total += axis_table_blocks(d[k]);
        }
        if (total > 0x7fffffff) return fail(GRF_EINVAL, "%s: batch tables too large for one launch", fn);
        blk.reserve(static_cast<size_t>(total));
        for (int32_t i = 0; i < n; ++i) {
            ws[i] = grid_ws(&items[i].modes, &items[i].grid, p->method, static_cast<char*>(p->d_tables) + toff[i]);
            AxisTableArgs d[3];
            const int nd2 = grid_table_descs(&items[i].modes, &items[i].grid, p->method, ws[i], d);
            for (int k = 0; k < nd2; ++k) {
                const uint64_t di = td.size();
                td.push_back(d[k]);
                const int64_t nb = axis_table_blocks(d[k]);
                for (int64_t w = 0; w < nb; ++w) blk.push_back((di << 40) | static_cast<uint64_t>(w));
            }
        }
    }
    if (td.size() >= (size_t(1) << 23)) return fail(GRF_EINVAL, "%s: too many tables in one batch", fn);
    p->n_desc = static_cast<int>(td.size());
    p->table_blocks = static_cast<int64_t>(blk.size());
    GRF_HIP(ensure(p->d_tdesc, p->cap_tdesc, align256(td.size() * sizeof(AxisTableArgs)) + blk.size() * sizeof(uint64_t)));
    p->d_tblk = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(p->d_tdesc) +
                                            align256(td.size() * sizeof(AxisTableArgs)));
    if (!td.empty()) {
        GRF_HIP(hipMemcpy(p->d_tdesc, td.data(), td.size() * sizeof(AxisTableArgs), hipMemcpyHostToDevice));
        GRF_HIP(hipMemcpy(p->d_tblk, blk.data(), blk.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    }
    if (!p->d_counter) {
        void* q = nullptr;
        GRF_HIP(hipMalloc(&q, kCounterBytes + kMaxQueues * sizeof(BatchQueue)));
        p->d_counter = static_cast<unsigned long long*>(q);
        p->d_queues = reinterpret_cast<BatchQueue*>(static_cast<char*>(q) + kCounterBytes);
    }
    if (!p->cap) GRF_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));

    const int cus = device_cus();
    p->grid = cus * (sep ? sep_batch_blocks_per_cu(p->method, p->d3) : direct_batch_blocks_per_cu());

    if (!sep) {
        std::vector<int32_t> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return items[a].grid.n[0] * items[a].grid.n[1] * items[a].grid.n[2] >
                   items[b].grid.n[0] * items[b].grid.n[1] * items[b].grid.n[2];
        });
        std::vector<DirectBatchItem> di(n);
        int64_t item = 0;
        for (int32_t r = 0; r < n; ++r) {
            const int32_t i = order[r];
            const grf_batch_item& it = items[i];
            DirectBatchItem& d = di[r];
            d.tx = static_cast<const float*>(ws[i].t[0]);
            d.ty = static_cast<const float*>(ws[i].t[1]);
            d.tz = static_cast<const float*>(ws[i].t[2]);
            d.w = it.modes.w;
            d.y = it.y;
            d.k = it.k;
            d.ind = it.ind;
            d.epi = make_epi(&it.epi);
            d.ldp = padded_modes(it.modes.n);
            d.nq = it.grid.n[1] * it.grid.n[2];
            d.n = static_cast<int32_t>(it.modes.n);
            d.nx = static_cast<int32_t>(it.grid.n[0]);
            d.ny = static_cast<int32_t>(it.grid.n[1]);
            d.nxt = static_cast<int32_t>((it.grid.n[0] + kDirectTile - 1) / kDirectTile);
            d.amp = static_cast<float>(it.modes.sigma * std::sqrt(2.0 / static_cast<double>(it.modes.n)));
            d.item0 = item;
            item += static_cast<int64_t>(d.nxt) * ((d.nq + kDirectTile - 1) / kDirectTile);
        }
        p->total_items = item;
        GRF_HIP(ensure(p->d_items, p->cap_items, di.size() * sizeof(DirectBatchItem)));
        GRF_HIP(hipMemcpy(p->d_items, di.data(), di.size() * sizeof(DirectBatchItem), hipMemcpyHostToDevice));
        p->tile_m = p->tile_n = kDirectTile;
    } else {
        // ---- per-instance SepArgs and tile variant
        std::vector<SepBatchItem> si(n);
        std::vector<std::string> keys(n);
        for (int32_t i = 0; i < n; ++i) {
            const grf_batch_item& it = items[i];
            SepArgs& a = si[i].a;
            a = SepArgs{};
            a.method = p->method;
            a.n = it.modes.n;
            a.ldp = padded_modes(it.modes.n);
            a.nx = it.grid.n[0];
            a.ny = it.grid.n[1];
            a.nz = it.grid.n[2];
            a.px = ws[i].t[0];
            a.px_lo = ws[i].tlo[0];
            a.qy = ws[i].t[1];
            a.qy_lo = ws[i].tlo[1];
            a.ez = p->d3 ? static_cast<const float2*>(ws[i].t[2]) : nullptr;
            a.amp = static_cast<float>(it.modes.sigma * std::sqrt(2.0 / static_cast<double>(it.modes.n)));
            a.epi = make_epi(&it.epi);
            a.y = it.y;
            a.k = it.k;
            a.ind = it.ind;
            a.tile = -1;
            GenArgs& g = si[i].g;
            g = GenArgs{};
            if (gen) {
                g.rx = rx_of[i];
                g.md = md_of[i];
                g.hx = it.grid.h[0];
                g.hy = it.grid.h[1];
            }
            keys[i] = class_key(p->method, a.ldp, it.grid);
            auto f = p->tuned.find(keys[i]);
            si[i].variant = f != p->tuned.end() ? f->second : default_variant(it.grid);
        }
        auto tiles_of = [&](SepBatchItem& b) {
            const int t = b.variant == 0 ? 128 : 64;
            b.tiles_x = static_cast<int32_t>((b.a.nx + t - 1) / t);
            b.tiles_y = static_cast<int32_t>((b.a.ny + t - 1) / t);
            return static_cast<int64_t>(b.tiles_x) * b.tiles_y * b.a.nz;
        };

        // ---- autotune classes not seen before: time both tile shapes on up to 16 instances
        const bool tune = (p->flags & GRF_PLAN_AUTOTUNE) != 0;
        std::vector<std::string> pending;
        if (tune)
            for (int32_t i = 0; i < n; ++i)
                if (!p->tuned.count(keys[i]) && std::find(pending.begin(), pending.end(), keys[i]) == pending.end())
                    pending.push_back(keys[i]);
        if (!pending.empty()) {
            if (p->table_blocks > 0)
                GRF_HIP(launch_axis_tables_batched(p->d_tdesc, p->d_tblk, p->table_blocks, p->cap));
            if (gen) GRF_HIP(launch_gen_modes(p->d_gmd, n, p->ldp_max, p->cap));
            hipEvent_t e0, e1;
            GRF_HIP(hipEventCreate(&e0));
            GRF_HIP(hipEventCreate(&e1));
            for (const std::string& key : pending) {
                // Up to 16 instances of the class, repeated until even the larger tile gives
                // every resident block several work items: the comparison is then one of
                // throughput on a full device, as in the real batch.
                std::vector<SepBatchItem> cls;
                for (int32_t i = 0; i < n && cls.size() < 16; ++i)
                    if (keys[i] == key) cls.push_back(si[i]);
                std::vector<SepBatchItem> sub;
                int64_t big_tiles = 0;
                while (big_tiles < 4 * int64_t(p->grid) && sub.size() < 8192) {
                    for (const SepBatchItem& b : cls) {
                        sub.push_back(b);
                        big_tiles += ((b.a.nx + 127) / 128) * ((b.a.ny + 127) / 128) * b.a.nz;
                    }
                }
                float best = 1e30f;
                int bestv = 0;
                for (int v = 0; v < 2; ++v) {
                    int64_t item = 0;
                    for (auto& b : sub) {
                        b.variant = v;
                        b.item0 = item;
                        item += tiles_of(b);
                    }
                    GRF_HIP(ensure(p->d_items, p->cap_items, sub.size() * sizeof(SepBatchItem)));
                    GRF_HIP(hipMemcpy(p->d_items, sub.data(), sub.size() * sizeof(SepBatchItem), hipMemcpyHostToDevice));
                    const BatchQueue one{0, item};
                    GRF_HIP(hipMemcpy(p->d_queues, &one, sizeof(one), hipMemcpyHostToDevice));
                    float tot = 0.f;
                    for (int rep = 0; rep < 3; ++rep) {
                        GRF_HIP(launch_fill_u64(p->d_counter, 0ull, 1, kQueueStride, p->cap));
                        GRF_HIP(hipEventRecord(e0, p->cap));
                        GRF_HIP(launch_sep_batch(p->method, p->d3, static_cast<const SepBatchItem*>(p->d_items),
                                                 static_cast<int>(sub.size()), p->d_queues, 1, p->d_counter, p->grid,
                                                 p->cap));
                        GRF_HIP(hipEventRecord(e1, p->cap));
                        GRF_HIP(hipEventSynchronize(e1));
                        float ms = 0.f;
                        GRF_HIP(hipEventElapsedTime(&ms, e0, e1));
                        if (rep > 0) tot += ms;  // first run warms up
                    }
                    if (tot < best) {
                        best = tot;
                        bestv = v;
                    }
                }
                p->tuned[key] = bestv;
                save_cache_line(p, key, bestv);
            }
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            for (int32_t i = 0; i < n; ++i) si[i].variant = p->tuned[keys[i]];
        }

        // ---- queues: instances spread over the XCD queues by longest-processing-time-first
        // (cost in 64x64-tile units), then within a queue larger tiles first, then larger
        // instances; item0 runs over queue 0's instances, then queue 1's, ...
        std::vector<int64_t> cost(n);
        for (int32_t i = 0; i < n; ++i) cost[i] = tiles_of(si[i]) * (si[i].variant == 0 ? 4 : 1);
        std::vector<int32_t> by_cost(n);
        std::iota(by_cost.begin(), by_cost.end(), 0);
        std::stable_sort(by_cost.begin(), by_cost.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
        p->nq = kMaxQueues;
        std::vector<int64_t> load(p->nq, 0);
        std::vector<std::vector<int32_t>> members(p->nq);
        for (const int32_t i : by_cost) {
            const int g = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
            members[g].push_back(i);
            load[g] += cost[i];
        }
        std::vector<SepBatchItem> sorted;
        sorted.reserve(n);
        std::vector<BatchQueue> queues(p->nq);
        int64_t item = 0, big = 0;
        for (int g = 0; g < p->nq; ++g) {
            std::vector<int32_t>& order = members[g];
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                if (si[a].variant != si[b].variant) return si[a].variant < si[b].variant;
                return si[a].a.nx * si[a].a.ny * si[a].a.nz > si[b].a.nx * si[b].a.ny * si[b].a.nz;
            });
            queues[g].start = item;
            for (const int32_t i : order) {
                SepBatchItem b = si[i];
                b.item0 = item;
                const int64_t t = tiles_of(b);
                item += t;
                if (b.variant == 0) big += t * 4;  // in 64x64-tile units
                else big -= t;
                sorted.push_back(b);
            }
            queues[g].count = item - queues[g].start;
        }
        p->total_items = item;
        GRF_HIP(ensure(p->d_items, p->cap_items, sorted.size() * sizeof(SepBatchItem)));
        GRF_HIP(hipMemcpy(p->d_items, sorted.data(), sorted.size() * sizeof(SepBatchItem), hipMemcpyHostToDevice));
        GRF_HIP(hipMemcpy(p->d_queues, queues.data(), queues.size() * sizeof(BatchQueue), hipMemcpyHostToDevice));
        p->tile_m = p->tile_n = big >= 0 ? 128 : 64;
    }
    p->n_inst = n;

    if (p->flags & GRF_PLAN_GRAPH) {
        GRF_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
        hipError_t e = enqueue(p, p->cap, p->d_items, p->n_inst, p->total_items);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(p->cap, &g);
        if (e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return fail_hip(e, "eval_field_batch: capture");
        }
        if (e2 != hipSuccess) return fail_hip(e2, "hipStreamEndCapture");
        p->graph = g;
        GRF_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    p->built = true;
    return GRF_OK;
}

extern "C" {

int grf_plan_create(grf_plan** plan, int method, int flags, const char* tune_cache_path)
{
    if (!plan) return fail(GRF_EINVAL, "grf_plan_create: plan is NULL");
    *plan = nullptr;
    if (method == GRF_AUTO) method = GRF_SEP_F16;
    if (method != GRF_DIRECT_F32 && !is_sep(method))
        return fail(GRF_EINVAL, "grf_plan_create: method must be GRF_DIRECT_F32 or a separable method (got %d)", method);
    if (flags & ~(GRF_PLAN_GRAPH | GRF_PLAN_AUTOTUNE)) return fail(GRF_EINVAL, "grf_plan_create: unknown flags");
    grf_plan* p = new (std::nothrow) grf_plan();
    if (!p) return fail(GRF_ENOMEM, "grf_plan_create: out of host memory");
    p->method = method;
    p->flags = flags;
    if (tune_cache_path) p->cache_path = tune_cache_path;
    load_cache(p);
    *plan = p;
    return GRF_OK;
}

int grf_plan_destroy(grf_plan* p)
{
    if (!p) return GRF_OK;
    const bool touched = p->cap || p->d_tables || p->d_items || p->d_tdesc || p->d_counter || p->d_gmd;
    if (touched) {
        // Launches of this plan may still be queued on the caller's streams.
        if (p->cap) hipStreamSynchronize(p->cap);
        hipDeviceSynchronize();
    }
    destroy_graph(p);
    if (p->d_tables) hipFree(p->d_tables);
    if (p->d_items) hipFree(p->d_items);
    if (p->d_tdesc) hipFree(p->d_tdesc);
    if (p->d_counter) hipFree(p->d_counter);
    if (p->d_gmd) hipFree(p->d_gmd);
    if (p->cap) hipStreamDestroy(p->cap);
    delete p;
    return GRF_OK;
}

int eval_field_batch(grf_plan* p, const grf_batch_item* items, int32_t n, void* stream)
{
    const char* fn = "eval_field_batch";
    if (!p) return fail(GRF_EINVAL, "%s: plan is NULL", fn);
    if (n < 0) return fail(GRF_EINVAL, "%s: n < 0", fn);
    if (n == 0) return GRF_OK;
    if (!items) return fail(GRF_EINVAL, "%s: items is NULL", fn);
    for (int32_t i = 0; i < n; ++i) {
        int rc;
        if ((rc = check_modes(&items[i].modes, fn))) return rc;
        if ((rc = check_grid(&items[i].grid, items[i].modes.dim, fn))) return rc;
        if (!items[i].y && !items[i].k && !items[i].ind) return fail(GRF_EINVAL, "%s: item %d has no output", fn, i);
        if ((rc = check_epi(&items[i].epi, items[i].k, items[i].ind, fn))) return rc;
        if (items[i].modes.rotated)
            return fail(GRF_EUNSUPPORTED, "%s: item %d: rotated tables are not batched (pass k = rot diag(1/ell) z "
                        "as an axis-aligned table with ell = 1)", fn, i);
        if (is_sep(p->method) && items[i].modes.dim != items[0].modes.dim)
            return fail(GRF_EUNSUPPORTED, "%s: separable batches must not mix 2-D and 3-D grids", fn);
        if (items[i].grid.n[0] > 0x7fffffff || items[i].grid.n[1] > 0x7fffffff)
            return fail(GRF_EINVAL, "%s: grid side too large", fn);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uint64_t> sig = signature(p, items, n);
    p->replayed = 0;
    if (!p->built || sig != p->sig) {
        int rc = build_plan(p, items, n, s);
        if (rc) {
            p->sig.clear();
            return rc;
        }
        p->sig = std::move(sig);
    } else {
        p->replayed = (p->flags & GRF_PLAN_GRAPH) ? 1 : 0;
    }
    TimedScope timed(s);
    if (p->flags & GRF_PLAN_GRAPH) {
        GRF_HIP(hipGraphLaunch(p->exec, s));
    } else {
        GRF_HIP(enqueue(p, s, p->d_items, p->n_inst, p->total_items));
    }
    return GRF_OK;
}

int grf_plan_info(const grf_plan* p, int32_t* tile_m, int32_t* tile_n, int32_t* replayed, int64_t* work_items)
{
    if (!p) return fail(GRF_EINVAL, "grf_plan_info: plan is NULL");
    if (tile_m) *tile_m = p->tile_m;
    if (tile_n) *tile_n = p->tile_n;
    if (replayed) *replayed = p->replayed;
    if (work_items) *work_items = p->total_items;
    return GRF_OK;
}

}  // extern "C"
