// eval_field_grid for callers that cannot allocate device memory (code under graph capture,
// tight serving loops): the workspace (per-axis tables, partial sums) lives in a fixed array
// of the library's own device memory instead of a caller's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "grf_internal.h"

namespace {

// The workspace of one grid evaluation.  Each device the library runs on holds its own copy
// until the process ends; every call on a device uses that copy.
static __device__ __align__(256) unsigned char scratch[GRF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device with that
// device current.  (On the host the array's name is only a stand-in for the symbol.)
int scratch_on_current_device(void** out, const char* fn)
{
    int dev = 0;
    GRF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return grf::fail(GRF_EUNSUPPORTED, "%s: device ordinal %d >= %d", fn, dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return grf::fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p) return grf::fail(GRF_EDEVICE, "%s: no device address for the scratch array", fn);
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return GRF_OK;
}

}  // namespace

extern "C" int eval_field_grid_noalloc(const grf_modes* modes, const grf_grid* grid, int method, const grf_epi* epi,
                                       float* y, float* k, uint8_t* ind, void* stream)
{
    const char* fn = "eval_field_grid_noalloc";
    size_t full = 0, need = 0;  // with the scratch below `full` the mode split is not taken
    int rc = grf::grid_ws_bytes(fn, modes, grid, method, &full, &need);
    if (rc) return rc;
    if (need > GRF_NOALLOC_SCRATCH_BYTES)
        return grf::fail(GRF_ENOMEM, "%s: this grid and method need %zu bytes of tables, above the fixed %zu-byte "
                         "scratch; use eval_field_grid with a workspace", fn, need,
                         static_cast<size_t>(GRF_NOALLOC_SCRATCH_BYTES));
    void* ws = nullptr;
    if ((rc = scratch_on_current_device(&ws, fn))) return rc;
    return grf::grid_eval(fn, modes, grid, method, -1, epi, y, k, ind, ws, GRF_NOALLOC_SCRATCH_BYTES, stream);
}
