// Allocation-free tracing entry point, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  The trace's scratch -- one counter record per 8x8 block
// and, for overlaps beyond the LDS slot size, the wide path's per-workgroup
// slots -- lives in one file-scope device array instead of buffers the scene
// allocates on demand.  The kernels are the ones st_trace launches.
#include <cstring>
#include <mutex>
#include <string>

#include "st_internal.h"

namespace {

// 32 MiB: counter records for up to 161,319 blocks of 8x8 pixels (a
// 3840x2160 frame has 129,600 at every tile size), the rest for wide-path
// slots.  Each GPU the library runs on holds its own copy until the process
// ends.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  The host-side name of the array is not a
// device address and is never passed to a kernel or a copy.
st_status scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return st::device_error(e, "trace_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        st::set_error("trace_noalloc: device index " + std::to_string(dev) + " above the supported 64 devices");
        return ST_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return st::device_error(e, "trace_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) {
            st::set_error("trace_noalloc: hipGetSymbolAddress returned NULL");
            return ST_E_DEVICE;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return ST_OK;
}

}  // namespace

extern "C" st_status st_trace_noalloc(st_scene* s, const st_camera* cam, float* out_depth, float* out_normal,
                                      st_stats* out_stats, void* stream_v) {
    using namespace st;
    if (!s || !cam || !out_depth || !out_normal) { set_error("trace_noalloc: NULL argument"); return ST_E_INVALID; }
    hipStream_t stream = (hipStream_t)stream_v;
    if (!s->ab_valid || std::memcmp(cam, &s->ab_cam, sizeof(st_camera)) != 0) {
        set_error("trace_noalloc: the A-buffer was not built for this camera");
        return ST_E_STALE;
    }
    void* base = nullptr;
    st_status r = scratch_ptr(&base);
    if (r != ST_OK) return r;
    const TraceScratch ext{base, kScratchBytes};
    r = trace_device(s, s->ab_tune, out_depth, out_normal, nullptr, stream, nullptr, out_stats != nullptr, &ext);
    if (r != ST_OK) return r;
    if (out_stats) {
        unsigned long long h[kStatCount];
        hipError_t e = hipMemcpyAsync(h, s->d_stats, sizeof(h), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return device_error(e, "trace_noalloc stats");
        stats_from_counters(s, h, out_stats);
    }
    return ST_OK;
}
