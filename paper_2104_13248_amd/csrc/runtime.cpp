// Error reporting, pinned staging of host inputs and stream-ordered scratch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace fdk {

namespace {
thread_local std::string t_last_error;

// Pinned host buffers used to stage small host inputs (matrices, ellipsoid
// tables) for asynchronous copies.  A buffer is reused once the event
// recorded after its copy has completed.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    int device = -1;
};
std::mutex g_stage_mu;
std::vector<Staging> g_stage;
}  // namespace

void set_error(const std::string& msg) { t_last_error = msg; }

fdk_status fail(fdk_status code, const std::string& msg)
{
    t_last_error = msg;
    return code;
}

fdk_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(FDK_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return FDK_OK;
}

fdk_status device_alloc_async(size_t bytes, void* stream, void** dev)
{
    hipError_t e = hipMallocAsync(dev, bytes ? bytes : 1, (hipStream_t)stream);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return fail(FDK_E_NOMEM, "device allocation of scratch failed");
    }
    if (e != hipSuccess) return fail(FDK_E_DEVICE, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    return FDK_OK;
}

fdk_status device_free_async(void* dev, void* stream)
{
    if (!dev) return FDK_OK;
    hipError_t e = hipFreeAsync(dev, (hipStream_t)stream);
    if (e != hipSuccess) return fail(FDK_E_DEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(e));
    return FDK_OK;
}

fdk_status upload_async(const void* host, size_t bytes, void* stream, void** dev)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(FDK_E_DEVICE, "hipGetDevice failed");
    fdk_status st = device_alloc_async(bytes, stream, dev);
    if (st != FDK_OK) return st;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging* slot = nullptr;
    for (auto& b : g_stage) {
        if (b.device != device || b.cap < bytes) continue;
        if (hipEventQuery(b.done) == hipSuccess) { slot = &b; break; }
    }
    if (!slot) {
        Staging b;
        b.device = device;
        b.cap = bytes < 4096 ? 4096 : bytes;
        if (hipHostMalloc(&b.host, b.cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            device_free_async(*dev, stream);
            return fail(FDK_E_NOMEM, "pinned host allocation failed");
        }
        if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
            hipHostFree(b.host);
            device_free_async(*dev, stream);
            return fail(FDK_E_DEVICE, "hipEventCreate failed");
        }
        g_stage.push_back(b);
        slot = &g_stage.back();
    }
    std::memcpy(slot->host, host, bytes);
    hipError_t e = hipMemcpyAsync(*dev, slot->host, bytes, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(slot->done, (hipStream_t)stream);
    if (e != hipSuccess) {
        device_free_async(*dev, stream);
        return fail(FDK_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    return FDK_OK;
}

}  // namespace fdk

extern "C" const char* fdk_last_error(void) { return fdk::t_last_error.c_str(); }

extern "C" const char* fdk_status_string(int32_t s)
{
    switch (s) {
        case FDK_OK: return "ok";
        case FDK_E_INVALID: return "invalid argument";
        case FDK_E_GEOMETRY: return "unsupported or invalid geometry";
        case FDK_E_UNSUPPORTED: return "unsupported request";
        case FDK_E_DEVICE: return "device error";
        case FDK_E_NOMEM: return "out of memory";
    }
    return "unknown status";
}
