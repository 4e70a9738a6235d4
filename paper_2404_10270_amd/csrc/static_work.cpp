// static_work.cpp -- pic_init_static: a context whose workspace is a
// file-scope device array of the library instead of a caller buffer, for
// callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pic.h"
#include "pic_internal.h"

// The workspace of pic_init_static contexts: one copy on each GPU the library
// runs on, at its own device address.  Host code never uses this name as an
// address (it only stands in for the symbol); it uses the per-device pointer
// that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[PIC_STATIC_WORK_MAX];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices];   // device address of `scratch` on each device, once looked up
bool g_held[kMaxDevices];   // a live pic_init_static context uses that device's array

}  // namespace

namespace picx {

void static_release(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (device >= 0 && device < kMaxDevices) g_held[device] = false;
}

}  // namespace picx

extern "C" int pic_init_static(const pic_config *cfgs, int n_inst, const pic_buffers *bufs,
                               void *stream, unsigned flags, pic_ctx **out)
{
    if (!out) return PIC_E_ARG;
    *out = nullptr;
    if (!bufs || bufs->work) return PIC_E_ARG;
    int rc = 0;
    const uint64_t bytes = picx::work_bytes_of(cfgs, n_inst, &rc);
    if (rc) return rc;
    if (bytes > PIC_STATIC_WORK_MAX) return PIC_E_SCRATCH;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PIC_E_DEVICE;
    void *W = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_held[dev]) return PIC_E_BUSY;
        if (!g_ptr[dev]) {
            // first use on this device (current): its own copy of the array
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
                return PIC_E_DEVICE;
            g_ptr[dev] = p;
        }
        g_held[dev] = true;
        W = g_ptr[dev];
    }
    rc = picx::init_context(cfgs, n_inst, bufs, W, stream, flags, false, out);
    if (rc) {
        picx::static_release(dev);
        return rc;
    }
    picx::mark_static(*out, dev);
    return PIC_OK;
}
