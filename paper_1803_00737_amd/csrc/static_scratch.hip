// Static device scratch for the entry points that allocate nothing
// (dwt_fuse_backward_noalloc).  The array lives in this library's code
// object, so each GPU that loads the library holds its own copy, at its own
// address, until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): it asks
// the runtime for the device address once per device and uses that.
#include <mutex>

#include "fuse_internal.h"

namespace dwtf {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_address(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *ptr = g_addr[device];
    return hipSuccess;
}

}  // namespace dwtf
