// Fixed device scratch of the allocation-free GAP entry point
// (sci_gap_tv_noalloc): a file-scope device array, one copy per GPU the
// library runs on, held until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: in host
// code that name is a stand-in, not a device address. Its device address is
// looked up once per device (with that device current) by
// hipGetSymbolAddress, and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sci_internal.h"

namespace sci {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_addr[kMaxDevices] = {};

} // namespace

int noalloc_scratch_lookup(int device, void **addr)
{
    *addr = nullptr;
    if (device < 0 || device >= kMaxDevices) return SCI_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_addr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return SCI_ERR_HIP; // caller made it current
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SCI_ERR_HIP;
        g_addr[device] = p;
    }
    *addr = g_addr[device];
    return SCI_OK;
}

} // namespace sci
