// Fixed device scratch of the no-allocation interface solve
// (mesh_sdd_solve_interfaces_noalloc): one static device array per GPU the
// library runs on, resolved to its device address once per device.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// only way host code here uses it is hipGetSymbolAddress, and every buffer
// handed to a kernel or a copy is carved from the address that call returns.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "runtime_internal.hpp"

namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;   // the stated maximum: 64 MiB per device
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace msdd_rt {

namespace {
struct ScratchSlot {
    bool resolved = false;
    void *ptr = nullptr;
    hipError_t err = hipSuccess;
    std::mutex use;   // held by a no-allocation solve while it uses the array
};
std::mutex g_resolve_mu;
ScratchSlot g_slots[kMaxDevices];
}  // namespace

size_t scratch_capacity() { return kScratchBytes; }

// Resolve the array's address on `device`, which the caller has made
// current (the context's set-up does this once per device).  Returns the
// HIP status of the lookup, kept for later calls.
hipError_t scratch_resolve(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_resolve_mu);
    ScratchSlot &s = g_slots[device];
    if (!s.resolved) {
        void *p = nullptr;
        s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        s.ptr = s.err == hipSuccess ? p : nullptr;
        s.resolved = true;
    }
    return s.err;
}

// Device address of the array on `device` (resolved by scratch_resolve), and
// the lock that serialises its users.  E_DEVICE if the lookup failed or was
// never made.
int scratch_region(int device, void **base, std::mutex **use)
{
    if (device < 0 || device >= kMaxDevices) return fail(MESH_SDD_E_DEVICE, "device %d has no scratch slot", device);
    std::lock_guard<std::mutex> g(g_resolve_mu);
    ScratchSlot &s = g_slots[device];
    if (!s.resolved) return fail(MESH_SDD_E_DEVICE, "scratch of device %d was never resolved", device);
    if (s.err != hipSuccess || !s.ptr)
        return fail(MESH_SDD_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                    hipGetErrorString(s.err));
    *base = s.ptr;
    *use = &s.use;
    return MESH_SDD_OK;
}

}  // namespace msdd_rt
