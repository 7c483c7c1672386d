// Allocation-free stepping: cl_step's passes with their scratch (workgroup
// partial sums, the scalar blocks that carry the background between passes,
// the per-step record ring) in a fixed device array of this file instead of
// memory the handle allocates on demand.  For callers that cannot allocate.
#include "internal.h"

#include <hip/hip_runtime.h>
#include <mutex>

namespace {

using cl::Scal;

constexpr size_t kMaxRecords = 4096;
constexpr size_t kHalf = static_cast<size_t>(cl::kMaxSums) * cl::kMaxPassBlocks;  // doubles per half
constexpr size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }
constexpr size_t kPartialsBytes = align256(2 * kHalf * sizeof(double));
constexpr size_t kScalBytes = align256(2 * sizeof(Scal));
constexpr size_t kObsBytes = align256(kMaxRecords * sizeof(cl_observables));
constexpr size_t kScratchBytes = kPartialsBytes + kScalBytes + kObsBytes;

// Every device that runs the library holds its own copy of this array until
// the process ends.  In host code its name is not a device address: host code
// uses the address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current.
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" cl_status cl_step_noalloc(cl_lattice* h, cl_integrator integ, double dt, int n,
                                     cl_observables* per_step) {
    if (!h) return cl::set_error(nullptr, CL_EINVAL, "handle is NULL");
    if (h->device < 0 || h->device >= kMaxDevices) return cl::set_error(h, CL_EUNSUPPORTED, "device index too large");
    if (n > static_cast<int>(kMaxRecords))
        return cl::set_error(h, CL_EINVAL, "cl_step_noalloc: n exceeds 4096 steps per call");
    void* base = nullptr;
    const hipError_t e = scratch_address(h->device, &base);
    if (e != hipSuccess) return cl::set_error(h, CL_EDEVICE, hipGetErrorString(e));
    unsigned char* p = static_cast<unsigned char*>(base);
    cl::Work w;
    w.partials = reinterpret_cast<double*>(p);
    w.half = kHalf;
    w.scb = reinterpret_cast<Scal*>(p + kPartialsBytes);
    w.obs = reinterpret_cast<cl_observables*>(p + kPartialsBytes + kScalBytes);
    w.obs_cap = static_cast<int>(kMaxRecords);
    return cl::step_in_work(h, integ, dt, n, per_step, w);
}
