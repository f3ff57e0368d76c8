// noalloc.hip -- the fixed working memory of tartarus_trace_noalloc, the
// trace entry point for callers that cannot allocate device memory.
//
// The array below is a device global: every GPU the library runs on holds its
// own copy, at its own address, from module load until the process ends.  In
// host code its name is a host-side stand-in, not a device address; the host
// side looks the device address up with hipGetSymbolAddress, once per device
// with that device current (tartarus_init), and hands that pointer to the
// kernels like any other buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace tartarus {

static __device__ __align__(256) unsigned char scratch[NoallocLayout::bytes];

// One job-table entry, passed by value, into device memory (the allocation-free
// path has no pinned staging buffer to copy from).
__global__ void job_upload_kernel(DevJob J, DevJob* dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = J;
}

}  // namespace tartarus

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on `device`, which must be the current
// device on the first call for it; later calls return the cached address.
extern "C" hipError_t tartarus_noalloc_scratch(int device, void** ptr)
{
    if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(tartarus::scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

extern "C" hipError_t tartarus_launch_job_upload(const tartarus::DevJob* job, tartarus::DevJob* dst,
                                                 hipStream_t stream)
{
    hipLaunchKernelGGL(tartarus::job_upload_kernel, dim3(1), dim3(64), 0, stream, *job, dst);
    return hipGetLastError();
}
