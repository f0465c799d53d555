// Residuals of many instances without any allocation: the per-member results
// live in one file-scope device array (`scratch`), whose address on each
// device is looked up once and handed to the kernels; the job table travels
// in the kernel arguments.  The reduction bodies are the ones of the
// per-instance residual (reduce.h), so the values are bitwise those of
// sdugks_residual.
#include <mutex>

#include "device.h"
#include "reduce.h"

namespace sdg {

namespace {

// Per-device scratch: [kNoAllocMaxMembers][4] doubles of results.  The job
// table itself travels in the kernel arguments (kNoAllocPack members per
// launch), so nothing is copied from the host before the kernels run.
__device__ __align__(256) double scratch[kNoAllocMaxMembers * 4];

std::mutex g_mu;
void *g_ptr[kNoAllocMaxDevices] = {};

__global__ void __launch_bounds__(256) k_reduce_pack(ReducePack p)
{
    const ReduceJob &j = p.jobs[blockIdx.y];
    reduce_block(j.nc, j.np, j.W, j.area, j.snap, 1, j.partials, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_reduce_final_pack(ReducePack p, double *out)
{
    reduce_final(p.jobs[blockIdx.x].partials, out + 4 * (size_t)blockIdx.x);
}

}  // namespace

hipError_t noalloc_scratch(int device, double **out)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        // with that device current: each device holds its own copy of the array
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t back = hipSetDevice(cur);   // the caller's device, as it was
            if (e == hipSuccess) e = back;
        }
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
    }
    *out = static_cast<double *>(g_ptr[device]);
    return hipSuccess;
}

hipError_t launch_reduce_packs(const ReduceJob *jobs, int n, double *out, hipStream_t st)
{
    for (int k0 = 0; k0 < n; k0 += kNoAllocPack) {
        ReducePack p{};
        const int m = n - k0 < kNoAllocPack ? n - k0 : kNoAllocPack;
        for (int k = 0; k < m; k++) p.jobs[k] = jobs[k0 + k];
        hipLaunchKernelGGL(k_reduce_pack, dim3(kReduceBlocks, m), dim3(256), 0, st, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_reduce_final_pack, dim3(m), dim3(kReduceBlocks), 0, st, p, out + 4 * (size_t)k0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sdg
