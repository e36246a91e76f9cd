// Fixed device scratch of zs_query_noalloc, the query entry point that
// allocates nothing (for callers that cannot call hipMalloc: code under HIP
// graph capture, serving loops, harnesses that forbid allocation).
//
// The scratch is a file-scope device array, one copy per GPU the library
// runs on, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): its
// device address is looked up once per device with hipGetSymbolAddress and
// every use goes through that address.
#include "zs_internal.h"

#include <map>
#include <mutex>

namespace zs {
namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
std::map<int, void *> g_ptr;   // device -> address of that device's scratch

// Writes the descriptors of one planned query into the scratch: the plan
// itself (descriptor, problem, Partial-SVD pieces, Gram-tree nodes) arrives
// by value; the projection chunks and the identity piece order are formed
// here.
__global__ __launch_bounds__(kThreads) void plan_single_kernel(SinglePlan p)
{
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        if (tid == 0) {
            *p.d_qd = p.qd;
            *p.d_prob = p.prob;
        }
        if (tid < p.npidx) {
            p.d_pidx[tid] = p.pidx[tid];
            p.d_msrc[tid] = p.Mp + (int64_t)p.msrc[tid] * p.k * p.c;
        }
        for (int i = tid; i < p.ngsrc; i += kThreads) p.d_gsrc[i] = p.tree + p.gsrc[i] * p.c * p.c;
        for (int j = tid; j < p.nchunks; j += kThreads)
            p.d_chunks[j] = make_stack_chunk(j, p.qd.np, p.k, p.qd.kq, 0, 0, 0, j);
    }
    const int i = blockIdx.x * kThreads + tid;
    if (i < p.qd.np) p.d_perm[i] = i;
}

}  // namespace

hipError_t noalloc_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ptr.find(dev);
    if (it == g_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = g_ptr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

hipError_t launch_plan_single(const SinglePlan &p, hipStream_t stream)
{
    const unsigned grid = (unsigned)((p.qd.np + kThreads - 1) / kThreads);
    plan_single_kernel<<<grid, kThreads, 0, stream>>>(p);
    return hipGetLastError();
}

}  // namespace zs
