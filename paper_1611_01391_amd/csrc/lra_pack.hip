// Packing of the nucleus factors of a launch's problems for read-back.
//
// A problem's generator G = A[I,J] and nucleus U have a region of kcap^2
// binary64 entries each in the workspace, of which the final rank k uses the
// first k^2 (row-major k x k).  With thousands of far-field problems at a rank
// cap of 48 and final ranks near 8, reading whole regions back moves ~36 times
// the bytes the results hold.  Problem b's G and U are copied to offset
// P_b = sum_{j<b} k_j^2 of two packed arrays, so that the host reads back
// sum k^2 entries of each.  The host forms the same P_b from the task states
// it reads back.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lra_internal.h"

namespace lra {

// One workgroup per problem.  base: the workspace; off: per problem the byte
// offsets of its state, its G region and its U region (3 np entries);
// out_g / out_u: the packed arrays (binary64).
__global__ __launch_bounds__(256) void pack_factors_kernel(const uint8_t* base, const int64_t* off, int np,
                                                           double* out_g, double* out_u)
{
    __shared__ int64_t part[256];
    const int b = blockIdx.x;
    // P_b: every thread sums the k^2 of a share of the problems before b
    int64_t s = 0;
    for (int j = threadIdx.x; j < b; j += 256) {
        const int64_t kj = ((const TaskState*)(base + off[3 * j]))->k;
        s += kj * kj;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const int64_t pb = part[0];
    const int64_t k = ((const TaskState*)(base + off[3 * b]))->k;
    const double* g = (const double*)(base + off[3 * b + 1]);
    const double* u = (const double*)(base + off[3 * b + 2]);
    for (int64_t e = threadIdx.x; e < k * k; e += 256) {
        out_g[pb + e] = g[e];
        out_u[pb + e] = u[e];
    }
}

hipError_t launch_pack_factors(const void* base, const int64_t* off, int np, double* out_g, double* out_u,
                               hipStream_t stream)
{
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_factors_kernel, dim3(np), dim3(256), 0, stream, (const uint8_t*)base, off, np, out_g,
                       out_u);
    return hipGetLastError();
}

}  // namespace lra
