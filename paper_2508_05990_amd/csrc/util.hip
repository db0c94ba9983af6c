// Small helper kernels: filling device buffers without hipMemsetAsync, so the
// same code stays valid inside a captured HIP graph.
#include "internal.h"

namespace me {
namespace {

__global__ void fill_u8_kernel(uint8_t* p, size_t n, uint8_t v)
{
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

__global__ void fill_i32_kernel(int32_t* p, size_t n, int32_t v)
{
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

}  // namespace

hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace me
