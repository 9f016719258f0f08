// Device side of the batched uploads of libpbng's host code
// (pbng_hostutil.hpp): one transfer brings a table of CopyItem entries and
// the packed arrays; one launch places every array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "pbng_hostutil.hpp"

namespace pbng {

namespace {
constexpr int kUpBlock = 256;
}  // namespace

// Batched upload: entry y of the CopyItem table at the start of the staged
// payload copies its words; blocks along x stride over them.
__global__ __launch_bounds__(kUpBlock) void k_scatter_words(const uint32_t* staged, int n_items)
{
    const int i = blockIdx.y;
    if (i >= n_items) return;
    const CopyItem it = reinterpret_cast<const CopyItem*>(staged)[i];
    uint32_t* dst = static_cast<uint32_t*>(it.dst);
    const uint32_t* src = staged + it.src_off / 4;
    for (uint32_t w = blockIdx.x * kUpBlock + threadIdx.x; w < it.n_words; w += gridDim.x * kUpBlock) dst[w] = src[w];
}

hipError_t launch_scatter_words(const void* staged, int n_items, uint32_t max_words, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (n_items > 65535) return hipErrorInvalidValue;
    const uint32_t bx = std::min<uint32_t>(1024, (max_words + kUpBlock - 1) / kUpBlock);
    hipLaunchKernelGGL(k_scatter_words, dim3(std::max<uint32_t>(1, bx), n_items), dim3(kUpBlock), 0, s,
                       static_cast<const uint32_t*>(staged), n_items);
    return hipGetLastError();
}

}  // namespace pbng
