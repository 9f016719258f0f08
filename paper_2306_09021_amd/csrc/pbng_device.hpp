// Device helpers shared by the tetrahedral and the planar kernels of
// libpbng: 32-bit-offset addressing, the XCD-aware block order and the
// in-group sums over the lanes that own one vertex.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pbng {

// Element i of an array through a 32-bit byte offset, so that the load takes
// the array base from scalar registers and only the offset from a vector
// register (the host keeps every array under 4 GiB).
template <class T>
__device__ __forceinline__ T at(const T* base, int i)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                       uint32_t(i) * uint32_t(sizeof(T)));
}

template <class T>
__device__ __forceinline__ T* ptr_at(T* base, int i)
{
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + uint32_t(i) * uint32_t(sizeof(T)));
}

// Block index remapped so that the blocks the dispatcher places on one XCD
// (block b goes to XCD b % 8) cover one contiguous range of vertices: a
// colour's vertices are ordered by instance and position, so each XCD's L2
// then gathers the neighbour positions of a compact region instead of every
// eighth block of the whole mesh.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Value of v in another lane of the same 16-lane row (data-parallel
// primitive; CTRL is the row permutation code).
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)((unsigned long long)(unsigned)hi << 32 | (unsigned)lo));
}

// Sum over the LANES lanes of a group (groups are aligned, LANES | 64).  The
// first four stages pair lanes inside a row: quad permutations [1,0,3,2] and
// [2,3,0,1], then the half-row mirror (i <-> 7 - i) and the row mirror
// (i <-> 15 - i); wider groups continue with cross-row shuffles.  Each stage
// adds two equal partial sums in commuted order, so every lane of the group
// ends with the same bits.
template <int LANES, class T>
__device__ __forceinline__ T lsum(T v)
{
    if (LANES >= 2) v += dpp<0xB1>(v);
    if (LANES >= 4) v += dpp<0x4E>(v);
    if (LANES >= 8) v += dpp<0x141>(v);
    if (LANES >= 16) v += dpp<0x140>(v);
    if (LANES >= 32) v += __shfl_xor(v, 16, LANES);
    if (LANES >= 64) v += __shfl_xor(v, 32, LANES);
    return v;
}

}  // namespace pbng
