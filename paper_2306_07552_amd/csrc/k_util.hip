// Small device utilities of the runtime: an order-independent 64-bit hash of
// a u32 buffer (used by the autotuner to check that every launch
// configuration yields the same output bits).
#include "gal_internal.h"

namespace gal {

namespace {

__device__ __forceinline__ unsigned long long mix64(unsigned long long x)
{
    // SplitMix64 finaliser (Steele, Lea, Flood 2014)
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ void k_hash_u32(const uint32_t *__restrict__ a, uint64_t n, unsigned long long *out)
{
    unsigned long long h = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        h ^= mix64((i << 32) ^ (unsigned long long)a[i] ^ 0x9e3779b97f4a7c15ull);
    // wave reduction, then one atomic per wave
    for (int d = 32; d >= 1; d >>= 1) h ^= (unsigned long long)__shfl_xor((long long)h, d, 64);
    if ((threadIdx.x & 63) == 0) atomicXor(out, h);
}

}  // namespace

hipError_t launch_hash_u32(const uint32_t *a, uint64_t n, unsigned long long *out, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(out, 0, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_hash_u32, dim3((unsigned)blocks), dim3(256), 0, s, a, n, out);
    return hipGetLastError();
}

}  // namespace gal
