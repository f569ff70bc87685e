// su2_kcommon.h -- device helpers shared by the kernel files of libsu2:
// FP64 workgroup sums, the 64-bit fixed-point accumulators and the
// XCD-aware mapping of workgroups to tiles.
#pragma once

#include "su2_internal.h"

namespace su2rt {

// FP64 sum over the block; the result is valid in thread 0.  Fixed order.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double wsum[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) wsum[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r += wsum[i];
    }
    __syncthreads();  // wsum may be reused by the next call
    return r;
}

__device__ __forceinline__ unsigned long long to_fixed(double v)
{
    return (unsigned long long)__double2ll_rn(v * (double)(1ll << kFixedShift));
}

__device__ __forceinline__ double from_fixed(unsigned long long u)
{
    return (double)(long long)u * (1.0 / (double)(1ll << kFixedShift));
}

__device__ __forceinline__ unsigned long long *bucket(unsigned long long *acc, int which, uint32_t b)
{
    return acc + ((size_t)which * kBuckets + (b % kBuckets)) * kBucketStride;
}

// Thread 0 adds the block's FP64 sum to bucket (b mod kBuckets) of
// fixed-point accumulator `which`.
__device__ __forceinline__ void block_accumulate(double v, unsigned long long *acc, int which,
                                                 uint32_t b)
{
    const double s = block_sum(v);
    if (threadIdx.x == 0) atomicAdd(bucket(acc, which, b), to_fixed(s));
}

// Exact integer total of accumulator `which` over its buckets, computed by a
// block of kBuckets threads (valid in thread 0); the buckets are reset.
__device__ __forceinline__ unsigned long long take_total(unsigned long long *acc, int which)
{
    __shared__ unsigned long long part[kBuckets / 64];
    unsigned long long *p = bucket(acc, which, threadIdx.x);
    unsigned long long v = *p;
    *p = 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0ull;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBuckets / 64; ++i) t += part[i];
    __syncthreads();
    return t;
}

// Map the hardware workgroup id to a logical tile so that the workgroups one
// XCD runs (dispatched round-robin over the 8 XCDs) cover one contiguous
// stretch of the lattice and share that XCD's L2.  With `reverse`, each XCD
// walks its stretch backwards: alternating passes then start where the
// previous pass ended, on data still held by the memory-side cache.
__device__ __forceinline__ uint32_t logical_block(uint32_t b, uint32_t nb, int remap, int reverse)
{
    if (!remap) return reverse ? nb - 1u - b : b;
    const uint32_t per = nb >> 3;  // full rounds
    const uint32_t full = per << 3;
    if (b >= full) return b;  // ragged tail keeps its id
    const uint32_t local = reverse ? per - 1u - (b >> 3) : (b >> 3);
    return (b & 7u) * per + local;
}

}  // namespace su2rt
