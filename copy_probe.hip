// Reference streams for the HBM roofline of the lattice sweep: hand-written
// copy, read-only and write-only kernels over plain device buffers, so that
// the rate a read-and-write stream reaches on this part can be measured beside
// the sweep (which reads and writes the same number of bytes per node).
//
// Variants (copy_probe_launch):
//   0 copy, 16-byte loads and stores, grid-stride loop over the buffer
//   1 copy, 16-byte non-temporal loads and stores, grid-stride loop
//   2 copy, 16-byte loads and stores, one workgroup per 4 KiB chunk per thread row
//     (no loop: as many workgroups as chunks, like the sweep's one workgroup per tile)
//   3 copy, as 2 with non-temporal loads and stores
//   4 read only: 16-byte non-temporal loads, one 4-byte result per workgroup
//   5 write only: 16-byte non-temporal stores of a constant
//
// Built by copy_probe.py (hipcc, gfx950) into copy_probe.so; measurement only,
// no part of the library.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f4 __attribute__((ext_vector_type(4)));
#define AS1 __attribute__((address_space(1)))

template <bool NT>
__device__ __forceinline__ f4 ld(const AS1 f4* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT>
__device__ __forceinline__ void st(AS1 f4* p, f4 v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT>
__global__ void __launch_bounds__(256) k_copy_loop(AS1 f4* __restrict__ dst, const AS1 f4* __restrict__ src, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    // four independent 16-byte loads in flight per thread
    for (; i + 3 * stride < n; i += 4 * stride) {
        const f4 a = ld<NT>(src + i), b = ld<NT>(src + i + stride), c = ld<NT>(src + i + 2 * stride),
                 d = ld<NT>(src + i + 3 * stride);
        st<NT>(dst + i, a);
        st<NT>(dst + i + stride, b);
        st<NT>(dst + i + 2 * stride, c);
        st<NT>(dst + i + 3 * stride, d);
    }
    for (; i < n; i += stride) st<NT>(dst + i, ld<NT>(src + i));
}

// one workgroup per chunk of 256 threads x 4 vectors (16 KiB)
template <bool NT>
__global__ void __launch_bounds__(256) k_copy_chunk(AS1 f4* __restrict__ dst, const AS1 f4* __restrict__ src, size_t n) {
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    f4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t i = base + 256 * k;
        if (i < n) v[k] = ld<NT>(src + i);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t i = base + 256 * k;
        if (i < n) st<NT>(dst + i, v[k]);
    }
}

__global__ void __launch_bounds__(256) k_read(float* __restrict__ out, const AS1 f4* __restrict__ src, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc += ld<true>(src + i);
    float s = acc.x + acc.y + acc.z + acc.w;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_fill(AS1 f4* __restrict__ dst, size_t n, float v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const f4 c = {v, v, v, v};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) st<true>(dst + i, c);
}

extern "C" {

// bytes must be a multiple of 16 and the pointers 16-byte aligned; grid is
// ignored by the chunk variants (one workgroup per 16 KiB); scratch (variant 4)
// holds one float per workgroup.  Returns a hipError_t value.
int copy_probe_launch(int variant, void* dst, const void* src, size_t bytes, int grid, void* scratch, void* stream) {
    if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || grid <= 0) return (int)hipErrorInvalidValue;
    const size_t n = bytes / 16;
    hipStream_t s = (hipStream_t)stream;
    AS1 f4* d = (AS1 f4*)dst;
    const AS1 f4* r = (const AS1 f4*)src;
    const unsigned chunks = (unsigned)((n + 1023) / 1024);
    switch (variant) {
        case 0: hipLaunchKernelGGL(k_copy_loop<false>, dim3(grid), dim3(256), 0, s, d, r, n); break;
        case 1: hipLaunchKernelGGL(k_copy_loop<true>, dim3(grid), dim3(256), 0, s, d, r, n); break;
        case 2: hipLaunchKernelGGL(k_copy_chunk<false>, dim3(chunks), dim3(256), 0, s, d, r, n); break;
        case 3: hipLaunchKernelGGL(k_copy_chunk<true>, dim3(chunks), dim3(256), 0, s, d, r, n); break;
        case 4:
            if (!scratch) return (int)hipErrorInvalidValue;
            hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, s, (float*)scratch, r, n);
            break;
        case 5: hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, d, n, 1.0f); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}
}
