// Hardware-queue check for the batch's second lane.
//
// The runtime maps every stream of a process onto a few hardware queues.  Two
// streams that share one run their kernels one after the other, so two lanes
// on them lose all overlap (measured: a served mix at 0.33 instead of 0.19 ms
// per step when the second lane's stream was created after enough request
// streams to land on the batch stream's queue).  The check launches, on the
// first stream, a kernel that waits a bounded time for a flag and, on the
// second, a kernel that sets it: the flag is seen only when both kernels run
// at the same time, i.e. when the streams reach the GPU through different
// queues.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lbmib {

// 200 us of the 100 MHz wall clock: the waiting kernel always ends.
constexpr long long kProbeTicks = 20000;

__global__ void k_queue_wait(const int* flag, int* seen, long long ticks) {
    if (threadIdx.x != 0) return;
    const long long t0 = wall_clock64();
    int v = 0;
    do {
        v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0) break;
        __builtin_amdgcn_s_sleep(2);
    } while (wall_clock64() - t0 < ticks);
    *seen = v;
}

__global__ void k_queue_set(int* flag) {
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t streams_run_concurrently(hipStream_t first, hipStream_t second, int* flags, bool* concurrent) {
    *concurrent = false;
    hipError_t e = hipMemsetAsync(flags, 0, 2 * sizeof(int), first);
    if (e == hipSuccess) e = hipStreamSynchronize(first);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_queue_wait, dim3(1), dim3(64), 0, first, flags, flags + 1, kProbeTicks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_queue_set, dim3(1), dim3(64), 0, second, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(second)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(first)) != hipSuccess) return e;
    int seen = 0;
    if ((e = hipMemcpy(&seen, flags + 1, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) return e;
    *concurrent = seen != 0;
    return hipSuccess;
}

}  // namespace lbmib
