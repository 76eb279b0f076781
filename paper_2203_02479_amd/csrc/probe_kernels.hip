// probe_kernels.hip -- a measurement aid with no counterpart in the method:
// the peak rate of the device-scope float atomics that the raster's tile
// flushes issue (one wave writes 64 consecutive floats of the grid with one
// atomic instruction).  Each wave adds 1.0f to one 64-float segment at a
// slot spread over the buffer by a multiplicative hash, so the requests land
// on every L2 channel and memory page the way scattered tile flushes do.
#include "lar_internal.hpp"

namespace lar {

typedef __attribute__((address_space(1))) float probe_global_float;

__global__ __launch_bounds__(256) void k_atomic_probe(float* __restrict__ buf, int64_t slots, int64_t n_seg) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); sg < n_seg; sg += waves) {
        const uint64_t slot = ((uint64_t)sg * 0x9E3779B97F4A7C15ull >> 17) % (uint64_t)slots;
        __hip_atomic_fetch_add((probe_global_float*)(buf + slot * 64 + lane), 1.0f, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Segments slot*64 .. slot*64+63 with slot < n_floats/64: every access is
// inside buf.  Grid-stride loop over at most 64 workgroups per CU.
hipError_t launch_atomic_probe(float* buf, int64_t n_floats, int64_t n_seg, hipStream_t s) {
    const int64_t slots = n_floats / 64;
    if (slots <= 0 || n_seg <= 0) return hipSuccess;
    const int64_t blocks = (n_seg + 3) / 4, cap = 64 * (int64_t)device_cus();
    hipLaunchKernelGGL(k_atomic_probe, dim3((unsigned)(blocks < cap ? blocks : cap)), dim3(256), 0, s, buf, slots,
                       n_seg);
    return hipGetLastError();
}

}  // namespace lar
