// probe_kernels.hip -- measurement aids with no counterpart in the method.
//
//  k_atomic_probe  the peak rate of the device-scope float atomics that the
//                  raster's tile flushes issue (one wave writes 64
//                  consecutive floats of the grid with one atomic
//                  instruction).  Each wave adds 1.0f to one 64-float
//                  segment at a slot spread over the buffer by a
//                  multiplicative hash, so the requests land on every L2
//                  channel and memory page the way scattered tile flushes do.
//  k_philox_probe  the rate of the raster's per-bin draw: Philox4x32-10
//                  blocks and their 52-bit uniforms, independent per thread,
//                  summed so that none is skipped.
//  k_row_copy_probe  the memory floor of the time R2C's access pattern: the
//                  same persistent grid of 384-thread workgroups, rows read
//                  as float pairs with the next row's loads in flight, rows
//                  of complex values written at a padded pitch, and no
//                  transform in between.
#include <algorithm>

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

// Thread t draws blocks i = t, t + T, ... < n_blocks (T threads in all),
// each from the counter (i mod 2^32, 0x5EED, i >> 32, 0) under a fixed key,
// and writes the sum of their first uniforms to out[t].
__global__ __launch_bounds__(256) void k_philox_probe(double* __restrict__ out, int64_t n_blocks) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x, T = (int64_t)gridDim.x * 256;
    double acc = 0.0;
    for (int64_t i = t; i < n_blocks; i += T) {
        uint32_t c0 = (uint32_t)i, c1 = 0x5EEDu, c2 = (uint32_t)(i >> 32), c3 = 0u;
        philox4x32_10(c0, c1, c2, c3, 0x12345678u, 0x9ABCDEF0u);
        acc += u52(c0, c1);
    }
    out[t] = acc;
}

hipError_t launch_philox_probe(double* out, int64_t n_threads, int64_t n_blocks, hipStream_t s) {
    if (n_threads <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_probe, dim3((unsigned)(n_threads / 256)), dim3(256), 0, s, out, n_blocks);
    return hipGetLastError();
}

// Row r: pairs k < n_in/2 of the input row (k = tid + 384 i, i < 8) go to
// element k of the output row; elements n_in/2 .. n_out-1 repeat the last
// pair (the writes the transform would make there).  n_in <= 6144 and
// n_out <= 3073 (checked by the caller): every read index is clamped into
// the row and every write index is below n_out.
__global__ __launch_bounds__(384) void k_row_copy_probe(const float* __restrict__ in, int64_t ld_in, int n_in,
                                                        int nrows, float2* __restrict__ out, int64_t ld_out,
                                                        int n_out) {
    const int tid = threadIdx.x, last = (n_in >> 1) - 1;
    float2 v[8], vl = make_float2(0.f, 0.f);
    int row = blockIdx.x;
    auto issue = [&](int r) {
        const float2* x2 = reinterpret_cast<const float2*>(in + (int64_t)r * ld_in);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = x2[min(tid + i * 384, last)];
        if (tid == 0) vl = x2[last];   // element 3072 (n_out = 3073)
    };
    if (row < nrows) issue(row);
    for (; row < nrows; row += gridDim.x) {
        float2 u[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) u[i] = v[i];
        const float2 ul = vl;
        if (row + (int)gridDim.x < nrows) issue(row + gridDim.x);
        float2* y = out + (int64_t)row * ld_out;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = tid + i * 384;
            if (k < n_out) y[k] = u[i];
        }
        if (tid == 0 && n_out > 3072) y[3072] = ul;
    }
}

hipError_t launch_row_copy_probe(const float* in, int64_t ld_in, int n_in, int nrows, float2* out, int64_t ld_out,
                                 int n_out, int per_cu, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(nrows, (int64_t)per_cu * device_cus());
    hipLaunchKernelGGL(k_row_copy_probe, dim3((unsigned)g), dim3(384), 0, s, in, ld_in, n_in, nrows, out, ld_out,
                       n_out);
    return hipGetLastError();
}

}  // namespace lar
