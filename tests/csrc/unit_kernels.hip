// unit_kernels.hip -- test-only entry points that run the library's device
// building blocks on caller-supplied data, so that each can be checked on
// its own against host arithmetic: the bit-parallel full adder (Section
// 3.1), the CSA_{16+4} network (Sections 3.2 and 4.2), the end-of-segment
// reduction of a wave's bit planes (Section 4.5) and the accumulation
// function f_w.  Built into tests/csrc/libppc_unit.so; not part of the
// library.  All pointers are device pointers; every entry point returns the
// hipError_t of its launch (0 = success).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppc_device.hpp"

using namespace ppc;

namespace {

// thread t < n: (carry[t], sum[t]) = FA(a[t], b[t], c[t])
__global__ void unit_full_add_kernel(const uint4 *a, const uint4 *b, const uint4 *c, uint4 *carry, uint4 *sum,
                                     uint32_t n) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint4 co, s;
    full_add(co, s, a[t], b[t], c[t]);
    carry[t] = co;
    sum[t] = s;
}

// thread t < n: accumulator state acc[4t .. 4t+3] = (a1, a2, a4, a8) and
// inputs in[16t .. 16t+15]; out[5t .. 5t+4] = (a1', a2', a4', a8', a16)
__global__ void unit_csa16_kernel(const uint4 *acc, const uint4 *in, uint4 *out, uint32_t n) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    Planes pl;
    pl.clear();
    pl.a1 = acc[4 * t + 0];
    pl.a2 = acc[4 * t + 1];
    pl.a4 = acc[4 * t + 2];
    pl.a8 = acc[4 * t + 3];
    uint4 v[kLoadsPerTile];
#pragma unroll
    for (int j = 0; j < kLoadsPerTile; ++j) v[j] = in[(size_t)kLoadsPerTile * t + j];
    const uint4 s16 = pl.csa16(v);
    out[5 * t + 0] = pl.a1;
    out[5 * t + 1] = pl.a2;
    out[5 * t + 2] = pl.a4;
    out[5 * t + 3] = pl.a8;
    out[5 * t + 4] = s16;
}

// block w < n_waves is one wave: lane L's planes are
// planes[(64 w + L) * kPlanes + e], e < kPlanes (planes e >= e_used must be
// zero); out[64 w + L] = the wave's count at address position L
__global__ __launch_bounds__(64) void unit_wave_counts_kernel(const uint4 *planes, uint32_t e_used, uint32_t *out,
                                                             uint32_t n_waves) {
    if (blockIdx.x >= n_waves) return;  // whole block: the wave stays converged
    const uint32_t lane = threadIdx.x;
    uint4 p[kPlanes];
#pragma unroll
    for (int e = 0; e < kPlanes; ++e) p[e] = planes[((size_t)kWave * blockIdx.x + lane) * kPlanes + e];
    out[(size_t)kWave * blockIdx.x + lane] = wave_position_counts(p, e_used);
}

// block w < n_waves is one wave: lane L holds v[64 w + L], the count at
// address position L; fold_add adds them into counts[64 w ..] for `width`
// (0 = total) and pointer residue m
__global__ __launch_bounds__(64) void unit_fold_kernel(const uint64_t *v, uint32_t width, uint32_t m,
                                                      unsigned long long *counts, uint32_t n_waves) {
    if (blockIdx.x >= n_waves) return;
    fold_add(v[(size_t)kWave * blockIdx.x + threadIdx.x], width, m, counts + (size_t)kWave * blockIdx.x);
}

}  // namespace

extern "C" {

int ppc_unit_full_add(const void *a, const void *b, const void *c, void *carry, void *sum, uint32_t n) {
    if (n == 0) return 0;
    hipLaunchKernelGGL(unit_full_add_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, (const uint4 *)a,
                       (const uint4 *)b, (const uint4 *)c, (uint4 *)carry, (uint4 *)sum, n);
    return (int)hipGetLastError();
}

int ppc_unit_csa16(const void *acc, const void *in, void *out, uint32_t n) {
    if (n == 0) return 0;
    hipLaunchKernelGGL(unit_csa16_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, (const uint4 *)acc,
                       (const uint4 *)in, (uint4 *)out, n);
    return (int)hipGetLastError();
}

int ppc_unit_wave_counts(const void *planes, uint32_t e_used, void *out, uint32_t n_waves) {
    if (n_waves == 0) return 0;
    if (e_used > (uint32_t)kPlanes) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(unit_wave_counts_kernel, dim3(n_waves), dim3(kWave), 0, 0, (const uint4 *)planes, e_used,
                       (uint32_t *)out, n_waves);
    return (int)hipGetLastError();
}

int ppc_unit_fold(const void *v, uint32_t width, uint32_t m, void *counts, uint32_t n_waves) {
    if (n_waves == 0) return 0;
    if (!(width == 0 || width == 8 || width == 16 || width == 32 || width == 64)) return (int)hipErrorInvalidValue;
    if (width != 0 && m >= width / 8) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(unit_fold_kernel, dim3(n_waves), dim3(kWave), 0, 0, (const uint64_t *)v, width, m,
                       (unsigned long long *)counts, n_waves);
    return (int)hipGetLastError();
}

int ppc_unit_planes(void) { return kPlanes; }

}  // extern "C"
