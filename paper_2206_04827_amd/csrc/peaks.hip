// Device peak checks (measurement support, not a step of the method): the
// rates the roofline fractions are quoted against, measured on the device
// itself next to the vendor figures.
//
// k_fma_peak: independent FP64 FMA chains in every lane of every compute
//   unit; the result is stored only under a condition that never holds, so
//   the chains stay live without memory traffic.
// k_copy_peak: streaming copy of n doubles, 16-byte accesses, grid-stride.
#include "kernels.hpp"

namespace cyl {
namespace {

constexpr int kChains = 16;     // independent accumulators per lane

__global__ __launch_bounds__(256) void k_fma_peak(double* sink, int iters, double x, double y) {
    double a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = 1e-3 * threadIdx.x + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = fma(a[i], x, y);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    if (s == 1.25e300) sink[blockIdx.x] = s;   // never true for |x| < 1, small y
}

__global__ __launch_bounds__(256) void k_copy_peak(const double2* __restrict__ src, double2* __restrict__ dst,
                                                   int64_t n2) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n2; i += stride)
        dst[i] = src[i];
}

__global__ void k_copy_tail(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
    if (threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

}  // namespace

hipError_t launch_fma_peak(double* sink, int blocks, int iters, hipStream_t s, double* flops) {
    hipLaunchKernelGGL(k_fma_peak, dim3(blocks), dim3(256), 0, s, sink, iters, 0.9999999, 1e-9);
    *flops = 2.0 * kChains * static_cast<double>(iters) * 256.0 * blocks;
    return hipGetLastError();
}

hipError_t launch_copy_peak(const double* src, double* dst, int64_t n, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_peak, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const double2*>(src),
                       reinterpret_cast<double2*>(dst), n / 2);
    if (n & 1) hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace cyl
