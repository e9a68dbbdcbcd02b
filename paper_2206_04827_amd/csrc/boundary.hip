// Boundary traces and the physical-parity fast path (Sections 1-3).
//
// k_trace_lift: the transfinite (Coons) interpolant in (r, z) of the four
//   faces of the doubled grid's box, for every theta line -- the lift whose
//   boundary values are the Dirichlet data (the r^2-weighted equations of
//   Section 3 make any such lift admissible).
// k_zero_blocks: zero the solution blocks that a physical-parity solve skips
//   (the r-parity blocks with j != w mod 2), so that recombination and the
//   residual see exact zeros there.
#include "kernels.hpp"

namespace cyl {
namespace {

// lift[l][k][j] from rface [2][p][n] (r = -1, r = +1), zface [2][p][m]
// (z = -1, z = +1), a_j = (1 + r_j) / 2, b_k = (1 + z_k) / 2; corner values
// from the z-faces.  One thread per value, r fastest.
__global__ __launch_bounds__(256) void k_trace_lift(const double* __restrict__ rface,
                                                     const double* __restrict__ zface,
                                                     const double* __restrict__ ra,
                                                     const double* __restrict__ zb, double* __restrict__ lift,
                                                     int m, int n, int p) {
    const int64_t total = static_cast<int64_t>(p) * n * m;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int j = static_cast<int>(i % m);
    const int64_t lk = i / m;
    const int k = static_cast<int>(lk % n);
    const int l = static_cast<int>(lk / n);
    const double a = ra[j], b = zb[k];
    const int64_t rp = static_cast<int64_t>(p) * n, zp = static_cast<int64_t>(p) * m;
    const double Rm = rface[static_cast<int64_t>(l) * n + k], Rp = rface[rp + static_cast<int64_t>(l) * n + k];
    const double* zm = zface + static_cast<int64_t>(l) * m;
    const double* zpl = zface + zp + static_cast<int64_t>(l) * m;
    const double Zm = zm[j], Zp = zpl[j];
    const double corner = (1 - a) * (1 - b) * zm[0] + a * (1 - b) * zm[m - 1] + (1 - a) * b * zpl[0] +
                          a * b * zpl[m - 1];
    lift[i] = (1 - a) * Rm + a * Rp + (1 - b) * Zm + b * Zp - corner;
}

// grid (chunks of 1024 values, nblocks): zero the me x ne solution of each block.
__global__ __launch_bounds__(256) void k_zero_blocks(const BlockDesc* __restrict__ blocks, double* X) {
    const BlockDesc bd = blocks[blockIdx.y];
    const int64_t cnt = static_cast<int64_t>(bd.me) * bd.ne;
    double* Xb = X + bd.xoff;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 1024 + threadIdx.x; i < cnt &&
                                                                           i < static_cast<int64_t>(blockIdx.x + 1) * 1024;
         i += blockDim.x)
        Xb[i] = 0.0;
}

// out[i] = 0 for i < n (grid-stride).  Used instead of hipMemsetAsync so that
// a captured graph holds kernel nodes only.
__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ out, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = 0.0;
}

}  // namespace

hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const unsigned grid = static_cast<unsigned>(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, s, out, n);
    return hipGetLastError();
}

hipError_t launch_trace_lift(const double* rface, const double* zface, const double* ra, const double* zb,
                             double* lift, int m, int n, int p, hipStream_t s) {
    const int64_t total = static_cast<int64_t>(p) * n * m;
    if (total == 0) return hipSuccess;
    const unsigned grid = static_cast<unsigned>((total + 255) / 256);
    hipLaunchKernelGGL(k_trace_lift, dim3(grid), dim3(256), 0, s, rface, zface, ra, zb, lift, m, n, p);
    return hipGetLastError();
}

hipError_t launch_zero_blocks(const BlockDesc* blocks, int nblocks, int me0, int ne0, double* X,
                              hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
    const int64_t most = static_cast<int64_t>(me0) * ne0;
    const dim3 grid(static_cast<unsigned>((most + 1023) / 1024), static_cast<unsigned>(nblocks));
    hipLaunchKernelGGL(k_zero_blocks, grid, dim3(256), 0, s, blocks, X);
    return hipGetLastError();
}

}  // namespace cyl
