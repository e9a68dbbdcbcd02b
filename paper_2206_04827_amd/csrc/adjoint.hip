// Transposed operators for reverse-mode differentiation of the heat run
// (chain rule through the discrete method of Section 3; the paper itself
// gives no adjoint).
//
// The transposed Sylvester solve of a parity block,
//     A^T Y B^T + C^T Y D^T = F,
// is run by the ordinary ADI kernels on the flipped unknowns Y~ = J Y J and
// data F~ = J F J (J reverses the index order inside the block), whose pencil
// (J A^T J, J C^T J), (J B^T J, J D^T J) has the band widths of the original.
// The kernels below therefore read and write adjoint quantities in that
// flipped orientation:  block element (i', k') <-> (me-1-i', ne-1-k').
#include "kernels.hpp"

namespace cyl {
namespace {

inline __device__ double part_of(double2 v, int part) { return part ? v.y : v.x; }

// out (E-layout, flipped) = s * Q_m^T U Q_n for every parity block, where U
// holds the T coefficients of each real mode plane:
//   (Q^T U Q)[a, l] = U[a+2, l+2] - U[a, l+2] - U[a+2, l] + U[a, l].
__global__ __launch_bounds__(256) void k_recombine_t(const double2* __restrict__ U, double s,
                                                     double* __restrict__ out,
                                                     const BlockDesc* __restrict__ blocks,
                                                     int m, int n) {
    const BlockDesc bd = blocks[blockIdx.y];
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(bd.me) * bd.ne) return;
    const int ip = static_cast<int>(e % bd.me), kp = static_cast<int>(e / bd.me);
    const int a = 2 * (bd.me - 1 - ip) + bd.pr, l = 2 * (bd.ne - 1 - kp) + bd.pz;
    const double2* Uw = U + static_cast<int64_t>(bd.w) * n * m;
    const int64_t o0 = static_cast<int64_t>(l) * m + a, o2 = o0 + 2 * static_cast<int64_t>(m);
    const double x = part_of(Uw[o2 + 2], bd.part) - part_of(Uw[o2], bd.part) -
                     part_of(Uw[o0 + 2], bd.part) + part_of(Uw[o0], bd.part);
    out[bd.eoff + static_cast<int64_t>(kp) * bd.mp + ip] = s * x;
}

// U[w, l, a] = s * sum_{i,k} R2[i, a] Y[i, k] C02[k, l]: the transpose of the
// tau right side [R2 F C02^T]_tau, with Y read flipped from X-layout blocks.
// Slots that are not a real mode plane (imaginary parts of w = 0 and Nyquist)
// are written as 0.
__global__ __launch_bounds__(256) void k_rhs_t(const double* __restrict__ Yf, double s,
                                               double2* __restrict__ U,
                                               const int* __restrict__ plane_of,
                                               const BlockDesc* __restrict__ blocks, int m, int n,
                                               RhsTables t) {
    const int w = blockIdx.y;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(m) * n) return;
    const int a = static_cast<int>(e % m), l = static_cast<int>(e / m);
    const int mi = m - 2, ni = n - 2;
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int pl = plane_of[2 * w + part];
        if (pl < 0) continue;
        const BlockDesc* b4 = blocks + 4 * pl;
        double acc = 0.0;
#pragma unroll
        for (int ta = 0; ta < 5; ++ta) {
            const int i = a + 2 - 2 * ta;          // R2[i, a] = r2[5 i + ta]
            if (i < 0 || i >= mi) continue;
            const double r = t.r2[5 * i + ta];
            if (r == 0.0) continue;
            double zacc = 0.0;
#pragma unroll
            for (int sz = 0; sz < 3; ++sz) {
                const int k = l - 2 * sz;          // C02[k, l] = c02[3 k + sz]
                if (k < 0 || k >= ni) continue;
                const BlockDesc& bd = b4[2 * (i & 1) + (k & 1)];
                const int ip = bd.me - 1 - (i >> 1), kp = bd.ne - 1 - (k >> 1);
                zacc += t.c02[3 * k + sz] * Yf[bd.xoff + static_cast<int64_t>(ip) * bd.ne + kp];
            }
            acc += r * zacc;
        }
        v[part] = s * acc;
    }
    U[(static_cast<int64_t>(w) * n + l) * m + a] = make_double2(v[0], v[1]);
}

__global__ __launch_bounds__(256) void k_axpy(double* __restrict__ y, const double* __restrict__ x,
                                              double a, int64_t count) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < count) y[e] += a * x[e];
}

// partials[workgroup] += sum over the tile of Yf~(i, k) * (A X B + C X D)(i, k),
// where Yf~ is read flipped from an X-layout buffer.  Same tiling and record
// formats as the residual kernel (32 x 32 output tiles, X tile and halo in
// LDS); each workgroup owns one partial, so the sum is deterministic.
constexpr int kTile = 32;
constexpr int kTR = kTile + 5, kTC = kTile + 3;

__global__ __launch_bounds__(256) void k_apply_dot(const BlockDesc* __restrict__ blocks,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ Yf,
                                                   const double* __restrict__ atab,
                                                   int64_t a_wstride, int me0,
                                                   const double* __restrict__ ztabA, int ne0,
                                                   double* __restrict__ partials) {
    __shared__ double xs[kTR][kTC + 1];
    __shared__ double zs[kTile * 8];
    __shared__ double red[256];
    const BlockDesc bd = blocks[blockIdx.z];
    const int me = bd.me, ne = bd.ne;
    const int i0 = blockIdx.x * kTile, k0 = blockIdx.y * kTile;
    const int64_t slot = (static_cast<int64_t>(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (i0 >= me || k0 >= ne) return;
    const double* Xb = X + bd.xoff;
    const double* Yb = Yf + bd.xoff;
    // 256 threads: the tile of X and this thread's values of Yf are all
    // requested before the first is used
    constexpr int kIt = (kTR * kTC + 255) / 256, kOut = kTile * kTile / 256;
    double xv[kIt], yv[kOut];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = threadIdx.x + 256 * it;
        const int r = idx / kTC, c = idx - r * kTC;
        const int a = i0 - 2 + r, l = k0 - 1 + c;
        xv[it] = (idx < kTR * kTC && a >= 0 && a < me && l >= 0 && l < ne) ? Xb[static_cast<int64_t>(a) * ne + l]
                                                                          : 0.0;
    }
#pragma unroll
    for (int it = 0; it < kOut; ++it) {
        const int idx = threadIdx.x + 256 * it;
        const int i = i0 + idx % kTile, k = k0 + idx / kTile;
        yv[it] = (i < me && k < ne) ? Yb[static_cast<int64_t>(me - 1 - i) * ne + (ne - 1 - k)] : 0.0;
    }
    // the tile's column records (32 columns of 8, one per thread) go to LDS;
    // a thread's row is the same in every output it computes, so its row
    // records are read once
    const double* arow = atab + bd.w * a_wstride + (bd.pr ? me0 * 12 : 0);
    const double* zcol = ztabA + (bd.pz ? ne0 * 8 : 0);
    static_assert(kTile * 8 == 256 && kTile * kTile % 256 == 0, "one record per thread; whole rows per output");
    const int di = threadIdx.x % kTile, i = i0 + di;
    const double zv = (k0 + static_cast<int>(threadIdx.x >> 3) < ne) ? zcol[k0 * 8 + threadIdx.x] : 0.0;
    double ar[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) ar[q] = i < me ? arow[i * 12 + q] : 0.0;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = threadIdx.x + 256 * it;
        if (idx >= kTR * kTC) break;
        const int r = idx / kTC, c = idx - r * kTC;
        xs[r][c] = xv[it];
    }
    zs[threadIdx.x] = zv;
    __syncthreads();
    double local = 0.0;
#pragma unroll
    for (int it = 0; it < kOut; ++it) {
        const int idx = threadIdx.x + 256 * it;
        const int dk = idx / kTile;
        const int k = k0 + dk;
        if (i >= me || k >= ne) continue;
        const double* zc = zs + dk * 8;
        double sab = 0.0, scd = 0.0;
#pragma unroll
        for (int da = 0; da < 6; ++da) {
            double xb = 0.0, xd = 0.0;
#pragma unroll
            for (int dl = 0; dl < 4; ++dl) {
                const double x = xs[di + da][dk + dl];
                xb += x * zc[dl];
                xd += x * zc[4 + dl];
            }
            sab += ar[da] * xb;
            scd += ar[6 + da] * xd;
        }
        local += yv[it] * (sab + scd);
    }
    red[threadIdx.x] = local;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[slot] += red[0];
}

// out[0] = scale * sum(partials), one workgroup, fixed summation order.
__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ partials, int64_t count,
                                             double scale, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < count; e += blockDim.x) acc += partials[e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = scale * red[0];
}

// Diagonal factors that turn the transforms into their transposes.  With
// M = n - 1 Lobatto intervals, the DCT-I pair of Section 2 satisfies
//   F_r = (2/M) H V^T W,   F_r^-1 = V  (V[j, k] = T_k(r_j)),
// H = diag(1/2 at k = 0, M; else 1), W = diag(1/2 at the two end points; else 1),
// and the real DFT pair satisfies F_theta^-1 = p F_theta^T K with
// K = diag(1 at w = 0 and Nyquist; else 2).  Hence
//   F^T      = W . F^-1 . diag((2/M_r) h_j (2/M_z) h_k / (p K_w))      (mode 0)
//   F^-T     = diag((M_r / 2h_j)(M_z / 2h_k) p K_w) . F . W^-1          (mode 1)
__global__ __launch_bounds__(256) void k_scale_planes(double2* __restrict__ U, int m, int n, int p,
                                                      int nw, int mode) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(nw) * n * m) return;
    const int j = static_cast<int>(e % m);
    const int k = static_cast<int>((e / m) % n);
    const int w = static_cast<int>(e / (static_cast<int64_t>(m) * n));
    const double hr = (j == 0 || j == m - 1) ? 0.5 : 1.0;
    const double hz = (k == 0 || k == n - 1) ? 0.5 : 1.0;
    const bool single = (w == 0) || (2 * w == p);
    const double kw = single ? 1.0 : 2.0;
    const double f = mode == 0
                         ? (2.0 * hr / (m - 1)) * (2.0 * hz / (n - 1)) / (static_cast<double>(p) * kw)
                         : ((m - 1) / (2.0 * hr)) * ((n - 1) / (2.0 * hz)) * (static_cast<double>(p) * kw);
    double2 v = U[e];
    v.x *= f;
    v.y = single ? 0.0 : v.y * f;
    U[e] = v;
}

// out = W (mode 0) or W^-1 (mode 1) applied to values [p][n][m]: factor 1/2
// (or 2) at each of the r end points and each of the z end points.
__global__ __launch_bounds__(256) void k_scale_values(const double* __restrict__ in,
                                                      double* __restrict__ out, int m, int n,
                                                      int64_t total, int mode) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int j = static_cast<int>(e % m);
    const int k = static_cast<int>((e / m) % n);
    const double g = mode == 0 ? 0.5 : 2.0;
    double f = 1.0;
    if (j == 0 || j == m - 1) f *= g;
    if (k == 0 || k == n - 1) f *= g;
    out[e] = f * in[e];
}

unsigned blocks_for(int64_t count) { return static_cast<unsigned>((count + 255) / 256); }

}  // namespace

hipError_t launch_recombine_t(const double2* U, double s, double* out, const BlockDesc* blocks,
                              int nblocks, int64_t max_block_elems, int m, int n, hipStream_t st) {
    const dim3 grid(blocks_for(max_block_elems), static_cast<unsigned>(nblocks));
    hipLaunchKernelGGL(k_recombine_t, grid, dim3(256), 0, st, U, s, out, blocks, m, n);
    return hipGetLastError();
}

hipError_t launch_rhs_t(const double* Yf, double s, double2* U, const int* plane_of,
                        const BlockDesc* blocks, int nw, int m, int n, const RhsTables& t,
                        hipStream_t st) {
    const dim3 grid(blocks_for(static_cast<int64_t>(m) * n), static_cast<unsigned>(nw));
    hipLaunchKernelGGL(k_rhs_t, grid, dim3(256), 0, st, Yf, s, U, plane_of, blocks, m, n, t);
    return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, int64_t count, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(count)), dim3(256), 0, st, y, x, a, count);
    return hipGetLastError();
}

int64_t apply_dot_partials(int nblocks, int me0, int ne0) {
    return static_cast<int64_t>((me0 + kTile - 1) / kTile) * ((ne0 + kTile - 1) / kTile) * nblocks;
}

hipError_t launch_apply_dot(const BlockDesc* blocks, int nblocks, int me0, int ne0, const double* X,
                            const double* Yf, const double* atab, int64_t a_wstride,
                            const double* ztabA, double* partials, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((me0 + kTile - 1) / kTile),
                    static_cast<unsigned>((ne0 + kTile - 1) / kTile), static_cast<unsigned>(nblocks));
    hipLaunchKernelGGL(k_apply_dot, grid, dim3(256), 0, st, blocks, X, Yf, atab, a_wstride, me0,
                       ztabA, ne0, partials);
    return hipGetLastError();
}

hipError_t launch_sum(const double* partials, int64_t count, double scale, double* out,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, partials, count, scale, out);
    return hipGetLastError();
}

hipError_t launch_scale_planes(double2* U, int m, int n, int p, int mode, hipStream_t st) {
    const int nw = p / 2 + 1;
    const int64_t count = static_cast<int64_t>(nw) * n * m;
    hipLaunchKernelGGL(k_scale_planes, dim3(blocks_for(count)), dim3(256), 0, st, U, m, n, p, nw, mode);
    return hipGetLastError();
}

hipError_t launch_scale_values(const double* in, double* out, int m, int n, int p, int mode,
                               hipStream_t st) {
    const int64_t total = static_cast<int64_t>(p) * n * m;
    hipLaunchKernelGGL(k_scale_values, dim3(blocks_for(total)), dim3(256), 0, st, in, out, m, n,
                       total, mode);
    return hipGetLastError();
}

}  // namespace cyl
