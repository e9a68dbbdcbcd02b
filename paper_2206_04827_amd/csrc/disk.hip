// Horizontal (disk) Poisson solve of Section 4: Delta_h u = f, u = 0 at
// r = +-1, diagonalised in theta (DFT) and z (every Chebyshev z coefficient is
// its own problem, Delta_h having no z derivative).  Per (wavenumber slot,
// r parity, z coefficient k) one banded tau system in r:
//   [A_w Q]_tau x = [R^2 C02 f]_tau,   u = Q x   (Q: phi_j = T_(j+2) - T_j),
// within a parity a (1, 2)-banded no-pivot LU (host-built records) and a
// 5-tap right side.  One thread per line and parity (real and imaginary parts
// together), the two parities of a line in neighbouring lanes.
#include "kernels.hpp"

namespace cyl {
namespace {

constexpr int kDG = 8;         // rows per group (loads of the next group issued first)
constexpr int kDiskTaps = 5;   // right-side taps per row (same-parity T coefficients i-1 .. i+3)
constexpr int kDiskRec = 4;    // LU record per row: L, 1/d, U(i,i+1)/d, U(i,i+2)/d

// grid (ceil(n / 32), nw), 64 threads: lane 2c + par runs r parity par of
// the (wavenumber slot, z coefficient) line c of the workgroup, so the two
// lanes of a line read and write the two halves of the same 32-byte pieces in
// one instruction (whole cache lines per wave) while each recurrence is half
// as long as a line.  F, U: planes [nw][n][m] complex; U must not alias F.
// The forward sweep keeps g in U's line, the backward sweep overwrites it
// with the T coefficients of u behind itself.
__global__ __launch_bounds__(64) void k_disk(const double2* __restrict__ F, double2* __restrict__ U,
                                             const double* __restrict__ lu, const double* __restrict__ taps,
                                             int m, int n, int rmax, int rows0, int rows1) {
    const int k = blockIdx.x * 32 + (threadIdx.x >> 1);
    const int par = threadIdx.x & 1;
    if (k >= n) return;
    const int w = blockIdx.y;
    const int nr = par ? rows1 : rows0;
    const int64_t line = (static_cast<int64_t>(w) * n + k) * m;
    const double2* f = F + line;
    double2* u = U + line;
    const double* tp = taps + static_cast<int64_t>(par) * rmax * kDiskTaps;
    const double* rc = lu + (static_cast<int64_t>(w) * 2 + par) * rmax * kDiskRec;
    auto fc = [&](int q) {
        const int j = 2 * q + par;
        return (q >= 0 && j < m) ? f[j] : make_double2(0.0, 0.0);
    };
    // forward: g_q = b_q - L_q g_(q-1), b_q = sum_s taps_(q,s) f_(q-1+s)
    double2 fw[kDG + 4];                       // f_(q0-1) .. f_(q0+kDG+2)
#pragma unroll
    for (int i = 0; i < kDG + 4; ++i) fw[i] = fc(i - 1);
    double2 g = make_double2(0.0, 0.0);
    for (int q0 = 0; q0 < nr; q0 += kDG) {
        double2 nx[kDG];
#pragma unroll
        for (int i = 0; i < kDG; ++i) nx[i] = fc(q0 + kDG + 3 + i);
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            const int q = q0 + i;
            if (q < nr) {
                const double* t = tp + q * kDiskTaps;
                double2 bq = make_double2(0.0, 0.0);
#pragma unroll
                for (int s = 0; s < kDiskTaps; ++s)
                    bq = make_double2(bq.x + t[s] * fw[i + s].x, bq.y + t[s] * fw[i + s].y);
                const double l = rc[q * kDiskRec];
                g = make_double2(bq.x - l * g.x, bq.y - l * g.y);
                u[2 * q + par] = g;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) fw[i] = fw[i + kDG];
#pragma unroll
        for (int i = 0; i < kDG; ++i) fw[4 + i] = nx[i];
    }
    // backward: x_q = g_q / d_q - (U_(q,q+1)/d_q) x_(q+1) - (U_(q,q+2)/d_q) x_(q+2);
    // u_(q+1) = x_q - x_(q+1) (T coefficient 2(q+1) + par), u_par = -x_0
    auto gl = [&](int q) { return (q >= 0 && q < nr) ? u[2 * q + par] : make_double2(0.0, 0.0); };
    double2 gc[kDG], x1 = make_double2(0.0, 0.0), x2 = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < kDG; ++i) gc[i] = gl(nr - 1 - i);
    for (int q0 = nr - 1; q0 >= 0; q0 -= kDG) {
        double2 gn[kDG];
#pragma unroll
        for (int i = 0; i < kDG; ++i) gn[i] = gl(q0 - kDG - i);
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            const int q = q0 - i;
            if (q >= 0) {
                const double* r = rc + q * kDiskRec;
                const double2 x = make_double2(r[1] * gc[i].x - r[2] * x1.x - r[3] * x2.x,
                                               r[1] * gc[i].y - r[2] * x1.y - r[3] * x2.y);
                if (2 * (q + 1) + par < m) u[2 * (q + 1) + par] = make_double2(x.x - x1.x, x.y - x1.y);
                x2 = x1;
                x1 = x;
            }
        }
#pragma unroll
        for (int i = 0; i < kDG; ++i) gc[i] = gn[i];
    }
    if (par < m) u[par] = make_double2(-x1.x, -x1.y);
}

}  // namespace

hipError_t launch_disk(const double2* F, double2* U, const double* lu, const double* taps, int m, int n,
                       int nw, int rmax, int rows0, int rows1, hipStream_t s) {
    if (n == 0 || nw == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + 31) / 32), static_cast<unsigned>(nw));
    hipLaunchKernelGGL(k_disk, grid, dim3(64), 0, s, F, U, lu, taps, m, n, rmax, rows0, rows1);
    return hipGetLastError();
}

}  // namespace cyl
