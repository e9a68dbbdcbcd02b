// Horizontal (disk) Poisson solve of Section 4: Delta_h u = f, u = 0 at
// r = +-1, diagonalised in theta (DFT) and z (every Chebyshev z coefficient is
// its own problem, Delta_h having no z derivative).  Per (wavenumber slot,
// r parity, z coefficient k) one banded tau system in r:
//   [A_w Q]_tau x = [R^2 C02 f]_tau,   u = Q x   (Q: phi_j = T_(j+2) - T_j),
// within a parity a (1, 2)-banded no-pivot LU (host-built records) and a
// 5-tap right side.  One thread per line (both parities, real and imaginary
// parts together).
#include "kernels.hpp"

namespace cyl {
namespace {

constexpr int kDG = 4;         // rows per group (loads of the next group issued first)
constexpr int kDiskTaps = 5;   // right-side taps per row (same-parity T coefficients i-1 .. i+3)
constexpr int kDiskRec = 4;    // LU record per row: L, 1/d, U(i,i+1)/d, U(i,i+2)/d

// grid (ceil(n / 64), nw), 64 threads; one thread per (wavenumber slot, z
// coefficient) line runs both r parities as two interleaved recurrences, so
// that its reads and writes cover whole cache lines.  F, U: planes
// [nw][n][m] complex; U must not alias F.  The forward sweep keeps g in U's
// line, the backward sweep overwrites it with the T coefficients of u behind
// itself.
__global__ __launch_bounds__(64) void k_disk(const double2* __restrict__ F, double2* __restrict__ U,
                                             const double* __restrict__ lu, const double* __restrict__ taps,
                                             int m, int n, int rmax, int rows0, int rows1) {
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= n) return;
    const int w = blockIdx.y;
    const int nr[2] = {rows0, rows1};
    const int nmax = rows0 > rows1 ? rows0 : rows1;
    const int64_t line = (static_cast<int64_t>(w) * n + k) * m;
    const double2* f = F + line;
    double2* u = U + line;
    const double* tp[2] = {taps, taps + static_cast<int64_t>(rmax) * kDiskTaps};
    const double* rc[2] = {lu + static_cast<int64_t>(w) * 2 * rmax * kDiskRec,
                           lu + (static_cast<int64_t>(w) * 2 + 1) * rmax * kDiskRec};
    auto fc = [&](int q, int par) {
        const int j = 2 * q + par;
        return (q >= 0 && j < m) ? f[j] : make_double2(0.0, 0.0);
    };
    // forward: g_q = b_q - L_q g_(q-1), b_q = sum_s taps_(q,s) f_(q-1+s), per parity
    double2 fw[2][kDG + 4];                    // f_(q0-1) .. f_(q0+kDG+2) of each parity
#pragma unroll
    for (int i = 0; i < kDG + 4; ++i) { fw[0][i] = fc(i - 1, 0); fw[1][i] = fc(i - 1, 1); }
    double2 g[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    for (int q0 = 0; q0 < nmax; q0 += kDG) {
        double2 nx[2][kDG];
#pragma unroll
        for (int i = 0; i < kDG; ++i) { nx[0][i] = fc(q0 + kDG + 3 + i, 0); nx[1][i] = fc(q0 + kDG + 3 + i, 1); }
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            const int q = q0 + i;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                if (q < nr[par]) {
                    const double* t = tp[par] + q * kDiskTaps;
                    double2 bq = make_double2(0.0, 0.0);
#pragma unroll
                    for (int s = 0; s < kDiskTaps; ++s)
                        bq = make_double2(bq.x + t[s] * fw[par][i + s].x, bq.y + t[s] * fw[par][i + s].y);
                    const double l = rc[par][q * kDiskRec];
                    g[par] = make_double2(bq.x - l * g[par].x, bq.y - l * g[par].y);
                    u[2 * q + par] = g[par];
                }
            }
        }
#pragma unroll
        for (int par = 0; par < 2; ++par) {
#pragma unroll
            for (int i = 0; i < 4; ++i) fw[par][i] = fw[par][i + kDG];
#pragma unroll
            for (int i = 0; i < kDG; ++i) fw[par][4 + i] = nx[par][i];
        }
    }
    // backward: x_q = g_q / d_q - (U_(q,q+1)/d_q) x_(q+1) - (U_(q,q+2)/d_q) x_(q+2);
    // u_(q+1) = x_q - x_(q+1) (T coefficient 2(q+1) + par), u_0 = -x_0.  The
    // two parities run from their own last rows (the counts differ by at
    // most one): q counts down from nmax - 1 and a parity joins at its row.
    auto gl = [&](int q, int par) { return (q >= 0 && q < nr[par]) ? u[2 * q + par] : make_double2(0.0, 0.0); };
    double2 gc[2][kDG], x1[2], x2[2];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        x1[par] = make_double2(0.0, 0.0);
        x2[par] = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < kDG; ++i) gc[par][i] = gl(nmax - 1 - i, par);
    }
    for (int q0 = nmax - 1; q0 >= 0; q0 -= kDG) {
        double2 gn[2][kDG];
#pragma unroll
        for (int i = 0; i < kDG; ++i) { gn[0][i] = gl(q0 - kDG - i, 0); gn[1][i] = gl(q0 - kDG - i, 1); }
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            const int q = q0 - i;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                if (q >= 0 && q < nr[par]) {
                    const double* r = rc[par] + q * kDiskRec;
                    const double2 x = make_double2(r[1] * gc[par][i].x - r[2] * x1[par].x - r[3] * x2[par].x,
                                                   r[1] * gc[par][i].y - r[2] * x1[par].y - r[3] * x2[par].y);
                    if (2 * (q + 1) + par < m)
                        u[2 * (q + 1) + par] = make_double2(x.x - x1[par].x, x.y - x1[par].y);
                    x2[par] = x1[par];
                    x1[par] = x;
                }
            }
        }
#pragma unroll
        for (int par = 0; par < 2; ++par)
#pragma unroll
            for (int i = 0; i < kDG; ++i) gc[par][i] = gn[par][i];
    }
    u[0] = make_double2(-x1[0].x, -x1[0].y);
    if (m > 1) u[1] = make_double2(-x1[1].x, -x1[1].y);
}

}  // namespace

hipError_t launch_disk(const double2* F, double2* U, const double* lu, const double* taps, int m, int n,
                       int nw, int rmax, int rows0, int rows1, hipStream_t s) {
    if (n == 0 || nw == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + 63) / 64), static_cast<unsigned>(nw));
    hipLaunchKernelGGL(k_disk, grid, dim3(64), 0, s, F, U, lu, taps, m, n, rmax, rows0, rows1);
    return hipGetLastError();
}

}  // namespace cyl
