// Horizontal (disk) Poisson solve of Section 4: Delta_h u = f, u = 0 at
// r = +-1, diagonalised in theta (DFT) and z (every Chebyshev z coefficient is
// its own problem, Delta_h having no z derivative).  Per (wavenumber slot,
// r parity, z coefficient k) one banded tau system in r:
//   [A_w Q]_tau x = [R^2 C02 f]_tau,   u = Q x   (Q: phi_j = T_(j+2) - T_j),
// within a parity a (1, 2)-banded no-pivot LU (host-built records) and a
// 5-tap right side.  The poloidal-toroidal decomposition runs the same
// solve with the curl right side of its lambda potential.  One thread per line and parity (real and imaginary parts
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
// kPT (poloidal-toroidal decomposition, Section 4): the right side is the
// r^2-weighted curl -(PTa F) + i w (PTb F2) of F = V_theta, F2 = V_r, whose
// coefficients of the other r parity feed each row (w taken as 0 in the slot
// wnyq, the Nyquist mode); otherwise it is scale * (R^2 C02 F).
template <bool kPT>
__global__ __launch_bounds__(64) void k_disk(const double2* __restrict__ F, const double2* __restrict__ F2,
                                             double2* __restrict__ U, const double* __restrict__ lu,
                                             const double* __restrict__ taps, int m, int n, int rmax,
                                             int rows0, int rows1, double scale, int wnyq) {
    constexpr int NT = kPT ? 2 * kDiskTaps : kDiskTaps;   // taps per row
    const int k = blockIdx.x * 32 + (threadIdx.x >> 1);
    const int par = threadIdx.x & 1;
    if (k >= n) return;
    const int w = blockIdx.y;
    const int nr = par ? rows1 : rows0;
    const int src = kPT ? 1 - par : par;            // r parity of the right side's inputs
    const int64_t line = (static_cast<int64_t>(w) * n + k) * m;
    const double2* f = F + line;
    const double2* f2 = kPT ? F2 + line : nullptr;
    double2* u = U + line;
    const double* tp = taps + static_cast<int64_t>(par) * rmax * NT;
    const double* rc = lu + (static_cast<int64_t>(w) * 2 + par) * rmax * kDiskRec;
    const double wd = (kPT && w != wnyq) ? static_cast<double>(w) : 0.0;
    auto fc = [&](const double2* a, int q) {
        const int j = 2 * q + src;
        return (q >= 0 && j < m) ? a[j] : make_double2(0.0, 0.0);
    };
    // forward: g_q = b_q - L_q g_(q-1), b_q from the taps on f_(q-1) .. f_(q+3)
    double2 fw[kDG + 4], hw[kPT ? kDG + 4 : 1];     // f (and f2) at q0-1 .. q0+kDG+2
#pragma unroll
    for (int i = 0; i < kDG + 4; ++i) {
        fw[i] = fc(f, i - 1);
        if constexpr (kPT) hw[i] = fc(f2, i - 1);
    }
    double2 g = make_double2(0.0, 0.0);
    for (int q0 = 0; q0 < nr; q0 += kDG) {
        double2 nx[kDG], nh[kPT ? kDG : 1];
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            nx[i] = fc(f, q0 + kDG + 3 + i);
            if constexpr (kPT) nh[i] = fc(f2, q0 + kDG + 3 + i);
        }
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            const int q = q0 + i;
            if (q < nr) {
                const double* t = tp + q * NT;
                double2 bq = make_double2(0.0, 0.0);
#pragma unroll
                for (int s = 0; s < kDiskTaps; ++s)
                    bq = make_double2(bq.x + t[s] * fw[i + s].x, bq.y + t[s] * fw[i + s].y);
                if constexpr (kPT) {
                    double2 cq = make_double2(0.0, 0.0);
#pragma unroll
                    for (int s = 0; s < kDiskTaps; ++s)
                        cq = make_double2(cq.x + t[kDiskTaps + s] * hw[i + s].x,
                                          cq.y + t[kDiskTaps + s] * hw[i + s].y);
                    bq = make_double2(-bq.x - wd * cq.y, -bq.y + wd * cq.x);
                } else {
                    bq = make_double2(scale * bq.x, scale * bq.y);
                }
                const double l = rc[q * kDiskRec];
                g = make_double2(bq.x - l * g.x, bq.y - l * g.y);
                u[2 * q + par] = g;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            fw[i] = fw[i + kDG];
            if constexpr (kPT) hw[i] = hw[i + kDG];
        }
#pragma unroll
        for (int i = 0; i < kDG; ++i) {
            fw[4 + i] = nx[i];
            if constexpr (kPT) hw[4 + i] = nh[i];
        }
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
                       int nw, int rmax, int rows0, int rows1, hipStream_t s, double scale) {
    if (n == 0 || nw == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + 31) / 32), static_cast<unsigned>(nw));
    hipLaunchKernelGGL(k_disk<false>, grid, dim3(64), 0, s, F, nullptr, U, lu, taps, m, n, rmax, rows0, rows1,
                       scale, -1);
    return hipGetLastError();
}

hipError_t launch_disk_pt(const double2* Vt, const double2* Vr, double2* U, const double* lu,
                          const double* pt_taps, int m, int n, int nw, int rmax, int rows0, int rows1, int wnyq,
                          hipStream_t s) {
    if (n == 0 || nw == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + 31) / 32), static_cast<unsigned>(nw));
    hipLaunchKernelGGL(k_disk<true>, grid, dim3(64), 0, s, Vt, Vr, U, lu, pt_taps, m, n, rmax, rows0, rows1,
                       1.0, wnyq);
    return hipGetLastError();
}

}  // namespace cyl
