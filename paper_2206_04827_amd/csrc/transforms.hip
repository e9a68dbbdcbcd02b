// Value <-> coefficient transforms of Section 2 on CDNA4.
//
// theta: a real DFT of length p along the slowest axis; two neighbouring
//        r-lines are packed into one complex line (a + i b) and separated
//        from the Hermitian symmetry of the result.
// r, z : DCT-I of length M + 1 through a length-M DFT of the folded line
//        (see k_dct); complex lines carry the DCT of their real and
//        imaginary parts at once.
// Every DFT is a mixed-radix Stockham FFT in LDS whose butterflies run in
// registers (radices 16, 8, 4, 2 and 3, 5, 7, 11, 13, 15, 17); the twiddle
// table is staged in LDS once per workgroup.  One larger prime factor (up to
// 257) is taken as a direct first pass by all threads of a line together
// (prime_pass); lengths with other factors go through Bluestein's chirp-z
// identity with a power-of-two convolution.  The kernels are instantiated
// per radix mode (powers of two, mixed radices, led by a prime pass) and
// points per thread (8 or 16, chosen with the plan), so that each instance
// holds only the registers its passes need.
#include <type_traits>
#include <cstdlib>

#include "kernels.hpp"

namespace cyl {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ __forceinline__ double2 cmi(double2 a) { return make_double2(a.y, -a.x); }

// ---------------------------------------------------------------------------
// in-register DFTs (forward, exp(-2 pi i j k / R))
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dft2(double2& a, double2& b) {
    const double2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3) {
    const double2 a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = cmi(csub(x1, x3));
    x0 = cadd(a0, a2);
    x2 = csub(a0, a2);
    x1 = cadd(a1, a3);
    x3 = csub(a1, a3);
}

// cos and sin of 2 pi k / 16 for k = 0..9 (exp(-2 pi i k / 16) = (C - i S))
__constant__ double kC16[10] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                0.38268343236508977173, 0.0, -0.38268343236508977173,
                                -0.70710678118654752440, -0.92387953251128675613, -1.0,
                                -0.92387953251128675613};
__constant__ double kS16[10] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                                0.92387953251128675613, 1.0, 0.92387953251128675613,
                                0.70710678118654752440, 0.38268343236508977173, 0.0,
                                -0.38268343236508977173};

template <int R>
__device__ __forceinline__ void dft_reg(double2* x);

template <>
__device__ __forceinline__ void dft_reg<1>(double2*) {}
template <>
__device__ __forceinline__ void dft_reg<2>(double2* x) { dft2(x[0], x[1]); }
template <>
__device__ __forceinline__ void dft_reg<4>(double2* x) { dft4(x[0], x[1], x[2], x[3]); }

// 8 = 4 x 2: DFT-4 over even/odd halves, twiddles exp(-2 pi i k / 8), DFT-2.
template <>
__device__ __forceinline__ void dft_reg<8>(double2* x) {
    double2 e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
    dft4(e[0], e[1], e[2], e[3]);
    dft4(o[0], o[1], o[2], o[3]);
    const double h = 0.70710678118654752440;
    o[1] = make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));     // * (1 - i)/sqrt2
    o[2] = cmi(o[2]);
    o[3] = make_double2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));    // * (-1 - i)/sqrt2
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = cadd(e[k], o[k]);
        x[k + 4] = csub(e[k], o[k]);
    }
}

// 16 = 4 x 4 Cooley-Tukey with twiddles exp(-2 pi i j k / 16).
template <>
__device__ __forceinline__ void dft_reg<16>(double2* x) {
    double2 y[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        y[j][0] = x[j]; y[j][1] = x[j + 4]; y[j][2] = x[j + 8]; y[j][3] = x[j + 12];
        dft4(y[j][0], y[j][1], y[j][2], y[j][3]);
    }
#pragma unroll
    for (int j = 1; j < 4; ++j)
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            const int e = j * k;
            y[j][k] = cmul(y[j][k], make_double2(kC16[e], -kS16[e]));
        }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double2 a = y[0][k], b = y[1][k], c = y[2][k], d = y[3][k];
        dft4(a, b, c, d);
        x[k] = a; x[k + 4] = b; x[k + 8] = c; x[k + 12] = d;
    }
}

// (cos, sin)(2 pi e / R) for 0 <= e < R (0 <= e <= 8 for R = 15), correctly
// rounded; e is a compile-time constant wherever these are called.
template <int R>
__device__ __forceinline__ double2 root(int e);

#define CYL_ROOTS(R, ...)                                                         \
    template <>                                                                   \
    __device__ __forceinline__ double2 root<R>(int e) {                           \
        constexpr double cs[2][R / 2 + 2] = __VA_ARGS__;                          \
        return 2 * e <= R ? make_double2(cs[0][e], cs[1][e])                      \
                          : make_double2(cs[0][R - e], -cs[1][R - e]);            \
    }
CYL_ROOTS(3, {{1.0, -0.5, 0.0}, {0.0, 0.8660254037844386, 0.0}})
CYL_ROOTS(5, {{1.0, 0.30901699437494745, -0.8090169943749475, 0.0},
              {0.0, 0.9510565162951535, 0.5877852522924731, 0.0}})
CYL_ROOTS(7, {{1.0, 0.6234898018587335, -0.2225209339563144, -0.9009688679024191, 0.0},
              {0.0, 0.7818314824680298, 0.9749279121818236, 0.4338837391175581, 0.0}})
CYL_ROOTS(11, {{1.0, 0.8412535328311812, 0.41541501300188644, -0.14231483827328514,
                -0.6548607339452851, -0.9594929736144974, 0.0},
               {0.0, 0.5406408174555976, 0.9096319953545183, 0.9898214418809327,
                0.7557495743542583, 0.28173255684142967, 0.0}})
CYL_ROOTS(13, {{1.0, 0.8854560256532099, 0.5680647467311558, 0.12053668025532305,
                -0.3546048870425356, -0.7485107481711011, -0.970941817426052, 0.0},
               {0.0, 0.46472317204376856, 0.8229838658936564, 0.992708874098054,
                0.9350162426854148, 0.6631226582407952, 0.23931566428755777, 0.0}})
CYL_ROOTS(15, {{1.0, 0.9135454576426009, 0.6691306063588582, 0.30901699437494745,
                -0.10452846326765347, -0.5, -0.8090169943749475, -0.9781476007338057,
                -0.9781476007338057},
               {0.0, 0.4067366430758002, 0.7431448254773942, 0.9510565162951535,
                0.9945218953682733, 0.8660254037844386, 0.5877852522924731,
                0.20791169081775934, -0.20791169081775934}})
CYL_ROOTS(17, {{1.0, 0.9324722294043558, 0.7390089172206591, 0.44573835577653825,
                0.092268359463302, -0.2736629900720829, -0.6026346363792564,
                -0.8502171357296141, -0.9829730996839018, 0.0},
               {0.0, 0.3612416661871529, 0.6736956436465572, 0.8951632913550623,
                0.9957341762950345, 0.961825643172819, 0.7980172272802395,
                0.5264321628773558, 0.18374951781657034, 0.0}})
#undef CYL_ROOTS

// Odd prime R, directly: with a_j = x_j + x_{R-j}, b_j = x_j - x_{R-j}
// (1 <= j <= R/2), A_k = x_0 + sum_j a_j cos(2 pi j k / R) and
// B_k = sum_j b_j sin(2 pi j k / R): X_k = A_k - i B_k, X_{R-k} = A_k + i B_k.
template <int R>
__device__ __forceinline__ void dft_odd(double2* x) {
    constexpr int H = R / 2;
    double2 a[H], b[H];
    double2 x0 = x[0];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        a[j - 1] = cadd(x[j], x[R - j]);
        b[j - 1] = csub(x[j], x[R - j]);
        x0 = cadd(x0, a[j - 1]);
    }
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        double2 A = x[0], B = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const double2 w = root<R>((j * k) % R);
            A = make_double2(A.x + a[j - 1].x * w.x, A.y + a[j - 1].y * w.x);
            B = make_double2(B.x + b[j - 1].x * w.y, B.y + b[j - 1].y * w.y);
        }
        x[k] = make_double2(A.x + B.y, A.y - B.x);
        x[R - k] = make_double2(A.x - B.y, A.y + B.x);
    }
    x[0] = x0;
}

template <>
__device__ __forceinline__ void dft_reg<3>(double2* x) { dft_odd<3>(x); }
template <>
__device__ __forceinline__ void dft_reg<5>(double2* x) { dft_odd<5>(x); }
template <>
__device__ __forceinline__ void dft_reg<7>(double2* x) { dft_odd<7>(x); }
template <>
__device__ __forceinline__ void dft_reg<11>(double2* x) { dft_odd<11>(x); }
template <>
__device__ __forceinline__ void dft_reg<13>(double2* x) { dft_odd<13>(x); }
template <>
__device__ __forceinline__ void dft_reg<17>(double2* x) { dft_odd<17>(x); }

// 15 = 3 x 5 Cooley-Tukey with twiddles exp(-2 pi i j k / 15).
template <>
__device__ __forceinline__ void dft_reg<15>(double2* x) {
    double2 y[3][5];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int q = 0; q < 5; ++q) y[j][q] = x[j + 3 * q];
        dft_odd<5>(y[j]);
    }
#pragma unroll
    for (int j = 1; j < 3; ++j)
#pragma unroll
        for (int k = 1; k < 5; ++k) {
            const double2 w = root<15>(j * k);
            y[j][k] = cmul(y[j][k], make_double2(w.x, -w.y));
        }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double2 t[3] = {y[0][k], y[1][k], y[2][k]};
        dft_odd<3>(t);
        x[k] = t[0]; x[k + 5] = t[1]; x[k + 10] = t[2];
    }
}

// Line buffers in LDS skip one slot after every 16 points, so that the
// stride-16 writes of a radix-16 pass fall in distinct banks.
__device__ __forceinline__ int P(int i) { return i + (i >> 4); }

// One Stockham pass of radix R over a line of N points in LDS, already
// combined into sub-transforms of length Ls: butterfly b reads x[b + q N/R],
// scales input q by exp(-2 pi i k q / (R Ls)) (k = b mod Ls), and writes
// output r to (b - k) R + k + r Ls.  With T >= N / kP threads per line a
// thread runs at most ceil(kP / R) butterflies, and one for R >= 11 (the
// thread count is then at least N / R).  The pass's twiddles are stored as
// tw[k (R-1) + q - 1].
template <int R, bool kFirst, int kP>
__device__ __forceinline__ void fft_pass(double2* buf, int N, int Ls, const double2* tw, int t, int T) {
    constexpr int B = R >= 11 ? 1 : (kP + R - 1) / R;
    const int nb = N / R;
    const bool ls_pow2 = (Ls & (Ls - 1)) == 0;
    double2 x[B][R];
    int ob[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
        const int b = t + c * T;
        ob[c] = -1;
        if (b < nb) {
            const int k = ls_pow2 ? (b & (Ls - 1)) : b % Ls;
#pragma unroll
            for (int q = 0; q < R; ++q) x[c][q] = buf[P(b + q * nb)];
            if (!kFirst && Ls > 1) {
                const double2* tk = tw + k * (R - 1) - 1;
#pragma unroll
                for (int q = 1; q < R; ++q) x[c][q] = cmul(x[c][q], tk[q]);
            }
            dft_reg<R>(x[c]);
            ob[c] = (b - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < B; ++c) {
        if (ob[c] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[P(ob[c] + r * Ls)] = x[c][r];
        }
    }
    __syncthreads();
}

// First pass of a plan led by a prime radix R > 17, too many points for one
// thread's registers: the N/R sub-transforms (inputs x[b + q nb], q < R,
// nb = N/R) are computed by the threads of the line together.  Stage 1 forms,
// in place, a_j = x_j + x_{R-j} and d_j = x_j - x_{R-j} (1 <= j <= R/2).
// Stage 2 gives each thread one item: kPrimePassOutputs output pairs of one
// sub-transform,
//   X_r     = x_0 + sum_j a_j cos(2 pi j r / R) - i sum_j d_j sin(2 pi j r / R),
//   X_{R-r} = x_0 + sum_j a_j cos(2 pi j r / R) + i sum_j d_j sin(2 pi j r / R),
// or X_0 = x_0 + sum_j a_j.  The angles j r advance by rotation with
// exp(2 pi i r / R), restarted from the table every 16 steps (rounding error
// of at most 16 rotations); roots[m - 1] = (cos, sin)(2 pi m / R).  Outputs
// go to b R + r (the first Stockham pass).  Needs T >= nb (ceil(H / kPrimePassOutputs) + 1).
__device__ __forceinline__ void prime_pass(double2* buf, int N, int R, const double2* roots, int t, int T) {
    constexpr int RB = kPrimePassOutputs;
    const int nb = N / R, H = R / 2;
    for (int it = t; it < nb * H; it += T) {
        const int b = it / H, j = 1 + it % H;
        const double2 u = buf[P(b + j * nb)], v = buf[P(b + (R - j) * nb)];
        buf[P(b + j * nb)] = cadd(u, v);
        buf[P(b + (R - j) * nb)] = csub(u, v);
    }
    __syncthreads();
    const int ng = (H + RB - 1) / RB;
    double2 oa[RB], od[RB];
    int ob = -1, r0 = 0, cnt = 0;
    if (t < nb * (ng + 1)) {
        const int b = t / (ng + 1), g = t % (ng + 1);
        const double2* xa = buf;                 // a_j at b + j nb, d_j at b + (R - j) nb
        const double2 x0 = xa[P(b)];
        ob = b;
        if (g == ng) {                           // X_0
            double2 s0 = x0;
            for (int j = 1; j <= H; ++j) s0 = cadd(s0, xa[P(b + j * nb)]);
            oa[0] = s0;
            r0 = 0;
            cnt = 1;
        } else {
            r0 = 1 + g * RB;
            cnt = H - r0 + 1 < RB ? H - r0 + 1 : RB;
            double2 A[RB], B[RB], w[RB], st[RB];
            int m[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int r = r0 + i <= H ? r0 + i : r0;    // unused lanes of the item repeat r0
                A[i] = x0;
                B[i] = make_double2(0.0, 0.0);
                st[i] = roots[r - 1];
                m[i] = 0;
            }
            for (int j0 = 1; j0 <= H; j0 += 16) {
#pragma unroll
                for (int i = 0; i < RB; ++i) {        // restart: angle j0 r
                    const int r = r0 + i <= H ? r0 + i : r0;
                    m[i] = (j0 * r) % R;
                    w[i] = roots[m[i] - 1];
                }
                const int je = j0 + 16 <= H + 1 ? j0 + 16 : H + 1;
                for (int j = j0; j < je; ++j) {
                    const double2 a = xa[P(b + j * nb)], d = xa[P(b + (R - j) * nb)];
#pragma unroll
                    for (int i = 0; i < RB; ++i) {
                        A[i] = make_double2(A[i].x + a.x * w[i].x, A[i].y + a.y * w[i].x);
                        B[i] = make_double2(B[i].x + d.x * w[i].y, B[i].y + d.y * w[i].y);
                        w[i] = make_double2(w[i].x * st[i].x - w[i].y * st[i].y, w[i].x * st[i].y + w[i].y * st[i].x);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                oa[i] = make_double2(A[i].x + B[i].y, A[i].y - B[i].x);
                od[i] = make_double2(A[i].x - B[i].y, A[i].y + B[i].x);
            }
        }
    }
    __syncthreads();
    if (ob >= 0) {
        if (r0 == 0) {
            buf[P(ob * R)] = oa[0];
        } else {
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                if (i < cnt) {
                    buf[P(ob * R + r0 + i)] = oa[i];
                    buf[P(ob * R + R - r0 - i)] = od[i];
                }
            }
        }
    }
    __syncthreads();
}

// In-place forward FFT of the line of d.Nb points in LDS (all threads of the
// workgroup must call it: it contains barriers), one pass per entry of
// d.rad.  tw: the per-pass twiddle tables, concatenated in pass order
// (Nb - 1 entries).  kMode 0: powers of two only; 1: the radix plan of a
// directly transformed length, whose odd prime factor 7, 11, 13 or 17 (at
// most one) comes first, where no twiddles apply; 2: the same led by a prime
// pass (radix 19..257).  kP: points per thread (T >= Nb / kP).  Keeping each
// instance to the passes it needs keeps the kernels within their registers.
template <int kMode, int kP>
__device__ __forceinline__ void fft_lds(double2* buf, const DftDev& d, const double2* tw, int t, int T) {
    const int N = d.Nb;
    int Ls = 1;
    for (int p = 0; p < d.nrad; ++p) {
        const int R = d.rad[p];
        // opaque per pass: keeps the per-radix LDS addresses from being
        // hoisted out of this loop (and spilled across it)
        asm volatile("" : "+v"(t));
        if (kMode == 2 && p == 0 && R > 17) {
            prime_pass(buf, N, R, tw, t, T);
        } else if (kMode != 0 && p == 0) {
            switch (R) {
                case 16: fft_pass<16, true, kP>(buf, N, Ls, tw, t, T); break;
                case 8: fft_pass<8, true, kP>(buf, N, Ls, tw, t, T); break;
                case 4: fft_pass<4, true, kP>(buf, N, Ls, tw, t, T); break;
                case 2: fft_pass<2, true, kP>(buf, N, Ls, tw, t, T); break;
                case 3: fft_pass<3, true, kP>(buf, N, Ls, tw, t, T); break;
                case 5: fft_pass<5, true, kP>(buf, N, Ls, tw, t, T); break;
                case 7: fft_pass<7, true, kP>(buf, N, Ls, tw, t, T); break;
                case 11: fft_pass<11, true, kP>(buf, N, Ls, tw, t, T); break;
                case 13: fft_pass<13, true, kP>(buf, N, Ls, tw, t, T); break;
                case 15: fft_pass<15, true, kP>(buf, N, Ls, tw, t, T); break;
                default: fft_pass<17, true, kP>(buf, N, Ls, tw, t, T); break;
            }
        } else if (kMode != 0) {
            switch (R) {
                case 16: fft_pass<16, false, kP>(buf, N, Ls, tw, t, T); break;
                case 8: fft_pass<8, false, kP>(buf, N, Ls, tw, t, T); break;
                case 4: fft_pass<4, false, kP>(buf, N, Ls, tw, t, T); break;
                case 2: fft_pass<2, false, kP>(buf, N, Ls, tw, t, T); break;
                case 3: fft_pass<3, false, kP>(buf, N, Ls, tw, t, T); break;
                case 5: fft_pass<5, false, kP>(buf, N, Ls, tw, t, T); break;
                case 7: fft_pass<7, false, kP>(buf, N, Ls, tw, t, T); break;
                default: fft_pass<15, false, kP>(buf, N, Ls, tw, t, T); break;
            }
        } else {
            switch (R) {
                case 16: fft_pass<16, false, kP>(buf, N, Ls, tw, t, T); break;
                case 8: fft_pass<8, false, kP>(buf, N, Ls, tw, t, T); break;
                case 4: fft_pass<4, false, kP>(buf, N, Ls, tw, t, T); break;
                default: fft_pass<2, false, kP>(buf, N, Ls, tw, t, T); break;
            }
        }
        tw += Ls * (R - 1);
        Ls *= R;
    }
}

// DFT of the length-L line held (pre-multiplied by the chirp when Bluestein)
// in buf[0..Nb); leaves X_k, k < L, in buf[0..L).
// Every thread owns at most kP (8 or 16, the plan's points per thread)
// points of a line (T >= Nb / kP threads per line), so the pointwise loops
// below have a fixed trip count and issue all of their table loads before
// the first use.
template <int kMode, int kP>
__device__ __forceinline__ void dft_lds(double2* buf, const DftDev& d, const double2* tw, int t, int T) {
    fft_lds<kMode, kP>(buf, d, tw, t, T);
    if (kMode == 0 && d.bluestein) {
        double2 bh[kP];
#pragma unroll
        for (int c = 0; c < kP; ++c) {
            const int k = t + c * T;
            bh[c] = k < d.Nb ? d.bhat[k] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int c = 0; c < kP; ++c) {
            const int k = t + c * T;
            if (k < d.Nb) buf[P(k)] = cconj(cmul(buf[P(k)], bh[c]));
        }
        __syncthreads();
        fft_lds<0, kP>(buf, d, tw, t, T);
#pragma unroll
        for (int c = 0; c < kP; ++c) {
            const int k = t + c * T;
            bh[c] = k < d.L ? d.chirp[k] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int c = 0; c < kP; ++c) {
            const int k = t + c * T;
            if (k < d.L) buf[P(k)] = cmul(cconj(buf[P(k)]), bh[c]);
        }
        __syncthreads();
    }
}

// Padded line length in LDS (odd, so that lines in neighbouring lanes fall in
// distinct banks).
__host__ __device__ __forceinline__ int line_stride(int Nb) { return Nb + (Nb >> 4) + 1; }

__device__ __forceinline__ double2 load_chirped(double2 v, const DftDev& d, int n) {
    return d.bluestein ? cmul(v, d.chirp[n]) : v;
}

// Stage the twiddle table in LDS (shared by every line of the workgroup).
__device__ __forceinline__ void stage_twiddles(double2* tws, const DftDev& d) {
    for (int k0 = 0; k0 < d.Nb; k0 += 4 * blockDim.x) {
        double2 v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k = k0 + threadIdx.x + c * blockDim.x;
            v[c] = k < d.Nb ? d.tw[k] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k = k0 + threadIdx.x + c * blockDim.x;
            if (k < d.Nb) tws[k] = v[c];
        }
    }
}

template <bool kLineFast>
__device__ __forceinline__ void line_thread(int LPW, int TPL, int* li, int* t) {
    if (kLineFast) { *li = threadIdx.x % LPW; *t = threadIdx.x / LPW; }
    else           { *li = threadIdx.x / TPL; *t = threadIdx.x % TPL; }
}

// DCT-I of every line through a DFT of length M (not 2M).  With y = pre * in
// (M + 1 points) and F_k = sum_n w_n y_n cos(pi k n / M), w = 1/2 at both ends:
//   z_j = (y_j + y_{M-j}) / 2 - sin(pi j / M) (y_j - y_{M-j}),  j < M,
//   C = DFT_M(z),
//   F_{2k} = (C_k + C_{M-k}) / 2,
//   F_{2k+1} = F_1 + sum_{k'=1..k} (i/2) (C_{k'} - C_{M-k'}),
//   F_1 = sum_n w_n y_n cos(pi n / M),
// which holds for complex y (real and imaginary parts at once).  The odd
// outputs are a prefix sum: each thread scans a contiguous chunk, chunk
// totals meet in LDS.  out_k = post_k * 2 F_k.
// LDS: [twiddles: Nb][line 0: line_stride(Nb)][line 1] ...
// Workgroup b of G runs on XCD b mod 8 (round robin).  With xcd set, it takes
// line group (b mod 8) G/8 + min(b mod 8, G mod 8) + b / 8 instead of b (a
// permutation of 0..G-1): neighbouring groups then run on one XCD at about
// the same time, and cache lines that two groups share (strided lines whose
// group is not a whole number of 128-byte lines) are fetched into one L2.
__device__ __forceinline__ int64_t line_group(int xcd) {
    const unsigned b = blockIdx.x, G = gridDim.x;
    if (!xcd) return b;
    const unsigned x = b & 7u, rem = G & 7u;
    return static_cast<int64_t>(x) * (G >> 3) + (x < rem ? x : rem) + (b >> 3);
}

template <bool kLineFast, int kMode, int kP>
__global__ __launch_bounds__(512) void k_dct(const double2* in, double2* out, LineSet ls,
                                              int mlen, DftDev d,
                                              const double* __restrict__ pre,
                                              const double* __restrict__ post,
                                              const double2* __restrict__ fold, int TPL, int LPW, int xcd) {
    extern __shared__ double2 lds[];
    double2* tws = lds;
    int li, t;
    line_thread<kLineFast>(LPW, TPL, &li, &t);
    const int64_t line = line_group(xcd) * LPW + li;
    const int64_t nlines = static_cast<int64_t>(ls.n_outer) * ls.n_inner;
    const bool valid = line < nlines;
    int64_t base = 0;
    if (valid) base = (line / ls.n_inner) * ls.outer + (line % ls.n_inner) * ls.inner;
    double2* buf = lds + d.Nb + li * line_stride(d.Nb);
    stage_twiddles(tws, d);
    const int M = mlen - 1;
    // M + 1 <= Nb + 1 points: at most kP + 1 per thread
    constexpr int kIn = kP + 1;
    double2 y[kIn], fc[kIn];
    double ps[kIn];
#pragma unroll
    for (int c = 0; c < kIn; ++c) {
        const int s = t + c * TPL;
        const bool ok = s <= M;
        y[c] = (ok && valid) ? in[base + s * ls.elem] : make_double2(0.0, 0.0);
        ps[c] = ok ? pre[s] : 0.0;
        fc[c] = ok ? fold[s] : make_double2(0.0, 0.0);
    }
    double2 f1 = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < kIn; ++c) {
        const int s = t + c * TPL;
        if (s <= M) {
            y[c] = make_double2(y[c].x * ps[c], y[c].y * ps[c]);
            const double wc = ((s == 0 || s == M) ? 0.5 : 1.0) * fc[c].x;
            f1 = make_double2(f1.x + wc * y[c].x, f1.y + wc * y[c].y);
            buf[P(s)] = y[c];
        }
    }
    __syncthreads();
    double2 z[kP];
#pragma unroll
    for (int c = 0; c < kP; ++c) {
        const int j = t + c * TPL;
        if (j < M) {
            const double2 a = y[c], b = buf[P(M - j)];
            const double sj = fc[c].y;
            z[c] = make_double2(0.5 * (a.x + b.x) - sj * (a.x - b.x), 0.5 * (a.y + b.y) - sj * (a.y - b.y));
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kP; ++c) {
        const int j = t + c * TPL;
        if (j < M) buf[P(j)] = load_chirped(z[c], d, j);
    }
    for (int s = M + t; s < d.Nb; s += TPL) buf[P(s)] = make_double2(0.0, 0.0);
    __syncthreads();
    dft_lds<kMode, kP>(buf, d, tws, t, TPL);
    // even outputs (strided) and odd increments (contiguous chunk per thread)
    const int Ko = (M + 1) / 2;                 // odd outputs 1, 3, .., <= M
    const int Q = (Ko + TPL - 1) / TPL;
    double2 ev[kP / 2 + 1], dk[kP / 2 + 1];
#pragma unroll
    for (int c = 0; c < kP / 2 + 1; ++c) {
        const int k = t + c * TPL;
        ev[c] = make_double2(0.0, 0.0);
        if (2 * k <= M) {
            const double2 a = buf[P(k)], b = buf[P(k == 0 ? 0 : M - k)];
            ev[c] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
        }
    }
#pragma unroll
    for (int q = 0; q < kP / 2 + 1; ++q) {
        const int k = t * Q + q;
        dk[q] = make_double2(0.0, 0.0);
        if (q < Q && k >= 1 && k < Ko) {
            const double2 a = buf[P(k)], b = buf[P(M - k)];
            dk[q] = make_double2(-0.5 * (a.y - b.y), 0.5 * (a.x - b.x));      // (i/2)(C_k - C_{M-k})
        }
    }
#pragma unroll
    for (int q = 1; q < kP / 2 + 1; ++q) dk[q] = make_double2(dk[q].x + dk[q - 1].x, dk[q].y + dk[q - 1].y);
    __syncthreads();
    const double2 tot = dk[kP / 2];
    buf[P(t)] = tot;
    buf[P(TPL + t)] = f1;
    __syncthreads();
    double2 off = make_double2(0.0, 0.0), F1 = make_double2(0.0, 0.0);
    for (int u = 0; u < TPL; ++u) {
        const double2 a = buf[P(u)], b = buf[P(TPL + u)];
        if (u < t) off = make_double2(off.x + a.x, off.y + a.y);
        F1 = make_double2(F1.x + b.x, F1.y + b.y);
    }
    if constexpr (!kLineFast) {
        // threads along a contiguous line: even and odd outputs would leave in
        // two strided halves (partial cache lines); stage the line in LDS and
        // write it in order
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kP / 2 + 1; ++c) {
            const int k = t + c * TPL;
            if (2 * k <= M) {
                const double sc = 2.0 * post[2 * k];
                buf[P(2 * k)] = make_double2(sc * ev[c].x, sc * ev[c].y);
            }
        }
#pragma unroll
        for (int q = 0; q < kP / 2 + 1; ++q) {
            const int k = t * Q + q;
            if (q < Q && k < Ko) {
                const double sc = 2.0 * post[2 * k + 1];
                buf[P(2 * k + 1)] = make_double2(sc * (F1.x + off.x + dk[q].x), sc * (F1.y + off.y + dk[q].y));
            }
        }
        __syncthreads();
        if (valid)
            for (int s = t; s <= M; s += TPL) out[base + s * ls.elem] = buf[P(s)];
    } else if (valid) {
#pragma unroll
        for (int c = 0; c < kP / 2 + 1; ++c) {
            const int k = t + c * TPL;
            if (2 * k <= M) {
                const double sc = 2.0 * post[2 * k];
                out[base + (2 * k) * ls.elem] = make_double2(sc * ev[c].x, sc * ev[c].y);
            }
        }
#pragma unroll
        for (int q = 0; q < kP / 2 + 1; ++q) {
            const int k = t * Q + q;
            if (q < Q && k < Ko) {
                const double sc = 2.0 * post[2 * k + 1];
                out[base + (2 * k + 1) * ls.elem] =
                    make_double2(sc * (F1.x + off.x + dk[q].x), sc * (F1.y + off.y + dk[q].y));
            }
        }
    }
}

// values [p][n][m] (real) -> planes [p/2+1][n][m] (complex): theta DFT with the
// (-1)^w phase of theta_0 = -pi and the 1/p normalisation.
template <int kMode, int kP>
__global__ __launch_bounds__(512) void k_theta_fwd(const double* __restrict__ val,
                                                    double2* __restrict__ planes, int m, int n,
                                                    int p, DftDev d, int TPL, int LPW) {
    extern __shared__ double2 lds[];
    double2* tws = lds;
    int li, t;
    line_thread<true>(LPW, TPL, &li, &t);
    const int hm = (m + 1) / 2;
    const int64_t pair = static_cast<int64_t>(blockIdx.x) * LPW + li;
    const bool valid = pair < static_cast<int64_t>(n) * hm;
    const int k = valid ? static_cast<int>(pair / hm) : 0;
    const int j0 = valid ? 2 * static_cast<int>(pair % hm) : 0;
    const bool has1 = valid && (j0 + 1 < m);
    double2* buf = lds + d.Nb + li * line_stride(d.Nb);
    stage_twiddles(tws, d);
    // every load of the thread is issued before the first is used (p <= Nb
    // <= kP TPL), so the HBM latency is paid once per line, not per point
    double2 v[kP];
#pragma unroll
    for (int c = 0; c < kP; ++c) {
        const int l = t + c * TPL;
        const int64_t off = (static_cast<int64_t>(l) * n + k) * m + j0;
        v[c] = make_double2(valid && l < p ? val[off] : 0.0, has1 && l < p ? val[off + 1] : 0.0);
    }
#pragma unroll
    for (int c = 0; c < kP; ++c) {
        const int l = t + c * TPL;
        if (l < p) buf[P(l)] = load_chirped(v[c], d, l);
    }
    for (int l = p + t; l < d.Nb; l += TPL) buf[P(l)] = make_double2(0.0, 0.0);
    __syncthreads();
    dft_lds<kMode, kP>(buf, d, tws, t, TPL);
    const int nw = p / 2 + 1;
    const double invp = 1.0 / p;
    for (int w = t; w < nw; w += TPL) {
        const double2 Zw = buf[P(w)];
        const double2 Zm = buf[P((p - w) % p)];
        const double sc = (w & 1) ? -invp : invp;
        double2 A = make_double2(0.5 * (Zw.x + Zm.x) * sc, 0.5 * (Zw.y - Zm.y) * sc);
        double2 B = make_double2(0.5 * (Zw.y + Zm.y) * sc, -0.5 * (Zw.x - Zm.x) * sc);
        if (w == 0 || 2 * w == p) { A.y = 0.0; B.y = 0.0; }
        const int64_t off = (static_cast<int64_t>(w) * n + k) * m + j0;
        if (valid) planes[off] = A;
        if (has1) planes[off + 1] = B;
    }
}

// planes -> values: f_l = sum_w Y_w e^{+2 pi i w l / p}, Y_w = (-1)^w c_w and
// its Hermitian extension; two r-lines per complex inverse DFT.
template <int kMode, int kP>
__global__ __launch_bounds__(512) void k_theta_inv(const double2* __restrict__ planes,
                                                    double* __restrict__ val, int m, int n, int p,
                                                    DftDev d, int TPL, int LPW) {
    extern __shared__ double2 lds[];
    double2* tws = lds;
    int li, t;
    line_thread<true>(LPW, TPL, &li, &t);
    const int hm = (m + 1) / 2;
    const int64_t pair = static_cast<int64_t>(blockIdx.x) * LPW + li;
    const bool valid = pair < static_cast<int64_t>(n) * hm;
    const int k = valid ? static_cast<int>(pair / hm) : 0;
    const int j0 = valid ? 2 * static_cast<int>(pair % hm) : 0;
    const bool has1 = valid && (j0 + 1 < m);
    double2* buf = lds + d.Nb + li * line_stride(d.Nb);
    stage_twiddles(tws, d);
    // all loads first (as in k_theta_fwd)
    double2 va[kP], vb[kP];
#pragma unroll
    for (int c = 0; c < kP; ++c) {
        const int l = t + c * TPL;
        const int wq = (2 * l <= p) ? l : p - l;
        const int64_t off = (static_cast<int64_t>(wq) * n + k) * m + j0;
        va[c] = valid && l < p ? planes[off] : make_double2(0.0, 0.0);
        vb[c] = has1 && l < p ? planes[off + 1] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < kP; ++c) {
        const int l = t + c * TPL;
        if (l >= p) break;
        const int wq = (2 * l <= p) ? l : p - l;
        const bool cj = 2 * l > p;
        double2 ca = va[c], cb = vb[c];
        if (wq == 0 || 2 * wq == p) { ca.y = 0.0; cb.y = 0.0; }
        const double sg = (wq & 1) ? -1.0 : 1.0;
        if (cj) { ca.y = -ca.y; cb.y = -cb.y; }
        // Z = Ya + i Yb; the inverse DFT is conj(DFT(conj(Z)))
        const double2 Z = make_double2(sg * (ca.x - cb.y), sg * (ca.y + cb.x));
        buf[P(l)] = load_chirped(cconj(Z), d, l);
    }
    for (int l = p + t; l < d.Nb; l += TPL) buf[P(l)] = make_double2(0.0, 0.0);
    __syncthreads();
    dft_lds<kMode, kP>(buf, d, tws, t, TPL);
    for (int l = t; l < p; l += TPL) {
        const double2 z = cconj(buf[P(l)]);
        const int64_t off = (static_cast<int64_t>(l) * n + k) * m + j0;
        if (valid) val[off] = z.x;
        if (has1) val[off + 1] = z.y;
    }
}

// Threads per line: chosen with the radix plan (about Nb / 16).  Lines per
// workgroup: line_config below.
int env_knob(const char* name, int def) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : def;
}

void line_config(int Nb, int tpl, bool strided, int* TPL, int* LPW, int* threads, size_t* lds,
                 bool theta = false, int max_lines = 0) {
    // lines per workgroup: strided lines (theta, z) take up to kMaxLines lines
    // within an LDS budget (neighbouring lines are neighbouring in memory: 8
    // complex lines are one 128-byte cache line, so every load and store of a
    // workgroup covers whole lines; measured as fast as 32 lines at 256^3 and
    // 4% faster at 512^3, where 10 lines read each line twice);
    // contiguous lines (r) fill a workgroup of kThreads threads.  Read once
    // from the environment for A/B measurements.
    static const int kMaxLinesZ = env_knob("CYLSPEC_DCT_LINES", 8);
    static const int kMaxLinesTheta = env_knob("CYLSPEC_THETA_LINES", 8);
    const int kMaxLines = theta ? kMaxLinesTheta : (max_lines > 0 ? max_lines : kMaxLinesZ);
    static const int kBudget = env_knob("CYLSPEC_DCT_LDS_BUDGET", 150000);
    static const int kThreads = env_knob("CYLSPEC_DCT_THREADS", 256);
    *TPL = tpl;
    int l;
    if (strided) {
        l = static_cast<int>(kBudget / (static_cast<size_t>(line_stride(Nb)) * sizeof(double2)));
        if (l > kMaxLines) l = kMaxLines;
        if (l * *TPL < 64) l = (64 + *TPL - 1) / *TPL;
        if (l * *TPL > 512) l = 512 / *TPL;
    } else {
        l = *TPL >= kThreads ? 1 : kThreads / *TPL;
    }
    // the lines and the twiddle table must fit the CU's 160 KB of LDS
    while (l > 1 && (static_cast<size_t>(l) * line_stride(Nb) + Nb) * sizeof(double2) > 163840) --l;
    if (l < 1) l = 1;
    *LPW = l;
    *threads = l * *TPL;           // exactly LPW lines x TPL threads
    *lds = (static_cast<size_t>(*LPW) * line_stride(Nb) + Nb) * sizeof(double2);
}

// Kernel instance of a length (fft_lds): 0 powers of two (and Bluestein), 1
// mixed radices, 2 mixed radices led by a prime pass.
int dft_mode(const DftDev& d) {
    if (d.bluestein) return 0;
    if (d.nrad > 0 && d.rad[0] > 17) return 2;
    for (int i = 0; i < d.nrad; ++i)
        if (d.rad[i] != 16 && d.rad[i] != 8 && d.rad[i] != 4 && d.rad[i] != 2) return 1;
    return 0;
}

template <int V>
using IntC = std::integral_constant<int, V>;

// Calls f(IntC<mode>, IntC<points per thread>) for the instance of the
// length; a prime pass always runs with 16 points per thread.
template <typename F>
hipError_t dft_dispatch(const DftDev& d, F&& f) {
    const int mode = dft_mode(d);
    if (d.pts != 8 && d.pts != 16) return hipErrorInvalidValue;
    if (mode == 2) {
        if (d.pts != 16) return hipErrorInvalidValue;
        f(IntC<2>{}, IntC<16>{});
    } else if (mode == 1) {
        if (d.pts == 8) f(IntC<1>{}, IntC<8>{});
        else f(IntC<1>{}, IntC<16>{});
    } else {
        if (d.pts == 8) f(IntC<0>{}, IntC<8>{});
        else f(IntC<0>{}, IntC<16>{});
    }
    return hipSuccess;
}

template <typename K>
void raise_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

}  // namespace

hipError_t launch_theta_fwd(const double* values, double2* planes, int m, int n, int p,
                            const DftDev& d, hipStream_t s) {
    int TPL, LPW, threads;
    size_t lds;
    line_config(d.Nb, d.tpl, true, &TPL, &LPW, &threads, &lds, true);
    const int64_t lines = static_cast<int64_t>(n) * ((m + 1) / 2);
    const unsigned grid = static_cast<unsigned>((lines + LPW - 1) / LPW);
    const hipError_t e = dft_dispatch(d, [&](auto M, auto P) {
        constexpr int kM = decltype(M)::value, kP = decltype(P)::value;
        raise_lds(k_theta_fwd<kM, kP>, lds);
        hipLaunchKernelGGL((k_theta_fwd<kM, kP>), dim3(grid), dim3(threads), lds, s, values, planes, m, n, p, d, TPL,
                           LPW);
    });
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_theta_inv(const double2* planes, double* values, int m, int n, int p,
                            const DftDev& d, hipStream_t s) {
    int TPL, LPW, threads;
    size_t lds;
    line_config(d.Nb, d.tpl, true, &TPL, &LPW, &threads, &lds, true);
    const int64_t lines = static_cast<int64_t>(n) * ((m + 1) / 2);
    const unsigned grid = static_cast<unsigned>((lines + LPW - 1) / LPW);
    const hipError_t e = dft_dispatch(d, [&](auto M, auto P) {
        constexpr int kM = decltype(M)::value, kP = decltype(P)::value;
        raise_lds(k_theta_inv<kM, kP>, lds);
        hipLaunchKernelGGL((k_theta_inv<kM, kP>), dim3(grid), dim3(threads), lds, s, planes, values, m, n, p, d, TPL,
                           LPW);
    });
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_dct(const double2* in, double2* out, const LineSet& ls, int mlen,
                      bool contiguous_lines, const DftDev& d, const double* pre,
                      const double* post, const double2* fold, hipStream_t s, int max_lines) {
    int TPL, LPW, threads;
    size_t lds;
    line_config(d.Nb, d.tpl, !contiguous_lines, &TPL, &LPW, &threads, &lds, false, max_lines);
    const int64_t lines = static_cast<int64_t>(ls.n_outer) * ls.n_inner;
    const unsigned grid = static_cast<unsigned>((lines + LPW - 1) / LPW);
    // strided line groups that split 128-byte lines: XCD-aware group order
    static const int kXcd = env_knob("CYLSPEC_DCT_XCD", 1);
    const int xcd = (kXcd != 0 && !contiguous_lines && (LPW * 16) % 128 != 0) ? 1 : 0;
    const hipError_t e = dft_dispatch(d, [&](auto M, auto P) {
        constexpr int kM = decltype(M)::value, kP = decltype(P)::value;
        if (contiguous_lines) {
            raise_lds(k_dct<false, kM, kP>, lds);
            hipLaunchKernelGGL((k_dct<false, kM, kP>), dim3(grid), dim3(threads), lds, s, in, out, ls, mlen, d, pre,
                               post, fold, TPL, LPW, xcd);
        } else {
            raise_lds(k_dct<true, kM, kP>, lds);
            hipLaunchKernelGGL((k_dct<true, kM, kP>), dim3(grid), dim3(threads), lds, s, in, out, ls, mlen, d, pre,
                               post, fold, TPL, LPW, xcd);
        }
    });
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace cyl
