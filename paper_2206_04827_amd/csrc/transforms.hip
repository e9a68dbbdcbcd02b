// Value <-> coefficient transforms of Section 2 on CDNA4.
//
// theta: a real DFT of length p along the slowest axis; two neighbouring
//        r-lines are packed into one complex line (a + i b) and separated
//        from the Hermitian symmetry of the result.
// r, z : DCT-I of length M + 1 as the length-2M DFT of the even extension;
//        complex lines carry the DCT of their real and imaginary parts at
//        once.
// Every DFT is a power-of-two Stockham FFT (radix 4, one radix-2 stage when
// log2 N is odd) in LDS; other lengths go through Bluestein's chirp-z
// identity with a power-of-two convolution.
#include "kernels.hpp"

namespace cyl {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// In-place forward FFT (sign -1) of one line of length N (power of two) held
// in LDS, by TPL cooperating threads (t = 0..TPL-1).  Every thread of the
// workgroup must call it (it contains barriers).  Each radix-4 stage reads
// all inputs to registers, synchronises, then writes: one buffer suffices.
__device__ void fft_lds(double2* buf, int N, const double2* __restrict__ tw, int t, int TPL) {
    int Ls = 1;
    while (4 * Ls <= N) {
        const int nb = N >> 2;
        const int tstride = N / (4 * Ls);
        double2 y0[4], y1[4], y2[4], y3[4];
        int ob[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int b = t + c * TPL;
            ob[c] = -1;
            if (b < nb) {
                const int k = b & (Ls - 1);
                double2 x0 = buf[b], x1 = buf[b + nb], x2 = buf[b + 2 * nb], x3 = buf[b + 3 * nb];
                if (Ls > 1) {
                    const int e = k * tstride;
                    x1 = cmul(x1, tw[e]);
                    x2 = cmul(x2, tw[2 * e]);
                    x3 = cmul(x3, tw[3 * e]);
                }
                const double2 a0 = make_double2(x0.x + x2.x, x0.y + x2.y);
                const double2 a1 = make_double2(x0.x - x2.x, x0.y - x2.y);
                const double2 a2 = make_double2(x1.x + x3.x, x1.y + x3.y);
                const double2 a3 = make_double2(x1.x - x3.x, x1.y - x3.y);
                // (-i) * a3 = (a3.y, -a3.x)
                y0[c] = make_double2(a0.x + a2.x, a0.y + a2.y);
                y2[c] = make_double2(a0.x - a2.x, a0.y - a2.y);
                y1[c] = make_double2(a1.x + a3.y, a1.y - a3.x);
                y3[c] = make_double2(a1.x - a3.y, a1.y + a3.x);
                ob[c] = ((b - k) << 2) + k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (ob[c] >= 0) {
                buf[ob[c]] = y0[c];
                buf[ob[c] + Ls] = y1[c];
                buf[ob[c] + 2 * Ls] = y2[c];
                buf[ob[c] + 3 * Ls] = y3[c];
            }
        }
        __syncthreads();
        Ls <<= 2;
    }
    if (Ls < N) {  // final radix-2 stage, Ls = N / 2
        const int nb = N >> 1;
        double2 y0[8], y1[8];
        int ob[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int b = t + c * TPL;
            ob[c] = -1;
            if (b < nb) {
                const double2 x0 = buf[b];
                const double2 x1 = cmul(buf[b + nb], tw[b]);
                y0[c] = make_double2(x0.x + x1.x, x0.y + x1.y);
                y1[c] = make_double2(x0.x - x1.x, x0.y - x1.y);
                ob[c] = b;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (ob[c] >= 0) {
                buf[ob[c]] = y0[c];
                buf[ob[c] + Ls] = y1[c];
            }
        }
        __syncthreads();
    }
}

// DFT of the length-L line held (pre-multiplied by the chirp when Bluestein)
// in buf[0..Nb); leaves X_k, k < L, in buf[0..L).
__device__ void dft_lds(double2* buf, const DftDev& d, int t, int TPL) {
    fft_lds(buf, d.Nb, d.tw, t, TPL);
    if (d.bluestein) {
        for (int k = t; k < d.Nb; k += TPL) buf[k] = cconj(cmul(buf[k], d.bhat[k]));
        __syncthreads();
        fft_lds(buf, d.Nb, d.tw, t, TPL);
        for (int k = t; k < d.L; k += TPL) buf[k] = cmul(cconj(buf[k]), d.chirp[k]);
        __syncthreads();
    }
}

__device__ __forceinline__ double2 load_chirped(double2 v, const DftDev& d, int n) {
    return d.bluestein ? cmul(v, d.chirp[n]) : v;
}

template <bool kLineFast>
__device__ __forceinline__ void line_thread(int LPW, int TPL, int* li, int* t) {
    if (kLineFast) { *li = threadIdx.x % LPW; *t = threadIdx.x / LPW; }
    else           { *li = threadIdx.x / TPL; *t = threadIdx.x % TPL; }
}

template <bool kLineFast>
__global__ __launch_bounds__(kThreads) void k_dct(const double2* in, double2* out, LineSet ls,
                                                  int mlen, DftDev d,
                                                  const double* __restrict__ pre,
                                                  const double* __restrict__ post, int TPL, int LPW) {
    extern __shared__ double2 lds[];
    int li, t;
    line_thread<kLineFast>(LPW, TPL, &li, &t);
    const int64_t line = static_cast<int64_t>(blockIdx.x) * LPW + li;
    const int64_t nlines = static_cast<int64_t>(ls.n_outer) * ls.n_inner;
    const bool valid = line < nlines;
    int64_t base = 0;
    if (valid) base = (line / ls.n_inner) * ls.outer + (line % ls.n_inner) * ls.inner;
    double2* buf = lds + li * (d.Nb + 1);
    const int M = mlen - 1, L = 2 * M;
    for (int s = t; s <= M; s += TPL) {
        double2 v = make_double2(0.0, 0.0);
        if (valid) {
            v = in[base + s * ls.elem];
            const double ps = pre[s];
            v.x *= ps; v.y *= ps;
        }
        buf[s] = load_chirped(v, d, s);
        if (s >= 1 && s < M) buf[L - s] = load_chirped(v, d, L - s);
    }
    for (int s = L + t; s < d.Nb; s += TPL) buf[s] = make_double2(0.0, 0.0);
    __syncthreads();
    dft_lds(buf, d, t, TPL);
    if (valid) {
        for (int k = t; k <= M; k += TPL) {
            const double2 X = buf[k];
            const double ps = post[k];
            out[base + k * ls.elem] = make_double2(X.x * ps, X.y * ps);
        }
    }
}

// values [p][n][m] (real) -> planes [p/2+1][n][m] (complex): theta DFT with the
// (-1)^w phase of theta_0 = -pi and the 1/p normalisation.
__global__ __launch_bounds__(kThreads) void k_theta_fwd(const double* __restrict__ val,
                                                        double2* __restrict__ planes, int m,
                                                        int n, int p, DftDev d, int TPL, int LPW) {
    extern __shared__ double2 lds[];
    int li, t;
    line_thread<true>(LPW, TPL, &li, &t);
    const int hm = (m + 1) / 2;
    const int64_t pair = static_cast<int64_t>(blockIdx.x) * LPW + li;
    const bool valid = pair < static_cast<int64_t>(n) * hm;
    const int k = valid ? static_cast<int>(pair / hm) : 0;
    const int j0 = valid ? 2 * static_cast<int>(pair % hm) : 0;
    const bool has1 = valid && (j0 + 1 < m);
    double2* buf = lds + li * (d.Nb + 1);
    for (int l = t; l < p; l += TPL) {
        const int64_t off = (static_cast<int64_t>(l) * n + k) * m + j0;
        const double a = valid ? val[off] : 0.0;
        const double b = has1 ? val[off + 1] : 0.0;
        buf[l] = load_chirped(make_double2(a, b), d, l);
    }
    for (int l = p + t; l < d.Nb; l += TPL) buf[l] = make_double2(0.0, 0.0);
    __syncthreads();
    dft_lds(buf, d, t, TPL);
    const int nw = p / 2 + 1;
    const double invp = 1.0 / p;
    for (int w = t; w < nw; w += TPL) {
        const double2 Zw = buf[w];
        const double2 Zm = buf[(p - w) % p];
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
__global__ __launch_bounds__(kThreads) void k_theta_inv(const double2* __restrict__ planes,
                                                        double* __restrict__ val, int m, int n,
                                                        int p, DftDev d, int TPL, int LPW) {
    extern __shared__ double2 lds[];
    int li, t;
    line_thread<true>(LPW, TPL, &li, &t);
    const int hm = (m + 1) / 2;
    const int64_t pair = static_cast<int64_t>(blockIdx.x) * LPW + li;
    const bool valid = pair < static_cast<int64_t>(n) * hm;
    const int k = valid ? static_cast<int>(pair / hm) : 0;
    const int j0 = valid ? 2 * static_cast<int>(pair % hm) : 0;
    const bool has1 = valid && (j0 + 1 < m);
    double2* buf = lds + li * (d.Nb + 1);
    for (int l = t; l < p; l += TPL) {
        const int wq = (2 * l <= p) ? l : p - l;
        const bool cj = 2 * l > p;
        const int64_t off = (static_cast<int64_t>(wq) * n + k) * m + j0;
        double2 ca = valid ? planes[off] : make_double2(0.0, 0.0);
        double2 cb = has1 ? planes[off + 1] : make_double2(0.0, 0.0);
        if (wq == 0 || 2 * wq == p) { ca.y = 0.0; cb.y = 0.0; }
        const double sg = (wq & 1) ? -1.0 : 1.0;
        if (cj) { ca.y = -ca.y; cb.y = -cb.y; }
        // Z = Ya + i Yb; the inverse DFT is conj(DFT(conj(Z)))
        const double2 Z = make_double2(sg * (ca.x - cb.y), sg * (ca.y + cb.x));
        buf[l] = load_chirped(cconj(Z), d, l);
    }
    for (int l = p + t; l < d.Nb; l += TPL) buf[l] = make_double2(0.0, 0.0);
    __syncthreads();
    dft_lds(buf, d, t, TPL);
    for (int l = t; l < p; l += TPL) {
        const double2 z = cconj(buf[l]);
        const int64_t off = (static_cast<int64_t>(l) * n + k) * m + j0;
        if (valid) val[off] = z.x;
        if (has1) val[off + 1] = z.y;
    }
}

void line_config(int Nb, int* TPL, int* LPW, size_t* lds) {
    *TPL = Nb >= 16 ? Nb / 16 : 1;
    if (*TPL > kThreads) *TPL = kThreads;
    *LPW = kThreads / *TPL;
    *lds = static_cast<size_t>(*LPW) * (Nb + 1) * sizeof(double2);
}

}  // namespace

hipError_t launch_theta_fwd(const double* values, double2* planes, int m, int n, int p,
                            const DftDev& d, hipStream_t s) {
    int TPL, LPW;
    size_t lds;
    line_config(d.Nb, &TPL, &LPW, &lds);
    const int64_t lines = static_cast<int64_t>(n) * ((m + 1) / 2);
    const unsigned grid = static_cast<unsigned>((lines + LPW - 1) / LPW);
    hipLaunchKernelGGL(k_theta_fwd, dim3(grid), dim3(kThreads), lds, s, values, planes, m, n, p, d, TPL, LPW);
    return hipGetLastError();
}

hipError_t launch_theta_inv(const double2* planes, double* values, int m, int n, int p,
                            const DftDev& d, hipStream_t s) {
    int TPL, LPW;
    size_t lds;
    line_config(d.Nb, &TPL, &LPW, &lds);
    const int64_t lines = static_cast<int64_t>(n) * ((m + 1) / 2);
    const unsigned grid = static_cast<unsigned>((lines + LPW - 1) / LPW);
    hipLaunchKernelGGL(k_theta_inv, dim3(grid), dim3(kThreads), lds, s, planes, values, m, n, p, d, TPL, LPW);
    return hipGetLastError();
}

hipError_t launch_dct(const double2* in, double2* out, const LineSet& ls, int mlen,
                      bool contiguous_lines, const DftDev& d, const double* pre,
                      const double* post, hipStream_t s) {
    int TPL, LPW;
    size_t lds;
    line_config(d.Nb, &TPL, &LPW, &lds);
    const int64_t lines = static_cast<int64_t>(ls.n_outer) * ls.n_inner;
    const unsigned grid = static_cast<unsigned>((lines + LPW - 1) / LPW);
    if (contiguous_lines)
        hipLaunchKernelGGL(k_dct<false>, dim3(grid), dim3(kThreads), lds, s, in, out, ls, mlen, d, pre, post, TPL, LPW);
    else
        hipLaunchKernelGGL(k_dct<true>, dim3(grid), dim3(kThreads), lds, s, in, out, ls, mlen, d, pre, post, TPL, LPW);
    return hipGetLastError();
}

}  // namespace cyl
