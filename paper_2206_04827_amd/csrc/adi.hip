// Per-mode Sylvester solves on CDNA4: tau right-hand side, ADI (Algorithm 1),
// operator application (residuals, heat history), recombination to T
// coefficients, heat right-hand side and norms.
//
// ADI (Section 3, Algorithm 1, with the sign and shift-role readings of the
// library): for A X B + C X D = E with shifts u_j in [c, d] and v_j in [a, b],
// each iteration is carried as two line sweeps over a parity block:
//
//   r-pass (one thread per column, a line along r):
//        Z = (u_j C - A)^{-1} [ (v_j C - A) W - (v_j - u_j) E ]
//   z-pass (one thread per row, a line along z):
//        X = Z (v_j B + D)^{-1},   W = X (u_{j+1} B + D)
//
// with W_0 = 0.  Here Z = X_{j+1} (v_j B + D) and W = X_j (u_j B + D); the
// first equation is step 1 of Algorithm 1 with X_{j+1/2} B eliminated through
// step 2 (substitute (u C - A) Y = C W - E into Z = C^{-1}((v C - A) Y + E)).
// Both sweeps work in place: the forward elimination overwrites the line with
// its intermediate, the back substitution with the result, and the sliding
// register windows hold the few neighbours still needed.
#include "kernels.hpp"

namespace cyl {
namespace {

constexpr int G = 8;          // rows per software-pipelined group
constexpr int kRRec = 12;
constexpr int kZRec = 8;

// r-pass on column k (stride ld between rows) of a block with me rows.
// RC: kRRec records per row; Ecol: E + k with row stride ne.
__device__ __forceinline__ void adi_rpass(double* S, int ld, int me, int k,
                                          const double* RC, const double* __restrict__ Ecol,
                                          int ne, double vmu) {
    // forward elimination: g_i = h_i - L_{i,i-1} g_{i-1} - L_{i,i-2} g_{i-2},
    // h = (v C - A) w - (v - u) e.
    double wv[14];                 // rows i0-2 .. i0+11 of W
    wv[0] = 0.0; wv[1] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[2 + q] = (q < me) ? S[q * ld + k] : 0.0;
    double eb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) eb[q] = (q < me) ? Ecol[static_cast<int64_t>(q) * ne] : 0.0;
    double g1 = 0.0, g2 = 0.0;
    for (int i0 = 0; i0 < me; i0 += G) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = i0 + 4 + q;
            wv[6 + q] = (r < me) ? S[r * ld + k] : 0.0;
        }
        double en[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int r = i0 + G + q;
            en[q] = (r < me) ? Ecol[static_cast<int64_t>(r) * ne] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int i = i0 + q;
            if (i < me) {
                const double* rc = RC + i * kRRec;
                double h = rc[0] * wv[q] + rc[1] * wv[q + 1] + rc[2] * wv[q + 2] +
                           rc[3] * wv[q + 3] + rc[4] * wv[q + 4] + rc[5] * wv[q + 5] - vmu * eb[q];
                h -= rc[6] * g2;
                const double g = h - rc[7] * g1;
                S[i * ld + k] = g;
                g2 = g1;
                g1 = g;
            }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) wv[q] = wv[8 + q];
#pragma unroll
        for (int q = 0; q < G; ++q) eb[q] = en[q];
    }
    // back substitution: z_i = dinv_i g_i - sum_t (dinv_i U_{i,i+t}) z_{i+t}
    const int ngr = (me + G - 1) / G;
    double gb[G];
    {
        const int i0 = (ngr - 1) * G;
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = (i0 + q < me) ? S[(i0 + q) * ld + k] : 0.0;
    }
    double z1 = 0.0, z2 = 0.0, z3 = 0.0;
    for (int gi = ngr - 1; gi >= 0; --gi) {
        const int i0 = gi * G;
        double gn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int r = i0 - G + q;
            gn[q] = (r >= 0) ? S[r * ld + k] : 0.0;
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const int i = i0 + q;
            if (i < me) {
                const double* rc = RC + i * kRRec;
                const double t = rc[8] * gb[q] - rc[11] * z3 - rc[10] * z2;
                const double z = t - rc[9] * z1;
                S[i * ld + k] = z;
                z3 = z2; z2 = z1; z1 = z;
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
}

// z-pass on one row (contiguous, ne entries).  ZC: kZRec records per column.
__device__ __forceinline__ void adi_zpass(double* row, int ne, const double* ZC, bool last) {
    // forward: g_k = z_k - L_k g_{k-1}
    double zb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) zb[q] = (q < ne) ? row[q] : 0.0;
    double gp = 0.0;
    for (int k0 = 0; k0 < ne; k0 += G) {
        double zn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) zn[q] = (k0 + G + q < ne) ? row[k0 + G + q] : 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int k = k0 + q;
            if (k < ne) {
                const double g = zb[q] - ZC[k * kZRec] * gp;
                row[k] = g;
                gp = g;
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) zb[q] = zn[q];
    }
    // back substitution x_k = dinv_k g_k - U1 x_{k+1} - U2 x_{k+2}, and unless
    // this is the last iteration, w_{k+1} = sum_t P_{k+1,t} x_{k+t}.
    const int ngr = (ne + G - 1) / G;
    double gb[G];
    {
        const int k0 = (ngr - 1) * G;
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = (k0 + q < ne) ? row[k0 + q] : 0.0;
    }
    double x1 = 0.0, x2 = 0.0, x3 = 0.0;
    for (int gi = ngr - 1; gi >= 0; --gi) {
        const int k0 = gi * G;
        double gn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int r = k0 - G + q;
            gn[q] = (r >= 0) ? row[r] : 0.0;
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const int k = k0 + q;
            if (k < ne) {
                const double* zc = ZC + k * kZRec;
                const double x = zc[1] * gb[q] - zc[3] * x2 - zc[2] * x1;
                if (last) {
                    row[k] = x;
                } else if (k + 1 < ne) {
                    const double* zn = zc + kZRec;
                    row[k + 1] = zn[4] * x + zn[5] * x1 + zn[6] * x2 + zn[7] * x3;
                }
                x3 = x2; x2 = x1; x1 = x;
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
    if (!last) row[0] = ZC[5] * x1 + ZC[6] * x2 + ZC[7] * x3;
}

// One workgroup per parity block, all J iterations.  kLDS: block state and
// the current shift's coefficient records live in LDS; otherwise the state
// lives in `state` (same offsets as E) and records are read from the tables.
template <bool kLDS>
__device__ __forceinline__ void adi_block(double* sm, const BlockDesc* __restrict__ blocks,
                                          const double* __restrict__ E, double* X,
                                          double* state, const double* __restrict__ rtab,
                                          const double* __restrict__ ztab,
                                          const double* __restrict__ vmu, int accumulate) {
    const BlockDesc bd = blocks[blockIdx.x];
    const int me = bd.me, ne = bd.ne;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ld = kLDS ? (ne | 1) : ne;
    double* S = kLDS ? sm : state + bd.eoff;
    double* RCs = sm + me * ld;
    double* ZCs = RCs + me * kRRec;
    for (int idx = tid; idx < me * ld; idx += nt) S[idx] = 0.0;
    const double* Eb = E + bd.eoff;
    for (int j = 0; j < bd.J; ++j) {
        const double* rsrc = rtab + bd.rbase + j * bd.rstride;
        const double* zsrc = ztab + bd.zbase + j * bd.zstride;
        const double* RC;
        const double* ZC;
        __syncthreads();
        if (kLDS) {
            for (int idx = tid; idx < me * kRRec; idx += nt) RCs[idx] = rsrc[idx];
            for (int idx = tid; idx < ne * kZRec; idx += nt) ZCs[idx] = zsrc[idx];
            __syncthreads();
            RC = RCs;
            ZC = ZCs;
        } else {
            RC = rsrc;
            ZC = zsrc;
        }
        const double vm = vmu[bd.soff + j];
        if (tid < ne) adi_rpass(S, ld, me, tid, RC, Eb + tid, ne, vm);
        __syncthreads();
        if (tid < me) adi_zpass(S + tid * ld, ne, ZC, j == bd.J - 1);
    }
    __syncthreads();
    double* Xb = X + bd.eoff;
    for (int idx = tid; idx < me * ne; idx += nt) {
        const int i = idx / ne, k = idx - i * ne;
        const double v = S[i * ld + k];
        Xb[idx] = accumulate ? Xb[idx] + v : v;
    }
}

__global__ __launch_bounds__(256) void k_adi_lds(const BlockDesc* __restrict__ blocks,
                                                 const double* __restrict__ E, double* X,
                                                 double* state, const double* __restrict__ rtab,
                                                 const double* __restrict__ ztab,
                                                 const double* __restrict__ vmu, int accumulate) {
    extern __shared__ double sm[];
    adi_block<true>(sm, blocks, E, X, state, rtab, ztab, vmu, accumulate);
}

__global__ __launch_bounds__(1024) void k_adi_global(const BlockDesc* __restrict__ blocks,
                                                     const double* __restrict__ E, double* X,
                                                     double* state,
                                                     const double* __restrict__ rtab,
                                                     const double* __restrict__ ztab,
                                                     const double* __restrict__ vmu,
                                                     int accumulate) {
    adi_block<false>(nullptr, blocks, E, X, state, rtab, ztab, vmu, accumulate);
}

// ---------------------------------------------------------------------------
// tau right-hand side (eq. HelmholtzMatEqn, right side, with r^2 weighting):
//   E = sF [R2 (F + cL L) C02^T]_tau + sL [A_w L C02^T + R2 L D2^T]_tau
// written into the parity blocks of each real mode plane (L may be NULL).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rhs(const double2* __restrict__ F,
                                             const double2* __restrict__ L, double sF, double cL,
                                             double sL, double* __restrict__ E,
                                             const BlockDesc* __restrict__ blocks, int m, int n,
                                             RhsTables t) {
    const int plane = blockIdx.y;
    const int mi = m - 2, ni = n - 2;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(mi) * ni) return;
    const int i = static_cast<int>(e % mi), k = static_cast<int>(e / mi);
    const BlockDesc b0 = blocks[4 * plane];
    const int w = b0.w, part = b0.part;
    const double2* Fw = F + static_cast<int64_t>(w) * n * m;
    const double2* Lw = L ? L + static_cast<int64_t>(w) * n * m : nullptr;
    auto comp = [part](double2 v) { return part ? v.y : v.x; };
    const double* c02 = t.c02 + 3 * k;
    const double* r2 = t.r2 + 5 * i;
    double acc = 0.0;
#pragma unroll
    for (int ta = 0; ta < 5; ++ta) {
        const int a = i - 2 + 2 * ta;
        if (a < 0 || a >= m || r2[ta] == 0.0) continue;
        double fz = 0.0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int l = k + 2 * s;
            if (l >= n) continue;
            const int64_t o = static_cast<int64_t>(l) * m + a;
            double fv = comp(Fw[o]);
            if (Lw != nullptr && cL != 0.0) fv += cL * comp(Lw[o]);
            fz += c02[s] * fv;
        }
        acc += r2[ta] * fz;
    }
    acc *= sF;
    if (Lw != nullptr && sL != 0.0) {
        const double ww = static_cast<double>(w) * w;
        const double* a0 = t.a0 + 4 * i;
        const double* s10 = t.s10 + 4 * i;
        double lacc = 0.0;
#pragma unroll
        for (int ta = 0; ta < 4; ++ta) {
            const int a = i - 2 + 2 * ta;
            const double aw = a0[ta] - ww * s10[ta];
            if (a < 0 || a >= m || aw == 0.0) continue;
            double lc = 0.0;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int l = k + 2 * s;
                if (l < n) lc += c02[s] * comp(Lw[static_cast<int64_t>(l) * m + a]);
            }
            lacc += aw * lc;
        }
        const double d2 = t.d2[k];
#pragma unroll
        for (int ta = 0; ta < 5; ++ta) {
            const int a = i - 2 + 2 * ta;
            if (a < 0 || a >= m || r2[ta] == 0.0) continue;
            lacc += r2[ta] * d2 * comp(Lw[static_cast<int64_t>(k + 2) * m + a]);
        }
        acc += sL * lacc;
    }
    const BlockDesc bd = blocks[4 * plane + 2 * (i & 1) + (k & 1)];
    E[bd.eoff + static_cast<int64_t>(i >> 1) * bd.ne + (k >> 1)] = acc;
}

// ---------------------------------------------------------------------------
// recombination U = Q_m Xt Q_n^T (+ L) into complex coefficient planes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double xt_at(const double* X, const BlockDesc* blocks, int plane,
                                        int i, int k, int mi, int ni) {
    if (plane < 0 || i < 0 || k < 0 || i >= mi || k >= ni) return 0.0;
    const BlockDesc& bd = blocks[4 * plane + 2 * (i & 1) + (k & 1)];
    return X[bd.eoff + static_cast<int64_t>(i >> 1) * bd.ne + (k >> 1)];
}

__global__ __launch_bounds__(256) void k_recombine(const double* __restrict__ X,
                                                   const double2* __restrict__ L,
                                                   double2* __restrict__ planes,
                                                   const int* __restrict__ plane_of,
                                                   const BlockDesc* __restrict__ blocks, int m,
                                                   int n) {
    const int w = blockIdx.y;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(m) * n) return;
    const int a = static_cast<int>(e % m), l = static_cast<int>(e / m);
    const int mi = m - 2, ni = n - 2;
    double v[2];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int pl = plane_of[2 * w + part];
        v[part] = xt_at(X, blocks, pl, a - 2, l - 2, mi, ni) - xt_at(X, blocks, pl, a - 2, l, mi, ni) -
                  xt_at(X, blocks, pl, a, l - 2, mi, ni) + xt_at(X, blocks, pl, a, l, mi, ni);
    }
    const int64_t off = (static_cast<int64_t>(w) * n + l) * m + a;
    double2 out = make_double2(v[0], v[1]);
    if (L != nullptr) {
        const double2 lv = L[off];
        out.x += lv.x;
        if (plane_of[2 * w + 1] >= 0) out.y += lv.y;
    }
    planes[off] = out;
}

// ---------------------------------------------------------------------------
// out = sE E - sAB (A X B) - sCD (C X D), blockwise.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_apply(const BlockDesc* __restrict__ blocks,
                                               const double* __restrict__ E, double sE,
                                               const double* __restrict__ X, double sAB,
                                               double sCD, double* __restrict__ out,
                                               const double* __restrict__ atab, int64_t a_wstride,
                                               int me0, const double* __restrict__ ztabA, int ne0) {
    const BlockDesc bd = blocks[blockIdx.y];
    const int me = bd.me, ne = bd.ne;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= me * ne) return;
    const int i = e / ne, k = e - i * ne;
    const double* Xb = X + bd.eoff;
    const double* ar = atab + bd.w * a_wstride + (bd.pr ? me0 * 12 : 0) + i * 12;
    const double* zc = ztabA + (bd.pz ? ne0 * 8 : 0) + k * 8;
    double sab = 0.0, scd = 0.0;
#pragma unroll
    for (int da = -2; da <= 3; ++da) {
        const int a = i + da;
        if (a < 0 || a >= me) continue;
        double xb = 0.0, xd = 0.0;
#pragma unroll
        for (int dl = -1; dl <= 2; ++dl) {
            const int l = k + dl;
            if (l < 0 || l >= ne) continue;
            const double x = Xb[a * ne + l];
            xb += x * zc[dl + 1];
            xd += x * zc[4 + dl + 1];
        }
        sab += ar[da + 2] * xb;
        scd += ar[6 + da + 2] * xd;
    }
    const double ev = (sE != 0.0) ? sE * E[bd.eoff + e] : 0.0;
    out[bd.eoff + e] = ev - sAB * sab - sCD * scd;
}

struct PList { const double* p[4]; double beta[4]; };

__global__ __launch_bounds__(256) void k_heat_rhs(double* __restrict__ E, PList P, int nb,
                                                  const double* __restrict__ Ec, int64_t total) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    double acc = Ec[e];
    for (int b = 0; b < nb; ++b) acc += P.beta[b] * P.p[b][e];
    E[e] = acc;
}

__global__ __launch_bounds__(256) void k_norms(const double* __restrict__ R,
                                               const double* __restrict__ E,
                                               const double* __restrict__ X, int64_t total,
                                               double* acc) {
    __shared__ double red[3][256];
    double r2 = 0.0, e2 = 0.0, bad = 0.0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double r = R[e], ev = E[e], x = X[e];
        r2 += r * r;
        e2 += ev * ev;
        if (!isfinite(x)) bad += 1.0;
    }
    red[0][threadIdx.x] = r2; red[1][threadIdx.x] = e2; red[2][threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) atomicAdd(&acc[threadIdx.x], red[threadIdx.x][0]);
}

}  // namespace

hipError_t launch_adi(const BlockDesc* blocks, int nblocks, int threads, const double* E,
                      double* X, double* state, const double* rtab, const double* ztab,
                      const double* vmu, bool accumulate, bool use_lds, size_t lds_bytes,
                      hipStream_t s) {
    if (use_lds)
        hipLaunchKernelGGL(k_adi_lds, dim3(nblocks), dim3(threads), lds_bytes, s, blocks, E, X,
                           state, rtab, ztab, vmu, accumulate ? 1 : 0);
    else
        hipLaunchKernelGGL(k_adi_global, dim3(nblocks), dim3(threads), 0, s, blocks, E, X, state,
                           rtab, ztab, vmu, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t adi_set_lds_limit(size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adi_lds),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

hipError_t launch_rhs3(const double2* F, const double2* L, double sF, double cL, double sL,
                       double* E, const BlockDesc* blocks, int nplanes, int m, int n,
                       const RhsTables& t, hipStream_t s) {
    const int64_t cnt = static_cast<int64_t>(m - 2) * (n - 2);
    const dim3 grid(static_cast<unsigned>((cnt + 255) / 256), nplanes);
    hipLaunchKernelGGL(k_rhs, grid, dim3(256), 0, s, F, L, sF, cL, sL, E, blocks, m, n, t);
    return hipGetLastError();
}

hipError_t launch_recombine(const double* X, const double2* L, double2* planes,
                            const int* plane_of, const BlockDesc* blocks, int nw, int m, int n,
                            int p, hipStream_t s) {
    (void)p;
    const int64_t cnt = static_cast<int64_t>(m) * n;
    const dim3 grid(static_cast<unsigned>((cnt + 255) / 256), nw);
    hipLaunchKernelGGL(k_recombine, grid, dim3(256), 0, s, X, L, planes, plane_of, blocks, m, n);
    return hipGetLastError();
}

hipError_t launch_apply2(const BlockDesc* blocks, int nblocks, int max_elems, const double* E,
                         double sE, const double* X, double sAB, double sCD, double* out,
                         const double* atab, int64_t a_wstride, int me0, const double* ztabA,
                         int ne0, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((max_elems + 255) / 256), nblocks);
    hipLaunchKernelGGL(k_apply, grid, dim3(256), 0, s, blocks, E, sE, X, sAB, sCD, out, atab,
                       a_wstride, me0, ztabA, ne0);
    return hipGetLastError();
}

hipError_t launch_heat_rhs(double* E, const double* const* P, const double* beta, int nb,
                           const double* Econst, int64_t total, hipStream_t s) {
    PList pl{};
    for (int b = 0; b < nb && b < 4; ++b) { pl.p[b] = P[b]; pl.beta[b] = beta[b]; }
    const unsigned grid = static_cast<unsigned>((total + 255) / 256);
    hipLaunchKernelGGL(k_heat_rhs, dim3(grid), dim3(256), 0, s, E, pl, nb, Econst, total);
    return hipGetLastError();
}

hipError_t launch_norms(const double* R, const double* E, const double* X, int64_t total,
                        double* acc, hipStream_t s) {
    int64_t blocks = (total + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_norms, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, R, E, X,
                       total, acc);
    return hipGetLastError();
}

}  // namespace cyl
