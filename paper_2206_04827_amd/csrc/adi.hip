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
// its intermediate, the back substitution with the result, and short register
// windows hold the few neighbours still needed.
//
// Layouts of a parity block (me x ne, rows padded to mp, columns to np, both
// multiples of G):
//   E-layout  (E, residuals, heat history): column-major, element (i, k) at
//             eoff + k * mp + i; rows me..mp-1 are zero.
//   X-layout  (solutions):                  row-major, element (i, k) at
//             xoff + i * ne + k.
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

#include "kernels.hpp"

namespace cyl {
namespace {

constexpr int G = 8;          // rows per software-pipelined group
constexpr int kRRec = 12;
constexpr int kZRec = 8;
constexpr int kRCouple = 3;   // record rows after a block's r records (5 x 5 coupling)
constexpr int kZCouple = 2;   // record rows after a block's z records (3 x 3 coupling)
constexpr int kResTileK = 128; // columns per LDS-staged residual tile (state in global memory)

// Pointers that may come from memory (the per-problem tables of a batch) are
// generic, and generic pointers compile to flat accesses, which also count
// against the LDS wait counter: every LDS wait then drains the outstanding
// global loads as well.  Rebuilt from their integer values as global-space
// pointers they compile to global accesses.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
    using G = __attribute__((address_space(1))) T*;
    return (T*)(G)(reinterpret_cast<uintptr_t>(p));
}

// ---------------------------------------------------------------------------
// LDS-resident sweeps with a compile-time row stride LD (so every row offset
// within a group is an instruction immediate).
// ---------------------------------------------------------------------------

// r-pass on column k.  S: state (rows padded to mp, followed by 4 zero guard
// rows); RC: kRRec records per row; Ecol: this column of E (contiguous rows).
// Each group of G rows first issues its record, window and E loads, then
// evaluates the banded products (independent of the recurrence) for all rows,
// then runs the dependent chain, one FMA deep per row.
template <int LD>
__device__ __forceinline__ void rpass_lds(double* __restrict__ S, int mp, int k,
                                          const double* __restrict__ RC,
                                          const double* __restrict__ Ecol, double vmu) {
    const double2* E2 = reinterpret_cast<const double2*>(Ecol);
    double* Sk = S + k;
    double wv[14];                 // rows i0-2 .. i0+11 of W
    wv[0] = 0.0; wv[1] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[2 + q] = Sk[q * LD];
    double2 eb[G / 2], en[G / 2];
#pragma unroll
    for (int q = 0; q < G / 2; ++q) { eb[q] = E2[q]; en[q] = E2[G / 2 + q]; }
    double g1 = 0.0, g2 = 0.0;
    for (int i0 = 0; i0 < mp; i0 += G) {
        double* Sg = Sk + i0 * LD;
        const double2* Rg = reinterpret_cast<const double2*>(RC + i0 * kRRec);
        double c[G][8];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double2 v = Rg[q * (kRRec / 2) + t];
                c[q][2 * t] = v.x;
                c[q][2 * t + 1] = v.y;
            }
#pragma unroll
        for (int q = 0; q < 8; ++q) wv[6 + q] = Sg[(4 + q) * LD];
        double2 enn[G / 2];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) enn[q] = E2[(i0 + 2 * G) / 2 + q];
        double e[G];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) { e[2 * q] = eb[q].x; e[2 * q + 1] = eb[q].y; }
        double h[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            h[q] = c[q][0] * wv[q] + c[q][1] * wv[q + 1] + c[q][2] * wv[q + 2] +
                   c[q][3] * wv[q + 3] + c[q][4] * wv[q + 4] + c[q][5] * wv[q + 5] - vmu * e[q];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double t = h[q] - c[q][6] * g2;
            const double g = t - c[q][7] * g1;
            Sg[q * LD] = g;
            g2 = g1;
            g1 = g;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) wv[q] = wv[8 + q];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) { eb[q] = en[q]; en[q] = enn[q]; }
    }
    // back substitution: z_i = dinv_i g_i - sum_t (dinv_i U_{i,i+t}) z_{i+t}
    double gb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = Sk[(mp - G + q) * LD];
    double z1 = 0.0, z2 = 0.0, z3 = 0.0;
    for (int i0 = mp - G; i0 >= 0; i0 -= G) {
        double* Sg = Sk + i0 * LD;
        const double2* Rg = reinterpret_cast<const double2*>(RC + i0 * kRRec + 8);
        double c[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const double2 v = Rg[q * (kRRec / 2) + t];
                c[q][2 * t] = v.x;
                c[q][2 * t + 1] = v.y;
            }
        double gn[G];
        if (i0 > 0) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = Sg[(q - G) * LD];
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double t = c[q][0] * gb[q] - c[q][3] * z3 - c[q][2] * z2;
            const double z = t - c[q][1] * z1;
            Sg[q * LD] = z;
            z3 = z2; z2 = z1; z1 = z;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
}

// z-pass on one row (np columns, a multiple of G; columns beyond the block's
// ne have zero records).  ZC: kZRec records per column.  The forward
// prefetch may read past the row end (into the next row or the guard rows);
// those values are never used.
template <bool kLast>
__device__ __forceinline__ void zpass_row(double* __restrict__ row, int np,
                                          const double* __restrict__ ZC) {
    double zb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) zb[q] = row[q];
    double gp = 0.0;
    for (int k0 = 0; k0 < np; k0 += G) {
        double* rg = row + k0;
        double l[G], zn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) l[q] = ZC[(k0 + q) * kZRec];
#pragma unroll
        for (int q = 0; q < G; ++q) zn[q] = rg[G + q];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double g = zb[q] - l[q] * gp;
            rg[q] = g;
            gp = g;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) zb[q] = zn[q];
    }
    // back substitution x_k = dinv_k g_k - U1 x_{k+1} - U2 x_{k+2}, and unless
    // this is the last iteration, w_{k+1} = sum_t P_{k+1,t} x_{k+t}.
    double gb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = row[np - G + q];
    double x1 = 0.0, x2 = 0.0, x3 = 0.0;
    double pn[4] = {0.0, 0.0, 0.0, 0.0};     // product record of column k0 + G
    for (int k0 = np - G; k0 >= 0; k0 -= G) {
        double* rg = row + k0;
        const double2* zg = reinterpret_cast<const double2*>(ZC + k0 * kZRec);
        double c[G][3], pr[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double2 a = zg[q * (kZRec / 2) + 0], b = zg[q * (kZRec / 2) + 1];
            const double2 d = zg[q * (kZRec / 2) + 2], e = zg[q * (kZRec / 2) + 3];
            c[q][0] = a.y; c[q][1] = b.x; c[q][2] = b.y;
            pr[q][0] = d.x; pr[q][1] = d.y; pr[q][2] = e.x; pr[q][3] = e.y;
        }
        double gn[G];
        if (k0 > 0) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = rg[q - G];
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double x = c[q][0] * gb[q] - c[q][2] * x2 - c[q][1] * x1;
            if (kLast) {
                rg[q] = x;
            } else {
                const double* p = (q == G - 1) ? pn : pr[q + 1];
                if (q < G - 1 || k0 + G < np)
                    rg[q + 1] = p[0] * x + p[1] * x1 + p[2] * x2 + p[3] * x3;
            }
            x3 = x2; x2 = x1; x1 = x;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) pn[t] = pr[0][t];
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
    if (!kLast) row[0] = pn[1] * x1 + pn[2] * x2 + pn[3] * x3;
}

__device__ __forceinline__ void zpass(double* row, int np, const double* ZC, bool last) {
    if (last) zpass_row<true>(row, np, ZC);
    else zpass_row<false>(row, np, ZC);
}

// Copy n doubles (rounded up to whole 128-double chunks) from global memory
// straight into LDS, one 16-byte piece per lane (no registers involved).  The
// source tables carry read slack after their end, the LDS regions are sized in
// whole chunks.  Completion is awaited with s_waitcnt before the next barrier.
__device__ __forceinline__ void copy_to_lds(double* dst, const double* __restrict__ src, int n) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int chunks = (n + 127) >> 7;
    for (int c = wave; c < chunks; c += nwaves)
        __builtin_amdgcn_global_load_lds(src + (c << 7) + 2 * lane, dst + (c << 7), 16, 0, 0);
}

__device__ __forceinline__ int lds_chunks(int n) { return (n + 127) / 128 * 128; }

// One workgroup per parity block, all J iterations, block state in LDS.
// While the z-pass of shift j runs, the r-records of shift j+1 stream into
// LDS; while the r-pass of shift j+1 runs, its z-records follow.
template <int LD>
__device__ __forceinline__ void adi_block_lds(double* sm, const BlockDesc& bd,
                                              const double* __restrict__ E, double* X,
                                              const double* __restrict__ rtab,
                                              const double* __restrict__ ztab,
                                              const double* __restrict__ vmu, int accumulate) {
    const int me = bd.me, ne = bd.ne, mp = bd.mp, np = bd.np;
    const int tid = threadIdx.x, nt = blockDim.x;
    double* S = sm;
    double* RCs = sm + (mp + 4) * LD;
    double* ZCs = RCs + lds_chunks(mp * kRRec);
    const int nr = mp * kRRec, nz = np * kZRec;
    for (int idx = tid; idx < (mp + 4) * LD; idx += nt) S[idx] = 0.0;
    copy_to_lds(RCs, rtab + bd.rbase, nr);
    copy_to_lds(ZCs, ztab + bd.zbase, nz);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const double* Ecol = E + bd.eoff + static_cast<int64_t>(tid) * mp;
    for (int j = 0; j < bd.J; ++j) {
        const double vm = vmu[bd.soff + j];
        if (tid < ne) rpass_lds<LD>(S, mp, tid, RCs, Ecol, vm);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const bool more = j + 1 < bd.J;
        if (more) copy_to_lds(RCs, rtab + bd.rbase + (j + 1) * bd.rstride, nr);
        if (tid < me) zpass(S + tid * LD, np, ZCs, j == bd.J - 1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (more) copy_to_lds(ZCs, ztab + bd.zbase + (j + 1) * bd.zstride, nz);
    }
    double* Xb = X + bd.xoff;
    for (int idx = tid; idx < me * ne; idx += nt) {
        const int i = idx / ne, k = idx - i * ne;
        const double v = S[i * LD + k];
        Xb[idx] = accumulate ? Xb[idx] + v : v;
    }
}

template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_adi_lds(const BlockDesc* __restrict__ blocks, const double* __restrict__ E, double* X,
               const double* __restrict__ rtab, const double* __restrict__ ztab,
               const double* __restrict__ vmu, int accumulate, const AdiPtrs* __restrict__ pp) {
    extern __shared__ double sm[];
    const BlockDesc bd = blocks[blockIdx.x];
    if (pp != nullptr) {
        const AdiPtrs q = pp[bd.prob];
        E = q.E; X = q.X; rtab = q.rtab; ztab = q.ztab; vmu = q.vmu;
    }
    adi_block_lds<NP + 1>(sm, bd, E, X, rtab, ztab, vmu, accumulate);
}

// ---------------------------------------------------------------------------
// Split sweeps: two threads per line, so that a block whose state fills the
// LDS of a CU still keeps all four SIMDs busy.  A line of n unknowns is cut
// at the split row t (a multiple of G): threads [0, L) eliminate [0, t)
// downwards with the LU records, threads [L, 2L) eliminate [t, n) upwards
// with the UL records; both exchange their last values through the LDS
// exchange area, solve the small coupling system for the unknowns around t,
// and substitute outwards from t.  Bands: r-pass (lo, hi) = (2, 3), coupling
// x_{t-2} .. x_{t+2}; z-pass (1, 2), coupling x_{t-1} .. x_{t+1}.
// ---------------------------------------------------------------------------

// Barrier for LDS traffic only: records streamed into LDS by the other half of
// the iteration and right-hand-side prefetches may stay in flight.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Rows of a split kernel's block state, stride LD.  kBand (state in global
// memory): rows [b0, b0 + nb) are kept in LDS at l instead, so their reads
// and writes in every sweep stay on the chip.
template <int LD, bool kBand>
struct StateRows {
    double* g;
    double* l;
    int b0, nb;
    __device__ __forceinline__ double* row(int i) const {
        if constexpr (kBand) {
            if (static_cast<unsigned>(i - b0) < static_cast<unsigned>(nb)) return l + (i - b0) * LD;
        }
        return g + i * LD;
    }
    // Element (i0 + q, k) from the group base at(i0, k): plain pointer steps
    // without a band (the code the sweeps were tuned with), the row lookup
    // with one.
    __device__ __forceinline__ double* at(int i0, int k) const { return g + i0 * LD + k; }
    __device__ __forceinline__ double& el(double* base, int i0, int q, int k) const {
        if constexpr (kBand) return row(i0 + q)[k];
        else return base[q * LD];
    }
};

// r-pass, rows [0, t) of column k (LU records).  pre: W rows t, t+1, t+2 of
// this column, read before any thread overwrote them.  Returns g_{t-2}, g_{t-1}.
template <int LD, int G, class ST>
__device__ __forceinline__ void rs_top_fwd(const ST& S, int t, int k,
                                           const double* __restrict__ RC,
                                           const double* __restrict__ Ecol, double vmu,
                                           const double pre[3], double* gt2, double* gt1) {
    const double2* E2 = reinterpret_cast<const double2*>(Ecol);
    static_assert(G >= 4 && G % 2 == 0, "row group");
    double wv[G + 6];              // rows i0-2 .. i0+G+3 of W
    wv[0] = 0.0; wv[1] = 0.0;
    double* Sk = S.at(0, k);
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[2 + q] = S.el(Sk, 0, q, k);
    double2 eb[G / 2], en[G / 2];
#pragma unroll
    for (int q = 0; q < G / 2; ++q) { eb[q] = E2[q]; en[q] = E2[G / 2 + q]; }
    double g1 = 0.0, g2 = 0.0;
    for (int i0 = 0; i0 < t; i0 += G) {
        double* Sg = S.at(i0, k);
        const double2* Rg = reinterpret_cast<const double2*>(RC + i0 * kRRec);
        double c[G][8];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double2 v = Rg[q * (kRRec / 2) + s];
                c[q][2 * s] = v.x;
                c[q][2 * s + 1] = v.y;
            }
        if (i0 + G < t) {
#pragma unroll
            for (int q = 0; q < G; ++q) wv[6 + q] = S.el(Sg, i0, 4 + q, k);
        } else {
#pragma unroll
            for (int q = 0; q < G - 4; ++q) wv[6 + q] = S.el(Sg, i0, 4 + q, k);
            wv[G + 2] = pre[0]; wv[G + 3] = pre[1]; wv[G + 4] = pre[2]; wv[G + 5] = 0.0;
        }
        double2 enn[G / 2];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) enn[q] = E2[(i0 + 2 * G) / 2 + q];
        double e[G];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) { e[2 * q] = eb[q].x; e[2 * q + 1] = eb[q].y; }
        double h[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            h[q] = c[q][0] * wv[q] + c[q][1] * wv[q + 1] + c[q][2] * wv[q + 2] +
                   c[q][3] * wv[q + 3] + c[q][4] * wv[q + 4] + c[q][5] * wv[q + 5] - vmu * e[q];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double tq = h[q] - c[q][6] * g2;
            const double g = tq - c[q][7] * g1;
            S.el(Sg, i0, q, k) = g;
            g2 = g1;
            g1 = g;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) wv[q] = wv[G + q];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) { eb[q] = en[q]; en[q] = enn[q]; }
    }
    *gt2 = g2;
    *gt1 = g1;
}

// r-pass back substitution on rows t-1 .. 0, starting from x_t, x_{t+1}, x_{t+2}.
template <int LD, int G, class ST>
__device__ __forceinline__ void rs_top_bwd(const ST& S, int t, int k,
                                           const double* __restrict__ RC, double z1, double z2,
                                           double z3) {
    double gb[G];
    double* St0 = S.at(t - G, k);
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = S.el(St0, t - G, q, k);
    for (int i0 = t - G; i0 >= 0; i0 -= G) {
        double* Sg = S.at(i0, k);
        const double2* Rg = reinterpret_cast<const double2*>(RC + i0 * kRRec + 8);
        double c[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double2 v = Rg[q * (kRRec / 2) + s];
                c[q][2 * s] = v.x;
                c[q][2 * s + 1] = v.y;
            }
        double gn[G];
        if (i0 > 0) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = S.el(Sg, i0, q - G, k);
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double tq = c[q][0] * gb[q] - c[q][3] * z3 - c[q][2] * z2;
            const double z = tq - c[q][1] * z1;
            S.el(Sg, i0, q, k) = z;
            z3 = z2; z2 = z1; z1 = z;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
}

// r-pass, rows mp-1 .. t of column k (UL records, upwards).  preb: W rows
// t-2, t-1 of this column.  Returns g'_t, g'_{t+1}, g'_{t+2}.
template <int LD, int G, class ST>
__device__ __forceinline__ void rs_bot_fwd(const ST& S, int mp, int t, int k,
                                           const double* __restrict__ RC,
                                           const double* __restrict__ Ecol, double vmu,
                                           const double preb[2], double* g0, double* g1,
                                           double* g2) {
    const double2* E2 = reinterpret_cast<const double2*>(Ecol);
    static_assert(G >= 4 && G % 2 == 0, "row group");
    double up[3] = {0.0, 0.0, 0.0};        // old W rows i0+G .. i0+G+2
    double gp1 = 0.0, gp2 = 0.0, gp3 = 0.0;  // g'_{i+1}, g'_{i+2}, g'_{i+3}
    double2 eb[G / 2], en[G / 2];
#pragma unroll
    for (int q = 0; q < G / 2; ++q) { eb[q] = E2[(mp - G) / 2 + q]; en[q] = E2[(mp - 2 * G) / 2 + q]; }
    for (int i0 = mp - G; i0 >= t; i0 -= G) {
        double* Sg = S.at(i0, k);
        const double2* Rg = reinterpret_cast<const double2*>(RC + i0 * kRRec);
        double c[G][10];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const double2 v = Rg[q * (kRRec / 2) + s];
                c[q][2 * s] = v.x;
                c[q][2 * s + 1] = v.y;
            }
        double w[G + 5];                   // rows i0-2 .. i0+G+2 of W
        if (i0 > t) {
            w[0] = S.el(Sg, i0, -2, k);
            w[1] = S.el(Sg, i0, -1, k);
        } else {
            w[0] = preb[0];
            w[1] = preb[1];
        }
#pragma unroll
        for (int q = 0; q < G; ++q) w[2 + q] = S.el(Sg, i0, q, k);
        w[G + 2] = up[0]; w[G + 3] = up[1]; w[G + 4] = up[2];
        double2 enn[G / 2];
        if (i0 >= 2 * G) {
#pragma unroll
            for (int q = 0; q < G / 2; ++q) enn[q] = E2[(i0 - 2 * G) / 2 + q];
        } else {
#pragma unroll
            for (int q = 0; q < G / 2; ++q) enn[q] = make_double2(0.0, 0.0);
        }
        double e[G];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) { e[2 * q] = eb[q].x; e[2 * q + 1] = eb[q].y; }
        double h[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            h[q] = c[q][0] * w[q] + c[q][1] * w[q + 1] + c[q][2] * w[q + 2] +
                   c[q][3] * w[q + 3] + c[q][4] * w[q + 4] + c[q][5] * w[q + 5] - vmu * e[q];
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double tq = h[q] - c[q][8] * gp3 - c[q][7] * gp2;
            const double g = tq - c[q][6] * gp1;
            S.el(Sg, i0, q, k) = g;
            gp3 = gp2; gp2 = gp1; gp1 = g;
        }
        up[0] = w[2]; up[1] = w[3]; up[2] = w[4];
#pragma unroll
        for (int q = 0; q < G / 2; ++q) { eb[q] = en[q]; en[q] = enn[q]; }
    }
    *g0 = gp1;
    *g1 = gp2;
    *g2 = gp3;
}

// r-pass forward substitution on rows t .. mp-1, starting from x_{t-1}, x_{t-2}.
template <int LD, int G, class ST>
__device__ __forceinline__ void rs_bot_bwd(const ST& S, int mp, int t, int k,
                                           const double* __restrict__ RC, double xm1, double xm2) {
    double gb[G];
    double* St0 = S.at(t, k);
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = S.el(St0, t, q, k);
    for (int i0 = t; i0 < mp; i0 += G) {
        double* Sg = S.at(i0, k);
        const double2* Rg = reinterpret_cast<const double2*>(RC + i0 * kRRec + 8);
        double c[G][3];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double2 a = Rg[q * (kRRec / 2)], b = Rg[q * (kRRec / 2) + 1];
            c[q][0] = a.y; c[q][1] = b.x; c[q][2] = b.y;     // dinv', L^(i,i-1), L^(i,i-2)
        }
        double gn[G];
        if (i0 + G < mp) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = S.el(Sg, i0, G + q, k);
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double tq = c[q][0] * gb[q] - c[q][2] * xm2;
            const double x = tq - c[q][1] * xm1;
            S.el(Sg, i0, q, k) = x;
            xm2 = xm1; xm1 = x;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
}

// z-pass, columns [0, t) of one row (LU records).  Returns g_{t-1}.
template <int G>
__device__ __forceinline__ double zs_top_fwd(double* __restrict__ row, int t,
                                             const double* __restrict__ ZC) {
    double zb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) zb[q] = row[q];
    double gp = 0.0;
    for (int k0 = 0; k0 < t; k0 += G) {
        double* rg = row + k0;
        double l[G], zn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) l[q] = ZC[(k0 + q) * kZRec];
#pragma unroll
        for (int q = 0; q < G; ++q) zn[q] = rg[G + q];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double g = zb[q] - l[q] * gp;
            rg[q] = g;
            gp = g;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) zb[q] = zn[q];
    }
    return gp;
}

// z-pass back substitution on columns t-1 .. 0 from x_t, x_{t+1}; unless this
// is the last iteration, each x is replaced by w = x (u' B + D) on the fly
// (columns < t only).
template <bool kLast, int G>
__device__ __forceinline__ void zs_top_bwd(double* __restrict__ row, int t,
                                           const double* __restrict__ ZC, double x1, double x2) {
    double gb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = row[t - G + q];
    double x3 = 0.0;
    double pn[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = t - G; k0 >= 0; k0 -= G) {
        double* rg = row + k0;
        const double2* zg = reinterpret_cast<const double2*>(ZC + k0 * kZRec);
        double c[G][3], pr[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double2 a = zg[q * (kZRec / 2) + 0], b = zg[q * (kZRec / 2) + 1];
            const double2 d = zg[q * (kZRec / 2) + 2], e = zg[q * (kZRec / 2) + 3];
            c[q][0] = a.y; c[q][1] = b.x; c[q][2] = b.y;
            pr[q][0] = d.x; pr[q][1] = d.y; pr[q][2] = e.x; pr[q][3] = e.y;
        }
        double gn[G];
        if (k0 > 0) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = rg[q - G];
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double x = c[q][0] * gb[q] - c[q][2] * x2 - c[q][1] * x1;
            if (kLast) {
                rg[q] = x;
            } else {
                const double* p = (q == G - 1) ? pn : pr[q + 1];
                if (q < G - 1 || k0 + G < t)
                    rg[q + 1] = p[0] * x + p[1] * x1 + p[2] * x2 + p[3] * x3;
            }
            x3 = x2; x2 = x1; x1 = x;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) pn[s] = pr[0][s];
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
    if (!kLast) row[0] = pn[1] * x1 + pn[2] * x2 + pn[3] * x3;
}

// z-pass, columns np-1 .. t of one row (UL records, leftwards).  Returns
// g'_t, g'_{t+1}.
template <int G>
__device__ __forceinline__ void zs_bot_fwd(double* __restrict__ row, int np, int t,
                                           const double* __restrict__ ZC, double* g0,
                                           double* g1) {
    double zb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) zb[q] = row[np - G + q];
    double gp1 = 0.0, gp2 = 0.0;
    for (int k0 = np - G; k0 >= t; k0 -= G) {
        double* rg = row + k0;
        double u1[G], u2[G], zn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double2 u = *reinterpret_cast<const double2*>(ZC + (k0 + q) * kZRec);
            u1[q] = u.x; u2[q] = u.y;
        }
        if (k0 - G >= t) {
#pragma unroll
            for (int q = 0; q < G; ++q) zn[q] = rg[q - G];
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double g = zb[q] - u2[q] * gp2 - u1[q] * gp1;
            rg[q] = g;
            gp2 = gp1; gp1 = g;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) zb[q] = zn[q];
    }
    *g0 = gp1;
    *g1 = gp2;
}

// z-pass forward substitution on columns t .. np-1 from x_{t-1}; unless this
// is the last iteration, w_{k-2} = x (u' B + D) at column k-2 >= t is written
// as soon as x_k is known, and the last two columns after the loop.
template <bool kLast, int G>
__device__ __forceinline__ void zs_bot_bwd(double* __restrict__ row, int np, int t,
                                           const double* __restrict__ ZC, double xm1) {
    double gb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = row[t + q];
    double xm2 = 0.0, xm3 = 0.0;
    for (int k0 = t; k0 < np; k0 += G) {
        double* rg = row + k0;
        double c[G][2], pr[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double2 a = *reinterpret_cast<const double2*>(ZC + (k0 + q) * kZRec + 2);
            c[q][0] = a.x; c[q][1] = a.y;                      // dinv', L^(k, k-1)
            if (!kLast) {
                const double2* p = reinterpret_cast<const double2*>(ZC + (k0 + q - 2) * kZRec + 4);
                const double2 d = p[0], e = p[1];
                pr[q][0] = d.x; pr[q][1] = d.y; pr[q][2] = e.x; pr[q][3] = e.y;
            }
        }
        double gn[G];
        if (k0 + G < np) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = rg[G + q];
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double x = c[q][0] * gb[q] - c[q][1] * xm1;
            if (kLast) {
                rg[q] = x;
            } else if (k0 + q - 2 >= t) {
                rg[q - 2] = pr[q][0] * xm3 + pr[q][1] * xm2 + pr[q][2] * xm1 + pr[q][3] * x;
            }
            xm3 = xm2; xm2 = xm1; xm1 = x;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
    if (!kLast) {
        const double2* pa = reinterpret_cast<const double2*>(ZC + (np - 2) * kZRec + 4);
        const double2* pb = reinterpret_cast<const double2*>(ZC + (np - 1) * kZRec + 4);
        const double2 a0 = pa[0], a1 = pa[1], b0 = pb[0];
        row[np - 2] = a0.x * xm3 + a0.y * xm2 + a1.x * xm1;
        row[np - 1] = b0.x * xm2 + b0.y * xm1;
    }
}

// One workgroup (2 L threads) per parity block, all J iterations in LDS.
// LDS: state (mp rows of LD), r records (+ coupling), z records (+ coupling),
// exchange area (5 x L).
// kGS: the block state lives in global memory (gS, mp rows of LD; blocks too
// large for LDS), records and the exchange area stay in LDS, and the barriers
// between the halves also wait for the state's vector-memory traffic.
template <bool kGS>
__device__ __forceinline__ void half_barrier() {
    if (kGS) __syncthreads();
    else lds_barrier();
}

template <int LD, bool kGS, int GB, int GZF = GB>
__device__ __forceinline__ void adi_block_split(double* sm, double* gS, const BlockDesc& bd,
                                                const double* __restrict__ E, double* X,
                                                const double* __restrict__ rtab,
                                                const double* __restrict__ ztab,
                                                const double* __restrict__ vmu, int accumulate,
                                                const ResArgs& res, int lds_doubles = 0) {
    const int me = bd.me, ne = bd.ne, mp = bd.mp, np = bd.np, tr = bd.tr, tz = bd.tz;
    const int tid = threadIdx.x, nt = blockDim.x, L = nt >> 1;
    const int line = tid % L;
    const bool top = tid < L;
    // rows per software-pipelined group of the forward r sweeps: 4 when the
    // state is in global memory (512-thread workgroups leave 256 registers
    // per thread)
    constexpr int GG = kGS ? 4 : G;
    // GB: rows/columns per group of the backward r sweeps and of the z
    // sweeps, whose rows carry fewer records: 8 with the state in global
    // memory; 16 in LDS when every half of every block is a multiple of 16.
    // More loads in flight per wait.  GZF: columns per group of the forward
    // z sweeps (three values per column): 16 with the state in global memory
    // when every z half is a multiple of 16.
    static_assert(GB % GG == 0 && GZF % GB == 0, "groups of the backward and z sweeps");
    // accumulate bit 1 (a test switch): fill the LDS this block uses with NaN
    // first, so that any read of LDS the block has not written shows up as a
    // non-finite solution
    if (accumulate & 2) {
        const int used = kGS ? lds_doubles
                             : mp * LD + lds_chunks((mp + kRCouple) * kRRec) + lds_chunks((np + kZCouple) * kZRec) + 5 * L;
        for (int idx = tid; idx < used; idx += nt) sm[idx] = __builtin_nan("");
        __syncthreads();
    }
    double* S = kGS ? gS : sm;
    const int nr = (mp + kRCouple) * kRRec, nz = (np + kZCouple) * kZRec;
    double* RCs = kGS ? sm : S + mp * LD;
    double* ZCs = RCs + lds_chunks(nr);
    double* XC = ZCs + lds_chunks(nz);
    // kGS: the rows around the r split (read and written in every sweep like
    // all others) that fit in the LDS left after the records and the exchange
    // area stay in LDS (lds_doubles: the launch's LDS, in doubles)
    StateRows<LD, kGS> St{S, nullptr, 0, 0};
    if constexpr (kGS) {
        double* band = XC + (5 * L + 15) / 16 * 16;
        const int room = (lds_doubles - static_cast<int>(band - sm)) / LD;
        St.nb = room < 0 ? 0 : (room < mp ? room : mp);
        const int b0 = tr - St.nb / 2;
        St.b0 = b0 < 0 ? 0 : (b0 > mp - St.nb ? mp - St.nb : b0);
        St.l = band;
        for (int idx = tid; idx < mp * LD; idx += nt) St.row(idx / LD)[idx % LD] = 0.0;
    } else {
        for (int idx = tid; idx < mp * LD; idx += nt) S[idx] = 0.0;
    }
    copy_to_lds(RCs, rtab + bd.rbase, nr);
    copy_to_lds(ZCs, ztab + bd.zbase, nz);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const double* Ecol = E + bd.eoff + static_cast<int64_t>(line) * mp;
    for (int j = 0; j < bd.J; ++j) {
        const double vm = vmu[bd.soff + j];
        // ---- r-pass: lines are columns
        double pre[3] = {0.0, 0.0, 0.0};
        if (line < ne) {
            if (top) {
#pragma unroll
                for (int s = 0; s < 3; ++s) pre[s] = St.row(tr + s)[line];
            } else {
#pragma unroll
                for (int s = 0; s < 2; ++s) pre[s] = St.row(tr - 2 + s)[line];
            }
        }
        half_barrier<kGS>();
        if (line < ne) {
            if (top) {
                double a, b;
                rs_top_fwd<LD, GG>(St, tr, line, RCs, Ecol, vm, pre, &a, &b);
                XC[line] = a;
                XC[L + line] = b;
            } else {
                double a, b, c;
                rs_bot_fwd<LD, GG>(St, mp, tr, line, RCs, Ecol, vm, pre, &a, &b, &c);
                XC[2 * L + line] = a;
                XC[3 * L + line] = b;
                XC[4 * L + line] = c;
            }
        }
        half_barrier<kGS>();
        if (line < ne) {
            double v[5], y[5];
#pragma unroll
            for (int s = 0; s < 5; ++s) v[s] = XC[s * L + line];
            const double* K5 = RCs + mp * kRRec;
#pragma unroll
            for (int r = 0; r < 5; ++r)
                y[r] = K5[5 * r] * v[0] + K5[5 * r + 1] * v[1] + K5[5 * r + 2] * v[2] +
                       K5[5 * r + 3] * v[3] + K5[5 * r + 4] * v[4];
            if (top) rs_top_bwd<LD, GB>(St, tr, line, RCs, y[2], y[3], y[4]);
            else rs_bot_bwd<LD, GB>(St, mp, tr, line, RCs, y[1], y[0]);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const bool more = j + 1 < bd.J;
        if (more) copy_to_lds(RCs, rtab + bd.rbase + (j + 1) * bd.rstride, nr);
        // ---- z-pass: lines are rows
        double* row = St.row(line);
        if (line < me) {
            if (top) {
                XC[line] = zs_top_fwd<GZF>(row, tz, ZCs);
            } else {
                double a, b;
                zs_bot_fwd<GZF>(row, np, tz, ZCs, &a, &b);
                XC[L + line] = a;
                XC[2 * L + line] = b;
            }
        }
        half_barrier<kGS>();
        if (line < me) {
            const double v0 = XC[line], v1 = XC[L + line], v2 = XC[2 * L + line];
            const double* K3 = ZCs + np * kZRec;
            const double y0 = K3[0] * v0 + K3[1] * v1 + K3[2] * v2;
            const double y1 = K3[3] * v0 + K3[4] * v1 + K3[5] * v2;
            const double y2 = K3[6] * v0 + K3[7] * v1 + K3[8] * v2;
            if (top) {
                if (more) zs_top_bwd<false, GB>(row, tz, ZCs, y1, y2);
                else zs_top_bwd<true, GB>(row, tz, ZCs, y1, y2);
            } else {
                if (more) zs_bot_bwd<false, GB>(row, np, tz, ZCs, y0);
                else zs_bot_bwd<true, GB>(row, np, tz, ZCs, y0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (more) copy_to_lds(ZCs, ztab + bd.zbase + (j + 1) * bd.zstride, nz);
    }
    double* Xb = X + bd.xoff;
    for (int idx = tid; idx < me * ne; idx += nt) {
        const int i = idx / ne, k = idx - i * ne;
        const double v = St.row(i)[k];
        Xb[idx] = (accumulate & 1) ? Xb[idx] + v : v;
    }
    if (res.R != nullptr) {
        if constexpr (kGS) {
            // the epilogue reuses the LDS: the band rows go back to their slot rows
            __syncthreads();
            for (int idx = tid; idx < St.nb * LD; idx += nt) S[(St.b0 + idx / LD) * LD + idx % LD] = St.l[idx];
            __syncthreads();
        }
        // R = E - (A X B + C X D) from the solution still held in S (the
        // block is the whole parity problem: outside it X is zero).  Tiles of
        // 64 rows by TK columns; a lane owns a row, a wave a run of columns
        // taken in groups of kRG, along which the 6 x 4 window of X under the
        // stencil slides.  The work is one flat sequence of (tile, group)
        // items, the same for every thread, and E of the next item is
        // requested before the current one is computed (one wave per SIMD
        // leaves nothing else to hide the latency).  With the state in global
        // memory each tile of X and its halo is first staged in LDS, whose
        // records are no longer needed.
        constexpr int kRG = 16;
        constexpr int TK = kGS ? kResTileK : LD;
        constexpr int TS = kResTileK + 3;
        const int lane = tid & 63;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nt >> 6;
        const double* at = res.atab + bd.w * res.a_wstride + (bd.pr ? res.me0 * 12 : 0);
        const double* zt = res.ztabA + (bd.pz ? res.ne0 * 8 : 0);
        const double* Eb = as_global(E) + bd.eoff;
        double* Rb = as_global(res.R) + bd.eoff;
        const int ntk = (ne + TK - 1) / TK;
        const int kcmax = ((ne < TK ? ne : TK) + nw - 1) / nw;
        const int ng = (kcmax + kRG - 1) / kRG;
        const int items = ((me + 63) / 64) * ntk * ng;
        // item t: rows i0 .. i0+63, tile columns k0 .. k0+kw-1; this wave's
        // columns kb .. ke-1 of the tile, this group's kg .. kg+kRG-1
        struct Item { int i0, k0, kw, kb, ke, kg; };
        auto item = [&](int t) {
            Item r;
            const int g = t % ng, tile = t / ng;
            r.i0 = (tile / ntk) * 64;
            r.k0 = (tile % ntk) * TK;
            r.kw = ne - r.k0 < TK ? ne - r.k0 : TK;
            const int kc = (r.kw + nw - 1) / nw;
            r.kb = r.k0 + wv * kc;
            r.ke = r.kb + kc < r.k0 + r.kw ? r.kb + kc : r.k0 + r.kw;
            r.kg = r.kb + g * kRG;
            return r;
        };
        double en[kRG];
        auto load_e = [&](int t) {
            const Item c = item(t);
            const int i = c.i0 + lane;
#pragma unroll
            for (int q = 0; q < kRG; ++q)
                en[q] = i < me && c.kg + q < c.ke ? Eb[static_cast<int64_t>(c.kg + q) * mp + i] : 0.0;
        };
        // the block's row and column records go to LDS (read as vector loads,
        // each use would wait for the whole memory queue, prefetches included)
        double* as = kGS ? sm + (64 + 5) * TS : RCs;
        double* zs = kGS ? as + 12 * mp : ZCs;
        for (int idx = tid; idx < me * 12; idx += nt) as[idx] = at[idx];
        for (int idx = tid; idx < ne * 8; idx += nt) zs[idx] = zt[idx];
        __syncthreads();
        double a[12], x[6][4];
        if (items > 0) load_e(0);
        for (int t = 0; t < items; ++t) {
            const Item c = item(t);
            const int i = c.i0 + lane;
            double ec[kRG];
#pragma unroll
            for (int q = 0; q < kRG; ++q) ec[q] = en[q];
            if (t + 1 < items) load_e(t + 1);
            auto xv = [&](int r, int col) {
                if (kGS) return sm[(r - c.i0 + 2) * TS + (col - c.k0 + 1)];
                return (r >= 0 && r < me && col >= 0 && col < ne) ? S[r * LD + col] : 0.0;
            };
            if (c.kg == c.kb) {                 // first group of a tile
                if (kGS) {
                    __syncthreads();
                    for (int idx = tid; idx < (64 + 5) * (c.kw + 3); idx += nt) {
                        const int rr = idx / (c.kw + 3), cc = idx - rr * (c.kw + 3);
                        const int r = c.i0 - 2 + rr, col = c.k0 - 1 + cc;
                        sm[rr * TS + cc] = (r >= 0 && r < me && col >= 0 && col < ne) ? S[r * LD + col] : 0.0;
                    }
                    __syncthreads();
                }
                if (i < me && c.kb < c.ke) {
#pragma unroll
                    for (int q = 0; q < 12; ++q) a[q] = as[i * 12 + q];
#pragma unroll
                    for (int da = 0; da < 6; ++da)
#pragma unroll
                        for (int dl = 0; dl < 3; ++dl) x[da][dl + 1] = xv(i - 2 + da, c.kb - 1 + dl);
                }
            }
            if (i >= me || c.kg >= c.ke) continue;
#pragma unroll
            for (int q = 0; q < kRG; ++q) {
                const int k = c.kg + q;
                if (k >= c.ke) break;
#pragma unroll
                for (int da = 0; da < 6; ++da) {
#pragma unroll
                    for (int dl = 0; dl < 3; ++dl) x[da][dl] = x[da][dl + 1];
                    x[da][3] = xv(i - 2 + da, k + 2);
                }
                const double* zc = zs + k * 8;
                double sab = 0.0, scd = 0.0;
#pragma unroll
                for (int da = 0; da < 6; ++da) {
                    double xb = 0.0, xd = 0.0;
#pragma unroll
                    for (int dl = 0; dl < 4; ++dl) {
                        xb += x[da][dl] * zc[dl];
                        xd += x[da][dl] * zc[4 + dl];
                    }
                    sab += a[da] * xb;
                    scd += a[6 + da] * xd;
                }
                Rb[static_cast<int64_t>(k) * mp + i] = ec[q] - sab - scd;
            }
        }
    }
}

// Next block of a work-queue launch (kQueue): thread 0 takes the next index
// from the launch's counter; every thread returns it (>= n: the queue is
// drained, every wave leaves).  The leading barrier keeps the previous block's
// LDS use and index reads ahead of the update.
__device__ __forceinline__ int queue_next(int* counter, int* slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    // uniform across the workgroup: keep the block's descriptor in scalar registers
    return __builtin_amdgcn_readfirstlane(*slot);
}

// kQueue: a persistent launch over a cost-sorted queue of `nblocks` blocks
// (grid at most the resident workgroups) of a batch: the per-problem pointer
// table is required and no residual is formed; otherwise block blockIdx.x.
template <int NP, int GB, bool kQueue>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_adi_split(const BlockDesc* __restrict__ blocks, const double* __restrict__ E, double* X,
                 const double* __restrict__ rtab, const double* __restrict__ ztab,
                 const double* __restrict__ vmu, int accumulate, const AdiPtrs* __restrict__ pp,
                 ResArgs res, int* queue, int nblocks) {
    extern __shared__ double sm[];
    if constexpr (!kQueue) {
        const BlockDesc bd = blocks[blockIdx.x];
        if (pp != nullptr) {
            const AdiPtrs q = pp[bd.prob];
            E = q.E; X = q.X; rtab = q.rtab; ztab = q.ztab; vmu = q.vmu;
        }
        adi_block_split<NP + 1, false, GB>(sm, nullptr, bd, E, X, rtab, ztab, vmu, accumulate, res);
    } else {
        __shared__ int qslot;
        for (int b = queue_next(queue, &qslot); b < nblocks; b = queue_next(queue, &qslot)) {
            const BlockDesc bd = blocks[b];
            const AdiPtrs q = pp[bd.prob];
            adi_block_split<NP + 1, false, GB>(sm, nullptr, bd, q.E, q.X, q.rtab, q.ztab, q.vmu, accumulate,
                                               ResArgs{nullptr, nullptr, nullptr, 0, 0, 0});
        }
    }
}

// Blocks too large for LDS (n up to 514): split sweeps with the state in
// global memory, slot blockIdx.x of `state` (state_stride doubles each).
// Row stride of the global-memory block state: np rounded up to 16 doubles,
// so that every row starts on a 128-byte cache line (the r-sweeps read and
// write whole lines of a row, the z-sweeps groups of 16 columns); the LDS
// kernels pad to np + 1 against bank conflicts instead.
__host__ __device__ constexpr int gs_row_stride(int np) { return (np + 15) / 16 * 16; }

// kQueue as for k_adi_split; the state slot is the workgroup's.
template <int NP, int GZF, bool kQueue>
__global__ __launch_bounds__(512) void k_adi_split_gs(const BlockDesc* __restrict__ blocks,
                                                      const double* __restrict__ E, double* X,
                                                      double* state, int64_t state_stride,
                                                      const double* __restrict__ rtab,
                                                      const double* __restrict__ ztab,
                                                      const double* __restrict__ vmu, int accumulate,
                                                      const AdiPtrs* __restrict__ pp, ResArgs res, int* queue,
                                                      int nblocks, int lds_doubles) {
    extern __shared__ double sm[];
    double* slot = state + static_cast<int64_t>(blockIdx.x) * state_stride;
    if constexpr (!kQueue) {
        const BlockDesc bd = blocks[blockIdx.x];
        if (pp != nullptr) {
            const AdiPtrs q = pp[bd.prob];
            E = q.E; X = q.X; rtab = q.rtab; ztab = q.ztab; vmu = q.vmu;
        }
        adi_block_split<gs_row_stride(NP), true, 8, GZF>(sm, slot, bd, E, X, rtab, ztab, vmu, accumulate, res,
                                                         lds_doubles);
    } else {
        __shared__ int qslot;
        for (int b = queue_next(queue, &qslot); b < nblocks; b = queue_next(queue, &qslot)) {
            const BlockDesc bd = blocks[b];
            const AdiPtrs q = pp[bd.prob];
            adi_block_split<gs_row_stride(NP), true, 8, GZF>(sm, slot, bd, q.E, q.X, q.rtab, q.ztab, q.vmu, accumulate,
                                                             ResArgs{nullptr, nullptr, nullptr, 0, 0, 0}, lds_doubles);
        }
    }
}

// ---------------------------------------------------------------------------
// HBM-resident variant (blocks too large for LDS): runtime strides; the
// state of block b lives at state + b * state_stride (rows padded to mp,
// columns to np, row stride np + 1, 4 guard rows), records are read from the
// tables directly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rpass_gen(double* __restrict__ S, int ld, int mp, int k,
                                          const double* __restrict__ RC,
                                          const double* __restrict__ Ecol, double vmu) {
    auto erow = [&](int r) { return Ecol[min(r, mp - 1)]; };
    double* Sk = S + k;
    double wv[14];
    wv[0] = 0.0; wv[1] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) wv[2 + q] = Sk[q * ld];
    double eb[G], en[G];
#pragma unroll
    for (int q = 0; q < G; ++q) { eb[q] = erow(q); en[q] = erow(G + q); }
    double g1 = 0.0, g2 = 0.0;
    for (int i0 = 0; i0 < mp; i0 += G) {
        double c[G][8];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int t = 0; t < 8; ++t) c[q][t] = RC[(i0 + q) * kRRec + t];
#pragma unroll
        for (int q = 0; q < 8; ++q) wv[6 + q] = Sk[(i0 + 4 + q) * ld];
        double enn[G];
#pragma unroll
        for (int q = 0; q < G; ++q) enn[q] = erow(i0 + 2 * G + q);
        double h[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
            h[q] = c[q][0] * wv[q] + c[q][1] * wv[q + 1] + c[q][2] * wv[q + 2] +
                   c[q][3] * wv[q + 3] + c[q][4] * wv[q + 4] + c[q][5] * wv[q + 5] - vmu * eb[q];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double t = h[q] - c[q][6] * g2;
            const double g = t - c[q][7] * g1;
            Sk[(i0 + q) * ld] = g;
            g2 = g1;
            g1 = g;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) wv[q] = wv[8 + q];
#pragma unroll
        for (int q = 0; q < G; ++q) { eb[q] = en[q]; en[q] = enn[q]; }
    }
    double gb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) gb[q] = Sk[(mp - G + q) * ld];
    double z1 = 0.0, z2 = 0.0, z3 = 0.0;
    for (int i0 = mp - G; i0 >= 0; i0 -= G) {
        double c[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t) c[q][t] = RC[(i0 + q) * kRRec + 8 + t];
        double gn[G];
        if (i0 > 0) {
#pragma unroll
            for (int q = 0; q < G; ++q) gn[q] = Sk[(i0 - G + q) * ld];
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const double t = c[q][0] * gb[q] - c[q][3] * z3 - c[q][2] * z2;
            const double z = t - c[q][1] * z1;
            Sk[(i0 + q) * ld] = z;
            z3 = z2; z2 = z1; z1 = z;
        }
#pragma unroll
        for (int q = 0; q < G; ++q) gb[q] = gn[q];
    }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_adi_global(const BlockDesc* __restrict__ blocks, const double* __restrict__ E, double* X,
                  double* state, int64_t state_stride, const double* __restrict__ rtab,
                  const double* __restrict__ ztab, const double* __restrict__ vmu,
                  int accumulate, const AdiPtrs* __restrict__ pp) {
    const BlockDesc bd = blocks[blockIdx.x];
    if (pp != nullptr) {
        const AdiPtrs q = pp[bd.prob];
        E = q.E; X = q.X; rtab = q.rtab; ztab = q.ztab; vmu = q.vmu;
    }
    const int me = bd.me, ne = bd.ne, mp = bd.mp, np = bd.np;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ld = np + 1;
    double* S = state + static_cast<int64_t>(blockIdx.x) * state_stride;
    for (int idx = tid; idx < (mp + 4) * ld; idx += nt) S[idx] = 0.0;
    const double* Ecol = E + bd.eoff + static_cast<int64_t>(tid) * mp;
    for (int j = 0; j < bd.J; ++j) {
        const double* RC = rtab + bd.rbase + j * bd.rstride;
        const double* ZC = ztab + bd.zbase + j * bd.zstride;
        const double vm = vmu[bd.soff + j];
        __syncthreads();
        if (tid < ne) rpass_gen(S, ld, mp, tid, RC, Ecol, vm);
        __syncthreads();
        if (tid < me) zpass(S + tid * ld, np, ZC, j == bd.J - 1);
    }
    __syncthreads();
    double* Xb = X + bd.xoff;
    for (int idx = tid; idx < me * ne; idx += nt) {
        const int i = idx / ne, k = idx - i * ne;
        const double v = S[i * ld + k];
        Xb[idx] = accumulate ? Xb[idx] + v : v;
    }
}

// ---------------------------------------------------------------------------
// tau right-hand side (eq. HelmholtzMatEqn, right side, with r^2 weighting):
//   E = sF [R2 (F + cL L) C02^T]_tau + sL [A_w L C02^T + R2 L D2^T]_tau
// written into the parity blocks (E-layout) of each real mode plane.
// One workgroup per (w, 64 tau rows, 16 tau columns): the input tile
// (rows i0-2 .. i0+69, columns k0 .. k0+19, both real planes of w as one
// complex value) is staged in LDS with reads along r; the z taps (C02, 3)
// and then the r taps (R2, 5) are applied separably; each store writes 32
// consecutive rows of one parity block's column.
// ---------------------------------------------------------------------------
constexpr int kRI = 64, kRK = 16;
constexpr int kRA = kRI + 8, kRL = kRK + 4;

template <bool kLift>
__global__ __launch_bounds__(256) void k_rhs(const double2* __restrict__ F,
                                             const double2* __restrict__ L, double sF, double cL,
                                             double sL, double* __restrict__ E,
                                             const BlockDesc* __restrict__ blocks,
                                             const int* __restrict__ plane_of, int m, int n,
                                             RhsTables t) {
    extern __shared__ double2 rsm[];
    double2* fs = rsm;                  // [kRL][kRA]  F + cL L
    double2* gs = fs + kRL * kRA;       // [kRK][kRA]  (F + cL L) C02^T
    double2* lt = gs + kRK * kRA;       // lift only: [kRL][kRA] L
    double2* gl = lt + kRL * kRA;       //            [kRK][kRA] L C02^T
    double2* ld = gl + kRK * kRA;       //            [kRK][kRA] L D2^T
    // Tiles in XCD-aware order (as in k_recombine): neighbouring tiles share
    // their halo rows of F, and run on one XCD at about the same time.
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned G = gx * gy * gridDim.z;
    const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned xcd = lin & 7u, rem = G & 7u;
    const unsigned g = xcd * (G >> 3) + (xcd < rem ? xcd : rem) + (lin >> 3);
    const int w = static_cast<int>(g / (gx * gy));
    const int i0 = static_cast<int>((g / gy) % gx) * kRI, k0 = static_cast<int>(g % gy) * kRK;
    const int mi = m - 2, ni = n - 2, tid = threadIdx.x;
    const double2* Fw = F + static_cast<int64_t>(w) * n * m;
    const double2* Lw = kLift ? L + static_cast<int64_t>(w) * n * m : nullptr;
    // 256 threads: every load of the tile is issued before the first is used
    constexpr int kIt = (kRL * kRA + 255) / 256;
    double2 fv[kIt], lvv[kLift ? kIt : 1];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = tid + 256 * it;
        const int ll = idx / kRA, al = idx - ll * kRA;
        const int a = i0 - 2 + al, l = k0 + ll;
        const bool in = idx < kRL * kRA && a >= 0 && a < m && l < n;
        fv[it] = in ? Fw[static_cast<int64_t>(l) * m + a] : make_double2(0.0, 0.0);
        if (kLift) lvv[it] = in ? Lw[static_cast<int64_t>(l) * m + a] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = tid + 256 * it;
        if (idx >= kRL * kRA) break;
        double2 f = fv[it];
        if (kLift) {
            const double2 lv = lvv[kLift ? it : 0];
            lt[idx] = lv;
            f = make_double2(f.x + cL * lv.x, f.y + cL * lv.y);
        }
        fs[idx] = f;
    }
    __syncthreads();
    for (int idx = tid; idx < kRK * kRA; idx += blockDim.x) {
        const int kl = idx / kRA, al = idx - kl * kRA;
        const int k = k0 + kl;
        double2 g = make_double2(0.0, 0.0), gL = g, dL = g;
        if (k < ni) {
            const double* c = t.c02 + 3 * k;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const double2 v = fs[(kl + 2 * s) * kRA + al];
                g = make_double2(g.x + c[s] * v.x, g.y + c[s] * v.y);
                if (kLift) {
                    const double2 u = lt[(kl + 2 * s) * kRA + al];
                    gL = make_double2(gL.x + c[s] * u.x, gL.y + c[s] * u.y);
                }
            }
            if (kLift) {
                const double d = t.d2[k];
                const double2 u = lt[(kl + 2) * kRA + al];
                dL = make_double2(d * u.x, d * u.y);
            }
        }
        gs[idx] = g;
        if (kLift) { gl[idx] = gL; ld[idx] = dL; }
    }
    __syncthreads();
    const int il = tid & 31, rest = tid >> 5;
    const int p0 = plane_of[2 * w], p1 = plane_of[2 * w + 1];
    const double ww = static_cast<double>(w) * w;
    for (int c = 0; c < (2 * kRK) / 8; ++c) {
        const int combo = rest + 8 * c;
        const int pr = combo & 1, kl = combo >> 1;
        const int i = i0 + 2 * il + pr, k = k0 + kl;
        if (i >= mi || k >= ni) continue;
        const double* r2 = t.r2 + 5 * i;
        const double2* gk = gs + kl * kRA + (i - i0);
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int ta = 0; ta < 5; ++ta) {
            const double2 v = gk[2 * ta];
            acc = make_double2(acc.x + r2[ta] * v.x, acc.y + r2[ta] * v.y);
        }
        acc = make_double2(sF * acc.x, sF * acc.y);
        if (kLift) {
            const double* a0 = t.a0 + 4 * i;
            const double* s10 = t.s10 + 4 * i;
            const double2* glk = gl + kl * kRA + (i - i0);
            const double2* ldk = ld + kl * kRA + (i - i0);
            double2 la = make_double2(0.0, 0.0);
#pragma unroll
            for (int ta = 0; ta < 4; ++ta) {
                const double aw = a0[ta] - ww * s10[ta];
                const double2 v = glk[2 * ta];
                la = make_double2(la.x + aw * v.x, la.y + aw * v.y);
            }
#pragma unroll
            for (int ta = 0; ta < 5; ++ta) {
                const double2 v = ldk[2 * ta];
                la = make_double2(la.x + r2[ta] * v.x, la.y + r2[ta] * v.y);
            }
            acc = make_double2(acc.x + sL * la.x, acc.y + sL * la.y);
        }
        const int bsel = 2 * pr + (k & 1);
        const BlockDesc& b0 = blocks[4 * p0 + bsel];
        const int64_t o = static_cast<int64_t>(k >> 1) * b0.mp + (i >> 1);
        E[b0.eoff + o] = acc.x;
        if (p1 >= 0) E[blocks[4 * p1 + bsel].eoff + o] = acc.y;
    }
}

// ---------------------------------------------------------------------------
// recombination U = Q_m Xt Q_n^T (+ L) into complex coefficient planes:
//   U[a, l] = Xt[a-2, l-2] - Xt[a-2, l] - Xt[a, l-2] + Xt[a, l].
// One workgroup per (w, 64 r-points, 32 z-points): the Xt tile of both real
// planes (rows a0-2 .. a0+63, columns l0-2 .. l0+31) is read along z from the
// row-major parity blocks into LDS, and the planes are written along r.
// ---------------------------------------------------------------------------
constexpr int kCA = 64, kCL = 32;
constexpr int kCS = kCA + 3;          // LDS row length (odd: conflict-free both ways)

__global__ __launch_bounds__(256) void k_recombine(const double* __restrict__ X,
                                                   const double2* __restrict__ L,
                                                   double2* __restrict__ planes,
                                                   const int* __restrict__ plane_of,
                                                   const BlockDesc* __restrict__ blocks, int m,
                                                   int n) {
    __shared__ double2 xs[(kCL + 2) * kCS];
    // Tiles in XCD-aware order: workgroup b (linear, x fastest) runs on XCD
    // b mod 8 and takes tile g = (b mod 8) G/8 + min(b mod 8, G mod 8) + b/8
    // (a permutation of the G tiles), tiles counted with l fastest, so that
    // neighbouring l-tiles, which read the same cache lines of the X rows,
    // run on one XCD at about the same time.
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned G = gx * gy * gridDim.z;
    const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned xcd = lin & 7u, rem = G & 7u;
    const unsigned g = xcd * (G >> 3) + (xcd < rem ? xcd : rem) + (lin >> 3);
    const int w = static_cast<int>(g / (gx * gy));
    const int a0 = static_cast<int>((g / gy) % gx) * kCA, l0 = static_cast<int>(g % gy) * kCL;
    const int mi = m - 2, ni = n - 2, tid = threadIdx.x;
    const int p0 = plane_of[2 * w], p1 = plane_of[2 * w + 1];
    int64_t x0[4], x1[4];
    int neb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        x0[b] = blocks[4 * p0 + b].xoff;
        neb[b] = blocks[4 * p0 + b].ne;
        x1[b] = p1 >= 0 ? blocks[4 * p1 + b].xoff : 0;
    }
    // 256 threads: every load of the tile is issued before the first is used
    constexpr int kIt = ((kCA + 2) * (kCL + 2) + 255) / 256;
    double2 v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = tid + 256 * it;
        const int il = idx / (kCL + 2), kl = idx - il * (kCL + 2);
        const int i = a0 - 2 + il, k = l0 - 2 + kl;
        v[it] = make_double2(0.0, 0.0);
        if (idx < (kCA + 2) * (kCL + 2) && i >= 0 && i < mi && k >= 0 && k < ni) {
            const int b = 2 * (i & 1) + (k & 1);
            const int64_t o = static_cast<int64_t>(i >> 1) * neb[b] + (k >> 1);
            v[it].x = X[x0[b] + o];
            if (p1 >= 0) v[it].y = X[x1[b] + o];
        }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = tid + 256 * it;
        if (idx >= (kCA + 2) * (kCL + 2)) break;
        const int il = idx / (kCL + 2), kl = idx - il * (kCL + 2);
        xs[kl * kCS + il] = v[it];
    }
    __syncthreads();
    for (int idx = tid; idx < kCA * kCL; idx += blockDim.x) {
        const int al = idx % kCA, ll = idx / kCA;
        const int a = a0 + al, l = l0 + ll;
        if (a >= m || l >= n) continue;
        const double2 p = xs[ll * kCS + al], q = xs[(ll + 2) * kCS + al];
        const double2 r = xs[ll * kCS + al + 2], s = xs[(ll + 2) * kCS + al + 2];
        double2 u = make_double2(p.x - q.x - r.x + s.x, p.y - q.y - r.y + s.y);
        const int64_t off = (static_cast<int64_t>(w) * n + l) * m + a;
        if (L != nullptr) {
            const double2 lv = L[off];
            u.x += lv.x;
            if (p1 >= 0) u.y += lv.y;
        }
        planes[off] = u;
    }
}

// ---------------------------------------------------------------------------
// out = sE E - sAB (A X B) - sCD (C X D), blockwise; X in X-layout, E and out
// in E-layout.  One workgroup per 32 x 32 output tile; the X tile with its
// halo (rows -2..+3, columns -1..+2) and the tile's column records are
// staged in LDS; each thread keeps its row's records in registers and
// produces four outputs of that row.
// ---------------------------------------------------------------------------
constexpr int kTile = 32;
constexpr int kTR = kTile + 5, kTC = kTile + 3;
constexpr int kTS = kTC + 2;          // odd LDS row length (conflict-free row reads)

// One 32 x 32 output tile (i0, k0) of block bd; xs, zs: LDS scratch.
__device__ __forceinline__ void apply_tile(double* xs, double* zs, const BlockDesc& bd, int i0, int k0,
                                           const double* __restrict__ E, double sE,
                                           const double* __restrict__ X, double sAB, double sCD,
                                           double* __restrict__ out, const double* __restrict__ atab,
                                           int64_t a_wstride, int me0,
                                           const double* __restrict__ ztabA, int ne0) {
    const int me = bd.me, ne = bd.ne;
    const int tid = threadIdx.x;
    const double* Xb = X + bd.xoff;
    // 256 threads: every load of the tile is issued before the first is used
    constexpr int kIt = (kTR * kTC + 255) / 256;
    double xv[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = tid + 256 * it;
        const int r = idx / kTC, c = idx - r * kTC;
        const int a = i0 - 2 + r, l = k0 - 1 + c;
        xv[it] = (idx < kTR * kTC && a >= 0 && a < me && l >= 0 && l < ne) ? Xb[static_cast<int64_t>(a) * ne + l]
                                                                          : 0.0;
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int idx = tid + 256 * it;
        if (idx >= kTR * kTC) break;
        const int r = idx / kTC, c = idx - r * kTC;
        xs[r * kTS + c] = xv[it];
    }
    const double* zcol = ztabA + (bd.pz ? ne0 * 8 : 0);
    for (int idx = tid; idx < kTile * 8; idx += blockDim.x) {
        const int k = k0 + (idx >> 3);
        zs[idx] = k < ne ? zcol[k0 * 8 + idx] : 0.0;
    }
    __syncthreads();
    const int di = tid & 31, kq = tid >> 5;
    const int i = i0 + di;
    if (i >= me) return;
    const double* ar = atab + bd.w * a_wstride + (bd.pr ? me0 * 12 : 0) + i * 12;
    double a[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) a[q] = ar[q];
#pragma unroll
    for (int c = 0; c < kTile / 8; ++c) {
        const int dk = kq + 8 * c, k = k0 + dk;
        if (k >= ne) continue;
        const double* zc = zs + dk * 8;
        double sab = 0.0, scd = 0.0;
#pragma unroll
        for (int da = 0; da < 6; ++da) {
            double xb = 0.0, xd = 0.0;
#pragma unroll
            for (int dl = 0; dl < 4; ++dl) {
                const double x = xs[(di + da) * kTS + dk + dl];
                xb += x * zc[dl];
                xd += x * zc[4 + dl];
            }
            sab += a[da] * xb;
            scd += a[6 + da] * xd;
        }
        const int64_t o = bd.eoff + static_cast<int64_t>(k) * bd.mp + i;
        const double ev = (sE != 0.0) ? sE * E[o] : 0.0;
        out[o] = ev - sAB * sab - sCD * scd;
    }
}

__global__ __launch_bounds__(256) void k_apply(const BlockDesc* __restrict__ blocks,
                                               const double* __restrict__ E, double sE,
                                               const double* __restrict__ X, double sAB,
                                               double sCD, double* __restrict__ out,
                                               const double* __restrict__ atab, int64_t a_wstride,
                                               int me0, const double* __restrict__ ztabA, int ne0) {
    __shared__ double xs[kTR * kTS];
    __shared__ double zs[kTile * 8];
    // Tiles in XCD-aware order (as in k_recombine), rows fastest: neighbouring
    // tiles share halo rows and columns of X and run on one XCD at about the
    // same time.
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned G = gx * gy * gridDim.z;
    const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned xcd = lin & 7u, rem = G & 7u;
    const unsigned g = xcd * (G >> 3) + (xcd < rem ? xcd : rem) + (lin >> 3);
    const BlockDesc bd = blocks[g / (gx * gy)];
    const int i0 = static_cast<int>(g % gx) * kTile, k0 = static_cast<int>((g / gx) % gy) * kTile;
    if (i0 >= bd.me || k0 >= bd.ne) return;
    apply_tile(xs, zs, bd, i0, k0, E, sE, X, sAB, sCD, out, atab, a_wstride, me0, ztabA, ne0);
}

__global__ __launch_bounds__(256) void k_apply_batch(const ApplyItem* __restrict__ items,
                                                     const BlockDesc* __restrict__ blocks,
                                                     const ApplyPtrs* __restrict__ pp, double sE,
                                                     double sAB, double sCD) {
    __shared__ double xs[kTR * kTS];
    __shared__ double zs[kTile * 8];
    const ApplyItem it = items[blockIdx.x];
    const BlockDesc bd = blocks[it.block];
    const ApplyPtrs q = pp[bd.prob];
    apply_tile(xs, zs, bd, it.ti * kTile, it.tk * kTile, q.E, sE, q.X, sAB, sCD, q.out, q.atab,
               q.a_wstride, q.me0, q.ztabA, q.ne0);
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

// Batched heat right side: workgroup g belongs to the item q with
// wg_start[q] <= g < wg_start[q + 1]; 256 threads x 4 elements per workgroup.
__global__ __launch_bounds__(256) void k_heat_rhs_batch(const HeatRhsItem* __restrict__ items,
                                                        int nitems,
                                                        const int64_t* __restrict__ wg_start) {
    const int64_t g = blockIdx.x;
    int lo = 0, hi = nitems;                 // wg_start[lo] <= g < wg_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wg_start[mid] <= g) lo = mid; else hi = mid;
    }
    const HeatRhsItem it = items[lo];
    const int64_t base = (g - wg_start[lo]) * 1024 + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t e = base + c * 256;
        if (e >= it.total) break;
        double acc = it.Ec[e];
#pragma unroll
        for (int b = 0; b < 4; ++b)          // fixed bound: the item stays in registers
            if (b < it.nb) acc += it.beta[b] * it.P[b][e];
        it.E[e] = acc;
    }
}

__global__ __launch_bounds__(256) void k_norms(const double* __restrict__ R,
                                               const double* __restrict__ E, int64_t etotal,
                                               const double* __restrict__ X, int64_t xtotal,
                                               double* acc) {
    __shared__ double red[3][256];
    double r2 = 0.0, e2 = 0.0, bad = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < etotal; e += stride) {
        const double r = R[e], ev = E[e];
        r2 += r * r;
        e2 += ev * ev;
    }
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < xtotal; e += stride)
        if (!isfinite(X[e])) bad += 1.0;
    red[0][threadIdx.x] = r2; red[1][threadIdx.x] = e2; red[2][threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) atomicAdd(&acc[threadIdx.x], red[threadIdx.x][0]);
}

template <int NP>
hipError_t launch_lds(const BlockDesc* blocks, int nblocks, int threads, const double* E,
                      double* X, const double* rtab, const double* ztab, const double* vmu,
                      bool accumulate, size_t lds_bytes, hipStream_t s, const AdiPtrs* pp) {
    hipLaunchKernelGGL(k_adi_lds<NP>, dim3(nblocks), dim3(threads), lds_bytes, s, blocks, E, X,
                           rtab, ztab, vmu, accumulate ? 1 : 0, pp);
    return hipGetLastError();
}

// The dynamic-LDS limit of a kernel only ever grows: plans of different
// sizes share the kernel instances, and a smaller plan created later must not
// lower the limit a larger one launches with (kept per device).
hipError_t raise_lds_limit(const void* fn, size_t bytes) {
    int dev = 0;
    const hipError_t d = hipGetDevice(&dev);
    if (d != hipSuccess) return d;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> set;
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = set[{dev, fn}];
    if (bytes <= cur) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
    if (e == hipSuccess) cur = bytes;
    return e;
}

template <int NP>
hipError_t set_limit(size_t bytes) {
    return raise_lds_limit(reinterpret_cast<const void*>(&k_adi_lds<NP>), bytes);
}

// CYLSPEC_ADI_POISON=1 (tests): the split kernels poison their LDS first
// (bit 1 of their accumulate argument).
int lds_poison() {
    const char* v = std::getenv("CYLSPEC_ADI_POISON");
    return (v && *v && *v != '0') ? 2 : 0;
}

template <int NP>
hipError_t launch_split(const BlockDesc* blocks, int nblocks, int threads, const double* E,
                        double* X, const double* rtab, const double* ztab, const double* vmu,
                        bool accumulate, size_t lds_bytes, hipStream_t s, const AdiPtrs* pp,
                        const ResArgs& res, bool g16, const BlockQueue* q) {
    const int acc = (accumulate ? 1 : 0) | lds_poison();
    if (q != nullptr && (pp == nullptr || q->counter == nullptr)) return hipErrorInvalidValue;
    if (q != nullptr) {
        const dim3 grid(static_cast<unsigned>(std::min(q->grid, nblocks)));
        if (g16)
            hipLaunchKernelGGL((k_adi_split<NP, 16, true>), grid, dim3(threads), lds_bytes, s, blocks, E, X, rtab,
                               ztab, vmu, acc, pp, res, q->counter, nblocks);
        else
            hipLaunchKernelGGL((k_adi_split<NP, G, true>), grid, dim3(threads), lds_bytes, s, blocks, E, X, rtab,
                               ztab, vmu, acc, pp, res, q->counter, nblocks);
    } else if (g16) {
        hipLaunchKernelGGL((k_adi_split<NP, 16, false>), dim3(nblocks), dim3(threads), lds_bytes, s, blocks, E, X,
                           rtab, ztab, vmu, acc, pp, res, nullptr, nblocks);
    } else {
        hipLaunchKernelGGL((k_adi_split<NP, G, false>), dim3(nblocks), dim3(threads), lds_bytes, s, blocks, E, X,
                           rtab, ztab, vmu, acc, pp, res, nullptr, nblocks);
    }
    return hipGetLastError();
}

template <int NP>
hipError_t launch_split_gs(const BlockDesc* blocks, int nblocks, int threads, const double* E, double* X,
                           double* state, int64_t state_stride, const double* rtab, const double* ztab,
                           const double* vmu, bool accumulate, size_t lds_bytes, hipStream_t s,
                           const AdiPtrs* pp, const ResArgs& res, bool z16, const BlockQueue* q) {
    const int acc = (accumulate ? 1 : 0) | lds_poison();
    const int band = static_cast<int>(lds_bytes / sizeof(double));   // LDS doubles (the band takes the rest)
    if (q != nullptr && (pp == nullptr || q->counter == nullptr)) return hipErrorInvalidValue;
    if (q != nullptr) {
        const dim3 grid(static_cast<unsigned>(std::min(q->grid, nblocks)));
        if (z16)
            hipLaunchKernelGGL((k_adi_split_gs<NP, 16, true>), grid, dim3(threads), lds_bytes, s, blocks, E, X,
                               state, state_stride, rtab, ztab, vmu, acc, pp, res, q->counter, nblocks, band);
        else
            hipLaunchKernelGGL((k_adi_split_gs<NP, 8, true>), grid, dim3(threads), lds_bytes, s, blocks, E, X,
                               state, state_stride, rtab, ztab, vmu, acc, pp, res, q->counter, nblocks, band);
    } else if (z16) {
        hipLaunchKernelGGL((k_adi_split_gs<NP, 16, false>), dim3(nblocks), dim3(threads), lds_bytes, s, blocks, E,
                           X, state, state_stride, rtab, ztab, vmu, acc, pp, res, nullptr, nblocks, band);
    } else {
        hipLaunchKernelGGL((k_adi_split_gs<NP, 8, false>), dim3(nblocks), dim3(threads), lds_bytes, s, blocks, E,
                           X, state, state_stride, rtab, ztab, vmu, acc, pp, res, nullptr, nblocks, band);
    }
    return hipGetLastError();
}

template <int NP>
hipError_t set_split_limit(size_t bytes) {
    const void* fns[4] = {reinterpret_cast<const void*>(&k_adi_split<NP, G, false>),
                          reinterpret_cast<const void*>(&k_adi_split<NP, 16, false>),
                          reinterpret_cast<const void*>(&k_adi_split<NP, G, true>),
                          reinterpret_cast<const void*>(&k_adi_split<NP, 16, true>)};
    for (const void* f : fns) {
        const hipError_t e = raise_lds_limit(f, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int NP>
hipError_t set_split_gs_limit(size_t bytes) {
    const void* fns[4] = {reinterpret_cast<const void*>(&k_adi_split_gs<NP, 8, false>),
                          reinterpret_cast<const void*>(&k_adi_split_gs<NP, 16, false>),
                          reinterpret_cast<const void*>(&k_adi_split_gs<NP, 8, true>),
                          reinterpret_cast<const void*>(&k_adi_split_gs<NP, 16, true>)};
    for (const void* f : fns) {
        const hipError_t e = raise_lds_limit(f, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

#define CYL_NP_CASES(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64) X(72) X(80) X(88) X(96) \
    X(104) X(112) X(120) X(128)

hipError_t launch_adi(const BlockDesc* blocks, int nblocks, int threads, int np0, const double* E,
                      double* X, double* state, int64_t state_stride, const double* rtab,
                      const double* ztab, const double* vmu, bool accumulate, bool use_lds,
                      size_t lds_bytes, hipStream_t s, const AdiPtrs* pp) {
    if (use_lds) {
        switch (np0) {
#define CYL_CASE(v) case v: return launch_lds<v>(blocks, nblocks, threads, E, X, rtab, ztab, vmu, accumulate, lds_bytes, s, pp);
            CYL_NP_CASES(CYL_CASE)
#undef CYL_CASE
            default: return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(k_adi_global, dim3(nblocks), dim3(threads), 0, s, blocks, E, X, state,
                           state_stride, rtab, ztab, vmu, accumulate ? 1 : 0, pp);
    return hipGetLastError();
}

bool adi_split_gs_z16(const BlockDesc& b) { return b.tz % 16 == 0 && (b.np - b.tz) % 16 == 0; }

bool adi_split_g16(const BlockDesc& b) {
    return b.tr % 16 == 0 && (b.mp - b.tr) % 16 == 0 && b.tz % 16 == 0 && (b.np - b.tz) % 16 == 0;
}

size_t adi_split_lds_bytes(int mp0, int np0) {
    auto chunks = [](int x) { return static_cast<size_t>((x + 127) / 128 * 128); };
    const size_t doubles = static_cast<size_t>(mp0) * (np0 + 1) + chunks((mp0 + kRCouple) * kRRec) +
                           chunks((np0 + kZCouple) * kZRec) + 5 * 128;
    return doubles * sizeof(double);
}

hipError_t launch_adi_split(const BlockDesc* blocks, int nblocks, int threads, int np0,
                            const double* E, double* X, const double* rtab, const double* ztab,
                            const double* vmu, bool accumulate, size_t lds_bytes, hipStream_t s,
                            const AdiPtrs* pp, const ResArgs* res, bool g16, const BlockQueue* q) {
    if (threads < 128 || threads > 256 || threads % 128 != 0) return hipErrorInvalidValue;
    const ResArgs ra = res ? *res : ResArgs{nullptr, nullptr, nullptr, 0, 0, 0};
    switch (np0) {
#define CYL_CASE(v) case v: return launch_split<v>(blocks, nblocks, threads, E, X, rtab, ztab, vmu, accumulate, lds_bytes, s, pp, ra, g16, q);
        CYL_NP_CASES(CYL_CASE)
#undef CYL_CASE
        default: return hipErrorInvalidValue;
    }
}

#define CYL_NP_GS_CASES(X) X(136) X(144) X(152) X(160) X(168) X(176) X(184) X(192) X(200) X(208) \
    X(216) X(224) X(232) X(240) X(248) X(256)

size_t adi_split_gs_lds_bytes(int mp0, int np0, int lines, bool residual) {
    auto chunks = [](int x) { return static_cast<size_t>((x + 127) / 128 * 128); };
    const size_t doubles = chunks((mp0 + kRCouple) * kRRec) + chunks((np0 + kZCouple) * kZRec) +
                           5 * static_cast<size_t>(lines);
    // residual epilogue: staged tile of X, then the row and column records
    const size_t tile = residual ? static_cast<size_t>(64 + 5) * (kResTileK + 3) + 12 * static_cast<size_t>(mp0) +
                                       8 * static_cast<size_t>(np0) : 0;
    return std::max(doubles, tile) * sizeof(double);
}

int64_t adi_split_gs_state_stride(int mp0, int np0) {
    return static_cast<int64_t>(mp0) * gs_row_stride(np0) + 64;
}

hipError_t launch_adi_split_gs(const BlockDesc* blocks, int nblocks, int threads, int np0,
                               const double* E, double* X, double* state, int64_t state_stride,
                               const double* rtab, const double* ztab, const double* vmu,
                               bool accumulate, size_t lds_bytes, hipStream_t s, const AdiPtrs* pp,
                               const ResArgs* res, bool z16, const BlockQueue* q) {
    if (threads < 128 || threads > 512 || threads % 128 != 0) return hipErrorInvalidValue;
    const ResArgs ra = res ? *res : ResArgs{nullptr, nullptr, nullptr, 0, 0, 0};
    switch (np0) {
#define CYL_CASE(v) case v: return launch_split_gs<v>(blocks, nblocks, threads, E, X, state, state_stride, rtab, ztab, vmu, accumulate, lds_bytes, s, pp, ra, z16, q);
        CYL_NP_GS_CASES(CYL_CASE)
#undef CYL_CASE
        default: return hipErrorInvalidValue;
    }
}

namespace {
template <typename K>
hipError_t resident_grid(K kernel, int threads, size_t lds, int* grid) {
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(kernel), threads, lds);
    if (e == hipSuccess) *grid = cus * (per > 0 ? per : 1);
    return e;
}
template <int NP>
hipError_t queue_grid_gs(int threads, size_t lds, bool g16, int* grid) {
    return g16 ? resident_grid(&k_adi_split_gs<NP, 16, true>, threads, lds, grid)
               : resident_grid(&k_adi_split_gs<NP, 8, true>, threads, lds, grid);
}
template <int NP>
hipError_t queue_grid_lds(int threads, size_t lds, bool g16, int* grid) {
    return g16 ? resident_grid(&k_adi_split<NP, 16, true>, threads, lds, grid)
               : resident_grid(&k_adi_split<NP, G, true>, threads, lds, grid);
}
}  // namespace

hipError_t adi_split_queue_grid(int np0, int threads, size_t lds, bool gs, bool g16, int* grid) {
    if (gs) {
        switch (np0) {
#define CYL_CASE(v) case v: return queue_grid_gs<v>(threads, lds, g16, grid);
            CYL_NP_GS_CASES(CYL_CASE)
#undef CYL_CASE
            default: return hipErrorInvalidValue;
        }
    }
    switch (np0) {
#define CYL_CASE(v) case v: return queue_grid_lds<v>(threads, lds, g16, grid);
        CYL_NP_CASES(CYL_CASE)
#undef CYL_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t adi_split_set_lds_limit(int np0, size_t bytes) {
    switch (np0) {
#define CYL_CASE(v) case v: return set_split_limit<v>(bytes);
        CYL_NP_CASES(CYL_CASE)
#undef CYL_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t adi_split_gs_set_lds_limit(int np0, size_t bytes) {
    switch (np0) {
#define CYL_CASE(v) case v: return set_split_gs_limit<v>(bytes);
        CYL_NP_GS_CASES(CYL_CASE)
#undef CYL_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t adi_set_lds_limit(int np0, size_t bytes) {
    switch (np0) {
#define CYL_CASE(v) case v: return set_limit<v>(bytes);
        CYL_NP_CASES(CYL_CASE)
#undef CYL_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rhs3(const double2* F, const double2* L, double sF, double cL, double sL,
                       double* E, const BlockDesc* blocks, const int* plane_of, int nw, int m, int n,
                       const RhsTables& t, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((m - 2 + kRI - 1) / kRI),
                    static_cast<unsigned>((n - 2 + kRK - 1) / kRK), static_cast<unsigned>(nw));
    if (L != nullptr) {
        const size_t lds = static_cast<size_t>(2 * kRL + 3 * kRK) * kRA * sizeof(double2);
        static bool raised = false;
        if (!raised) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rhs<true>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
            if (e != hipSuccess) return e;
            raised = true;
        }
        hipLaunchKernelGGL(k_rhs<true>, grid, dim3(256), lds, s, F, L, sF, cL, sL, E, blocks, plane_of,
                           m, n, t);
    } else {
        const size_t lds = static_cast<size_t>(kRL + kRK) * kRA * sizeof(double2);
        hipLaunchKernelGGL(k_rhs<false>, grid, dim3(256), lds, s, F, L, sF, cL, sL, E, blocks, plane_of,
                           m, n, t);
    }
    return hipGetLastError();
}

hipError_t launch_recombine(const double* X, const double2* L, double2* planes,
                            const int* plane_of, const BlockDesc* blocks, int nw, int m, int n,
                            int p, hipStream_t s) {
    (void)p;
    const dim3 grid(static_cast<unsigned>((m + kCA - 1) / kCA), static_cast<unsigned>((n + kCL - 1) / kCL),
                    static_cast<unsigned>(nw));
    hipLaunchKernelGGL(k_recombine, grid, dim3(256), 0, s, X, L, planes, plane_of, blocks, m, n);
    return hipGetLastError();
}

hipError_t launch_apply2(const BlockDesc* blocks, int nblocks, int me0, int ne0, const double* E,
                         double sE, const double* X, double sAB, double sCD, double* out,
                         const double* atab, int64_t a_wstride, const double* ztabA,
                         hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((me0 + kTile - 1) / kTile),
                    static_cast<unsigned>((ne0 + kTile - 1) / kTile), nblocks);
    hipLaunchKernelGGL(k_apply, grid, dim3(256), 0, s, blocks, E, sE, X, sAB, sCD, out, atab,
                       a_wstride, me0, ztabA, ne0);
    return hipGetLastError();
}

hipError_t launch_apply_batch(const ApplyItem* items, int nitems, const BlockDesc* blocks,
                              const ApplyPtrs* pp, double sE, double sAB, double sCD, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_apply_batch, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, s, items, blocks, pp,
                       sE, sAB, sCD);
    return hipGetLastError();
}

hipError_t launch_heat_rhs_batch(const HeatRhsItem* items, int nitems, const int64_t* wg_start,
                                 int64_t nwg, hipStream_t s) {
    if (nitems <= 0 || nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_heat_rhs_batch, dim3(static_cast<unsigned>(nwg)), dim3(256), 0, s, items, nitems,
                       wg_start);
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

hipError_t launch_norms(const double* R, const double* E, int64_t etotal, const double* X,
                        int64_t xtotal, double* acc, hipStream_t s) {
    int64_t blocks = (etotal + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_norms, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, R, E, etotal,
                       X, xtotal, acc);
    return hipGetLastError();
}

}  // namespace cyl
