// Launchers of the device kernels (plain pointers; called from the C API).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cyl {

// Device view of one DFT length (see DftTables): complex length L computed as
// a mixed-radix FFT of length Nb, directly (L == Nb) or by Bluestein
// (power-of-two Nb).  Pass p of the Stockham FFT has radix rad[p].
constexpr int kMaxDftPasses = 12;
struct DftDev {
    int L, Nb, tpl, bluestein;     // tpl: threads per line
    int pts;                       // points per thread (8 or 16; 16 with a prime pass)
    int nrad;
    int rad[kMaxDftPasses];
    const double2* tw;      // Nb: per-pass twiddles of the Stockham FFT
    const double2* chirp;   // L   (Bluestein only)
    const double2* bhat;    // Nb  (Bluestein only)
};

// Output pairs (X_r, X_{R-r}) one thread computes in the direct pass of a
// prime radix R > 17 (the first pass of such a plan; see transforms.hip).
constexpr int kPrimePassOutputs = 9;

// A family of equally strided lines: line = (o, i), o < n_outer, i < n_inner;
// element e of a line sits at o * outer + i * inner + e * elem (in double2).
struct LineSet {
    int64_t outer, inner, elem;
    int n_outer, n_inner;
};

// One ADI work item: a parity block (w, part, pr, pz) of a real mode plane.
// E-layout (right-hand sides, residuals, heat history): column-major with the
// rows padded to mp, element (i, k) at eoff + k * mp + i, padding rows zero.
// X-layout (solutions): row-major, element (i, k) at xoff + i * ne + k.
struct BlockDesc {
    int w, J, me, ne;
    int mp, np;              // me, ne rounded up to multiples of 8
    int pr, pz, part, plane;
    int tr, tz;              // split rows of the two-thread sweeps (0: not split)
    int prob;                // problem index in a batched launch (0 otherwise)
    int64_t eoff, xoff;
    int64_t rbase, zbase;    // offset of (j = 0) records in rtab / ztab
    int64_t rstride, zstride;// record stride between successive shifts
    int64_t soff;            // offset of v_j - u_j values
};

// Residual emitted by the split ADI kernels after their last iteration
// (R == nullptr: none): R = E - (A X B + C X D) of the block just solved, with
// the records of launch_apply2 (atab rows of 12 per (w, r parity), w stride
// a_wstride; ztabA columns of 8 per z parity), written in E-layout.
struct ResArgs {
    double* R;
    const double* atab;
    const double* ztabA;
    int64_t a_wstride;
    int me0, ne0;
};

// Per-problem pointers of a batched launch, indexed by BlockDesc::prob.  When a
// launcher receives a table, the table's pointers replace the launcher's own.
struct AdiPtrs {
    const double* E;
    double* X;
    const double* rtab;
    const double* ztab;
    const double* vmu;
};
// Work-queue launch of the split kernels (batched launches: the launcher's
// pointer table is required; no residual is formed): `grid` persistent
// workgroups take the blocks of the launch in order from `counter` (an int
// that must be zero when the launch starts; it ends at nblocks + grid).
struct BlockQueue {
    int* counter;
    int grid;
};
struct ApplyPtrs {
    const double* E;
    const double* X;
    double* out;
    const double* atab;
    const double* ztabA;
    int64_t a_wstride;
    int me0, ne0;
};
// One 32 x 32 output tile of a block in a batched apply launch.
struct ApplyItem {
    int block, ti, tk, pad;
};
// Elementwise heat right side of one problem in a batched launch.
struct HeatRhsItem {
    double* E;
    const double* P[4];
    double beta[4];
    const double* Ec;
    int64_t total;
    int nb, pad;
};

// ---- transforms (Section 2) ----
hipError_t launch_theta_fwd(const double* values, double2* planes, int m, int n, int p,
                            const DftDev& d, hipStream_t s);
hipError_t launch_theta_inv(const double2* planes, double* values, int m, int n, int p,
                            const DftDev& d, hipStream_t s);
// DCT-I of every line: out_k = post[k] * sum_n pre[n] in_n * w_n cos(pi k n / M)
// (w_n = 1 at both ends, 2 inside), M = mlen - 1, through a length-M DFT
// (d built for length M); fold[n] = (cos(pi n / M), sin(pi n / M)), n <= M.
// max_lines: strided lines per workgroup at most (0: the default, 8).
hipError_t launch_dct(const double2* in, double2* out, const LineSet& ls, int mlen,
                      bool contiguous_lines, const DftDev& d, const double* pre,
                      const double* post, const double2* fold, hipStream_t s, int max_lines = 0);

// ---- right-hand side (tau rows) and recombination ----
struct RhsTables {
    const double* r2;    // (m-2) x 5 : R2 row i at columns i-2, i, i+2, i+4, i+6
    const double* a0;    // (m-2) x 4 : (R C12 D1 + R^2 D2) row i at i-2, i, i+2, i+4
    const double* s10;   // (m-2) x 4 : C02 row i at i-2, i, i+2, i+4 (first entry 0)
    const double* c02;   // (n-2) x 3 : C02 row k at k, k+2, k+4
    const double* d2;    // (n-2)     : D2 row k at k+2
};
// E = sF [R2 (F + cL L) C02^T]_tau + sL [A_w L C02^T + R2 L D2^T]_tau (L may be NULL)
// plane_of[2 w + part]: real plane of (w, part), -1 if none; nw = floor(p/2) + 1.
hipError_t launch_rhs3(const double2* F, const double2* L, double sF, double cL, double sL,
                       double* E, const BlockDesc* blocks, const int* plane_of, int nw, int m, int n,
                       const RhsTables& t, hipStream_t s);
hipError_t launch_recombine(const double* X, const double2* L, double2* planes,
                            const int* block_of_plane, const BlockDesc* blocks, int nw,
                            int m, int n, int p, hipStream_t s);

// ---- ADI (Algorithm 1) ----
// Coefficient tables hold, per parity block, rows padded to a multiple of 8
// (zero records beyond the block).  state: HBM-resident variant only,
// state_stride doubles per block.
// np0: padded width of the widest block (selects the LDS kernel instance;
// multiples of 8 up to 128).  E-layout buffers need 64 doubles of slack
// after their end (read-ahead of the sweeps; values unused).
hipError_t launch_adi(const BlockDesc* blocks, int nblocks, int threads, int np0, const double* E,
                      double* X, double* state, int64_t state_stride, const double* rtab,
                      const double* ztab, const double* vmu, bool accumulate, bool use_lds,
                      size_t lds_bytes, hipStream_t s, const AdiPtrs* pp = nullptr);
// Split-sweep LDS-resident ADI (tables built with the split layout): two
// threads per line, 2 * lines threads per workgroup (lines a multiple of 64,
// at most 128).
hipError_t launch_adi_split(const BlockDesc* blocks, int nblocks, int threads, int np0,
                            const double* E, double* X, const double* rtab, const double* ztab,
                            const double* vmu, bool accumulate, size_t lds_bytes, hipStream_t s,
                            const AdiPtrs* pp = nullptr, const ResArgs* res = nullptr, bool g16 = false,
                            const BlockQueue* q = nullptr);
// Every half of the block is a multiple of 16 rows / columns (the split kernel's
// backward r sweeps and z sweeps may then take groups of 16; g16 of a launch
// needs it for all its blocks).
bool adi_split_g16(const BlockDesc& b);
// Workgroups of a work-queue split launch (np0, threads, LDS bytes; gs: the
// global-state kernel; g16 its instance) that are resident at once on the
// device: the grid such a launch should use.
hipError_t adi_split_queue_grid(int np0, int threads, size_t lds, bool gs, bool g16, int* grid);
// LDS bytes of the split kernel for padded block sizes mp0 x np0.
size_t adi_split_lds_bytes(int mp0, int np0);
// Split sweeps with the block state in global memory (np0 in 136..256, a
// multiple of 8; threads = 2 lines <= 512): state slot blockIdx.x of `state`,
// state_stride = adi_split_gs_state_stride(mp0, np0) doubles (or more).
hipError_t launch_adi_split_gs(const BlockDesc* blocks, int nblocks, int threads, int np0,
                               const double* E, double* X, double* state, int64_t state_stride,
                               const double* rtab, const double* ztab, const double* vmu,
                               bool accumulate, size_t lds_bytes, hipStream_t s,
                               const AdiPtrs* pp = nullptr, const ResArgs* res = nullptr, bool z16 = false,
                               const BlockQueue* q = nullptr);
// z16: groups of 16 columns in the forward z sweeps; every block must satisfy
// adi_split_gs_z16 (both z halves multiples of 16).
bool adi_split_gs_z16(const BlockDesc& b);
// residual: room for the fused residual epilogue's staged tile
size_t adi_split_gs_lds_bytes(int mp0, int np0, int lines, bool residual);
int64_t adi_split_gs_state_stride(int mp0, int np0);

// Raise the dynamic-LDS limit of the LDS-resident ADI kernels for width np0.
hipError_t adi_set_lds_limit(int np0, size_t bytes);
hipError_t adi_split_set_lds_limit(int np0, size_t bytes);
hipError_t adi_split_gs_set_lds_limit(int np0, size_t bytes);

// Coons lift of the doubled box's faces: rface [2][p][n] (r = -1, +1), zface
// [2][p][m] (z = -1, +1), ra_j = (1 + r_j)/2, zb_k = (1 + z_k)/2 -> lift
// [p][n][m] (boundary.hip).
hipError_t launch_trace_lift(const double* rface, const double* zface, const double* ra, const double* zb,
                             double* lift, int m, int n, int p, hipStream_t s);
// Horizontal (disk) Poisson (disk.hip): U = disk solve of F, planes
// [nw][n][m] complex, U not aliasing F; lu [nw][2][rmax][4] and taps
// [2][rmax][5] as built by build_disk_tables; rows0/rows1: parity row counts;
// the right side is scaled by `scale`.
hipError_t launch_disk(const double2* F, double2* U, const double* lu, const double* taps, int m, int n,
                       int nw, int rmax, int rows0, int rows1, hipStream_t s, double scale = 1.0);
// The lambda solve of the poloidal-toroidal decomposition: U = disk solve of
// the curl right side of (V_theta, V_r) planes; pt_taps [2][rmax][2][5] as
// built by build_disk_tables; wnyq: the Nyquist slot (p/2 for even p, else
// -1), whose theta derivative is taken as zero.  U aliases neither input.
hipError_t launch_disk_pt(const double2* Vt, const double2* Vr, double2* U, const double* lu,
                          const double* pt_taps, int m, int n, int nw, int rmax, int rows0, int rows1, int wnyq,
                          hipStream_t s);
// Device peak checks (peaks.hip).  launch_fma_peak: `blocks` workgroups of
// 256 lanes, each running independent FP64 FMA chains for `iters` rounds;
// *flops receives the launch's FP64 operation count.  launch_copy_peak:
// dst[i] = src[i] for n doubles (16-byte aligned, not overlapping).
hipError_t launch_fma_peak(double* sink, int blocks, int iters, hipStream_t s, double* flops);
hipError_t launch_copy_peak(const double* src, double* dst, int64_t n, int blocks, hipStream_t s);
// Zero the me x ne solution region (at xoff) of every listed block; me0, ne0
// bound the block sizes.
hipError_t launch_zero_blocks(const BlockDesc* blocks, int nblocks, int me0, int ne0, double* X,
                              hipStream_t s);
// out[i] = 0 for i < n, as a kernel (no memset node in a captured graph).
hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t s);

// out = sE * E - sAB * (A X B) - sCD * (C X D) blockwise.  atab: per (w, r
// parity) rows of 12 (A row i at i-2..i+3, then C row i at i-2..i+3), w stride
// a_wstride (0: the same rows for every w); ztabA: per z parity columns of 8
// (B column k at rows k-1..k+2, then D column k at rows k-1..k+2).
hipError_t launch_apply2(const BlockDesc* blocks, int nblocks, int me0, int ne0, const double* E,
                         double sE, const double* X, double sAB, double sCD, double* out,
                         const double* atab, int64_t a_wstride, const double* ztabA,
                         hipStream_t s);

// Batched apply: one workgroup per item (block, 32 x 32 tile); pointers,
// records and sizes of each block's problem from pp; sE, sAB, sCD as above.
hipError_t launch_apply_batch(const ApplyItem* items, int nitems, const BlockDesc* blocks,
                              const ApplyPtrs* pp, double sE, double sAB, double sCD, hipStream_t s);

// ---- heat ----
hipError_t launch_heat_rhs(double* E, const double* const* P, const double* beta, int nb,
                           const double* Econst, int64_t total, hipStream_t s);
// Batched heat right side: wg_start[q] is the first workgroup of item q
// (nitems + 1 entries, the last one the grid size); 1024 elements per workgroup.
hipError_t launch_heat_rhs_batch(const HeatRhsItem* items, int nitems, const int64_t* wg_start,
                                 int64_t nwg, hipStream_t s);

// ---- reductions ----
// acc[0] += sum R^2, acc[1] += sum E^2 (E-layout, etotal entries),
// acc[2] += count of non-finite X (X-layout, xtotal entries)
hipError_t launch_norms(const double* R, const double* E, int64_t etotal, const double* X,
                        int64_t xtotal, double* acc, hipStream_t s);

// ---- adjoint (transposed) operators, flipped block orientation ----
// Adjoint quantities of a parity block are stored flipped: block element
// (i', k') holds the entry (me-1-i', ne-1-k') (see adjoint.hip).
// out (E-layout, flipped) = s * Q_m^T U Q_n per block (transposed recombination).
hipError_t launch_recombine_t(const double2* U, double s, double* out, const BlockDesc* blocks,
                              int nblocks, int64_t max_block_elems, int m, int n, hipStream_t st);
// U (planes) = s * R2^T Y C02 restricted to tau rows (transposed tau right side);
// Y flipped in X-layout.
hipError_t launch_rhs_t(const double* Yf, double s, double2* U, const int* plane_of,
                        const BlockDesc* blocks, int nw, int m, int n, const RhsTables& t,
                        hipStream_t st);
// y += a x
hipError_t launch_axpy(double* y, const double* x, double a, int64_t count, hipStream_t st);
// partials[tile] += sum Yf~ . (A X B + C X D) over each 32 x 32 tile (records as launch_apply2)
int64_t apply_dot_partials(int nblocks, int me0, int ne0);
hipError_t launch_apply_dot(const BlockDesc* blocks, int nblocks, int me0, int ne0, const double* X,
                            const double* Yf, const double* atab, int64_t a_wstride,
                            const double* ztabA, double* partials, hipStream_t st);
// out[0] = scale * sum(partials) (one workgroup, deterministic order)
hipError_t launch_sum(const double* partials, int64_t count, double scale, double* out,
                      hipStream_t st);
// Diagonal factors of the transposed transforms: mode 0 before the inverse
// transform (F^T), mode 1 after the forward transform (F^-T); see adjoint.hip.
hipError_t launch_scale_planes(double2* U, int m, int n, int p, int mode, hipStream_t st);
hipError_t launch_scale_values(const double* in, double* out, int m, int n, int p, int mode,
                               hipStream_t st);

// ---- static scratch of the allocation-free entry point (scratch.hip) ----
// Bytes of the file-scope device array: the largest workspace an
// allocation-free solve may use.
constexpr size_t kScratchBytes = size_t(64) << 20;
// Take (once per device, with that device made current) and cache the
// device address of the scratch array; later calls return at once.
hipError_t scratch_init(int device);
// The cached address for `device` (nullptr before scratch_init succeeded).
void* scratch_device_ptr(int device);

}  // namespace cyl
