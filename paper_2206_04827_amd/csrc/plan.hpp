// Host-side planning for the CCF cylinder solver: banded operators of
// Section 3, spectral bounds, Zolotarev shifts, per-shift LU tables and the
// per-length DFT tables used by the transform kernels.  Pure C++; no HIP.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace cyl {

// Rectangular banded matrix: entry (i, j) is stored iff -lo <= j - i <= hi.
struct Band {
    int rows = 0, cols = 0, lo = 0, hi = 0;
    std::vector<double> v;
    Band() = default;
    Band(int r, int c, int l, int h);
    int width() const { return lo + hi + 1; }
    double get(int i, int j) const;
    void set(int i, int j, double x);
};

Band band_mul(const Band& A, const Band& B);
Band band_axpby(double alpha, const Band& A, double beta, const Band& B);
Band band_cut(const Band& A, int rows, int cols);
Band band_transpose(const Band& A);
// J A^T J for square A (J reverses the index order).  Same band widths as A;
// it turns a transposed banded solve into one of the original shape.
Band band_flip_transpose(const Band& A);
// Rows/columns of one index parity (p = 0 even, 1 odd); the operators here
// never couple the two parities, which is checked.
Band band_parity(const Band& A, int p);

// Operators of eq. (HelmholtzMatEqn) for one direction of size n.
struct DirOps {
    int n = 0;
    // Dirichlet-basis tau matrices, (n-2) x (n-2), full index (not parity split).
    Band A0;   // [(R C12 D1 + R^2 D2) Q]_tau           (radial part, w = 0)
    Band Cc;   // [C02 Q]_tau                            (coefficient of -w^2)
    Band R2Q;  // [R^2 C02 Q]_tau                        (r-direction C)
    Band C02Q; // [C02 Q]_tau                            (z-direction B^T)
    Band D2Q;  // [D2 Q]_tau                             (z-direction D^T)
    // Full T-coefficient operators, n x n, for right-hand sides and lifts.
    Band R2f, C02f, A0f, S10f, D2f;
    // Curl right side of the poloidal-toroidal decomposition (Section 4),
    // n x n, T coefficients -> C^(2): r^2 (z . curl V) =
    //   PTa V_theta - i w PTb V_r,  PTa = R (C02 + R C12 D1),  PTb = R C02.
    Band PTa, PTb;
};
DirOps build_dir_ops(int n);

// Spectral bounds of Section 3 for the Poisson pencils.
struct Bounds { double a, b, c, d; };
// Enclosing [a,b] of C^-1 A_w over both parity blocks, given A_w and C.
void pencil_bounds_r(const Band& A, const Band& C, double* a, double* b);
// Enclosing [c,d] of -D B^-1 over both parity blocks, given B = C02Q^T, D = D2Q^T.
void pencil_bounds_z(const Band& B, const Band& D, double* c, double* d);

// Zolotarev shifts (Section 3): u_j in [c,d] (first half-step), v_j in [a,b].
int adi_num_iterations(double a, double b, double c, double d, double eps);
void adi_shifts(double a, double b, double c, double d, int J, double* u, double* v);
double jacobi_dn_frac(double t, double kp);   // dn(t K(k), k), 0 <= t <= 1
double ellip_K_from_kp(double kp);

// Horizontal (disk) Poisson of Section 4 (Delta_h = nabla^2 - d_zz, diagonal
// in theta and z): per z coefficient one tau system [A_w Q]_tau x = [R^2 C02 f]_tau
// in r, split by r parity.  Per (wavenumber slot, parity), per parity row i:
// lu[4] = (L_i of the unit lower factor, 1/d_i, U_(i,i+1)/d_i, U_(i,i+2)/d_i)
// of the no-pivot LU (bandwidths 1 and 2 within a parity); per parity, per
// row, taps[5] of [R^2 C02]_tau on the same-parity T coefficients i-1 .. i+3.
constexpr int kDiskRec = 4, kDiskTaps = 5;
struct DiskTables {
    int rows[2] = {0, 0}, cols[2] = {0, 0}, rmax = 0;
    std::vector<double> lu;     // [nw][2][rmax][kDiskRec]
    std::vector<double> taps;   // [2][rmax][kDiskTaps]
    // PT decomposition: per parity row, taps of PTa then of PTb on the T
    // coefficients of the other parity, indices q-1 .. q+3 within that parity
    std::vector<double> pt_taps;   // [2][rmax][2][kDiskTaps]
};
DiskTables build_disk_tables(const DirOps& ops, int nw);

constexpr int kMaxRadixPasses = 12;
// Largest prime radix computed directly (longer prime factors use Bluestein),
// and the output pairs one thread computes in such a pass.
constexpr int kMaxPrimeRadix = 257;
constexpr int kPrimeOutputs = 9;
// Per-length DFT tables (complex length L; FFT length Nb = L when L factors
// into the supported radices, else the power of two >= 2L - 1 of Bluestein).
struct DftTables {
    int L = 0, Nb = 0, tpl = 1;     // tpl: threads per line in the kernels
    int pts = 16;                   // points per thread in the kernels (8 or 16)
    bool bluestein = false;
    std::vector<int> radices;   // Stockham pass radices, first pass first
    std::vector<double> tw;     // 2*Nb: per-pass FFT twiddles (see build_dft_tables)
    std::vector<double> chirp;  // 2*L : exp(-i pi n^2 / L)
    std::vector<double> bhat;   // 2*Nb: FFT of the Bluestein filter, times 1/Nb
};
// pts: points per thread of the kernels, 8 or 16; 8 applies only to direct
// FFTs of at most 256 points not led by a prime pass (first radix above 17).
DftTables build_dft_tables(int L, bool mixed = true, int pts = 8);
// Radix plan of a length-N FFT: a prime factor 19..257 first (at most one,
// computed directly), an odd prime factor 7, 11, 13 or 17 first (at most one;
// only 7 after a prime pass), 16/8/4/2 for the power-of-two part, then 15, 5,
// 3; false for any other N.
bool dft_radix_plan(int N, std::vector<int>* radices);
// Threads per line for a length-N FFT with the given passes: at least N / pts
// (and N / R for radices R >= 11), balancing the butterflies of every pass.
int dft_threads_per_line(int N, const std::vector<int>& radices, int pts = 16);

// Record layouts of the ADI coefficient tables (doubles per row).
constexpr int kRRec = 12;   // r-pass: (vC - A) row[6], L[2], dinv, dinv*U[3]
constexpr int kZRec = 8;    // z-pass: L, dinv, dinv*U[2], (u'B + D)^T row[4]
// Split sweeps (two threads per line, see build_adi_setup): rows below the
// split row t keep the LU records above; rows from t on hold UL records
//   r-pass: (vC - A) row[6], U'[3], dinv', dinv' L'[2]   (L' at i-1, i-2)
//   z-pass: U'[2], dinv', dinv' L'(k, k-1), (u'B + D)^T row[4]
// and each parity block's records are followed by its coupling matrix
// (r: 5 x 5 in kRCouple rows, z: 3 x 3 in kZCouple rows).
constexpr int kRCouple = 3;
constexpr int kZCouple = 2;
// Split row of a line of n unknowns: a multiple of 8 near n / 2.
int adi_split_row(int n);
// True when every parity block is long enough for the split sweeps.
bool adi_split_fits(int me_min, int ne_min);

// Pencil + tolerance -> everything the ADI kernels read.
struct AdiSetup {
    double kappa_alpha = 0.0, eps = 0.0;
    int nw = 0;
    std::vector<int> J;                 // per w slot
    std::vector<double> bounds;         // 4 per w slot
    std::vector<int64_t> roff, zoff;    // per w slot: offset of its tables
    std::vector<double> rtab, ztab;     // coefficient records
    std::vector<double> vmu;            // per (w, j): v_j - u_j, offset soff[w]
    std::vector<int64_t> soff;
    bool split = false;                 // split-sweep record layout
    int rrows[2] = {0, 0}, zrows[2] = {0, 0};   // record rows per parity block and shift
    int tr[2] = {0, 0}, tz[2] = {0, 0};         // split rows (split layout only)
    int J_max = 0, J_min = 0;
    double J_mean = 0.0;
};

struct Geometry {
    int m = 0, n = 0, p = 0;    // n_r, n_z, n_theta
    int nw = 0;                 // floor(p/2) + 1 coefficient slots
    int me[2] = {0, 0};         // r parity block sizes
    int ne[2] = {0, 0};         // z parity block sizes
    int mp[2] = {0, 0};         // me rounded up to a multiple of 8 (table rows)
    int np[2] = {0, 0};         // ne rounded up to a multiple of 8
    int nplanes = 0;            // real mode planes (= p)
    std::vector<int> plane_w, plane_part;   // per real plane
    int64_t plane_elems = 0;    // (m-2)(n-2): X-layout entries per plane
    int64_t total_elems = 0;    // nplanes * plane_elems
    int64_t eplane_elems = 0;   // (mp0+mp1)(ne0+ne1): E-layout entries per plane
    int64_t etotal_elems = 0;   // nplanes * eplane_elems
};
Geometry make_geometry(int m, int n, int p);

// Build the ADI setup for pencil (A_w - kappa_alpha-scaled) and tolerance eps.
// kappa_alpha == 0: Poisson pencil (A_w, C).  Otherwise the heat pencil
// (C - ka A_w, -ka C).  flip: the transposed equation
// A^T Y B^T + C^T Y D^T = F written for Y~ = J Y J, F~ = J F J inside every
// parity block, i.e. the pencil (J A^T J, J C^T J), (J B^T J, J D^T J); its
// spectra, shifts and iteration counts are those of the untransposed pencil.
// a_scale: test only (1 otherwise): the far end a of the interval enclosing
// spec(C^-1 A) is multiplied by it, so that a_scale < 1 gives bounds that no
// longer enclose the spectrum (shifts and J chosen for the wrong interval).
// split: records for the two-thread sweeps.  A line of n unknowns is cut at
// t = adi_split_row(n): rows [0, t) are eliminated downwards (LU), rows
// [t, n) upwards (UL), the lo + hi unknowns around t follow from a small
// coupling system, and each half then substitutes outwards from t.
AdiSetup build_adi_setup(const Geometry& g, const DirOps& r, const DirOps& z,
                         double kappa_alpha, double eps, bool flip = false, bool split = false,
                         double a_scale = 1.0);

// Bounds/J/shifts of one wavenumber (shared by the setup and the host query).
void mode_parameters(const DirOps& r, const DirOps& z, int w, double kappa_alpha,
                     double eps, double zc, double zd, double* bounds4, int* J,
                     std::vector<double>* u, std::vector<double>* v, double a_scale = 1.0);

}  // namespace cyl
