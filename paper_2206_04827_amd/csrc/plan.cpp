// Host-side planning: operators (Section 3), spectral bounds and Zolotarev
// shifts (Section 3, after Algorithm 1), LU tables for the ADI kernels, and
// DFT tables for the transform kernels (Section 2).
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <exception>
#include <stdexcept>
#include <string>
#include <thread>

namespace cyl {

// ----------------------------------------------------------------------------
// banded matrices
// ----------------------------------------------------------------------------

Band::Band(int r, int c, int l, int h) : rows(r), cols(c), lo(l), hi(h),
    v(static_cast<size_t>(r) * static_cast<size_t>(l + h + 1), 0.0) {}

double Band::get(int i, int j) const {
    const int d = j - i;
    if (i < 0 || i >= rows || j < 0 || j >= cols || d < -lo || d > hi) return 0.0;
    return v[static_cast<size_t>(i) * width() + (d + lo)];
}

void Band::set(int i, int j, double x) {
    const int d = j - i;
    if (i < 0 || i >= rows || j < 0 || j >= cols || d < -lo || d > hi)
        throw std::logic_error("Band::set outside the band");
    v[static_cast<size_t>(i) * width() + (d + lo)] = x;
}

Band band_mul(const Band& A, const Band& B) {
    if (A.cols != B.rows) throw std::logic_error("band_mul: shape mismatch");
    Band C(A.rows, B.cols, A.lo + B.lo, A.hi + B.hi);
    for (int i = 0; i < C.rows; ++i) {
        for (int d = -C.lo; d <= C.hi; ++d) {
            const int j = i + d;
            if (j < 0 || j >= C.cols) continue;
            const int k0 = std::max({0, i - A.lo, j - B.hi});
            const int k1 = std::min({A.cols - 1, i + A.hi, j + B.lo});
            double s = 0.0;
            for (int k = k0; k <= k1; ++k) s += A.get(i, k) * B.get(k, j);
            C.set(i, j, s);
        }
    }
    return C;
}

Band band_axpby(double alpha, const Band& A, double beta, const Band& B) {
    if (A.rows != B.rows || A.cols != B.cols) throw std::logic_error("band_axpby: shape mismatch");
    Band C(A.rows, A.cols, std::max(A.lo, B.lo), std::max(A.hi, B.hi));
    for (int i = 0; i < C.rows; ++i)
        for (int d = -C.lo; d <= C.hi; ++d) {
            const int j = i + d;
            if (j < 0 || j >= C.cols) continue;
            C.set(i, j, alpha * A.get(i, j) + beta * B.get(i, j));
        }
    return C;
}

Band band_cut(const Band& A, int rows, int cols) {
    Band C(rows, cols, A.lo, A.hi);
    for (int i = 0; i < rows; ++i)
        for (int d = -A.lo; d <= A.hi; ++d) {
            const int j = i + d;
            if (j < 0 || j >= cols) continue;
            C.set(i, j, A.get(i, j));
        }
    return C;
}

Band band_transpose(const Band& A) {
    Band T(A.cols, A.rows, A.hi, A.lo);
    for (int i = 0; i < A.rows; ++i)
        for (int d = -A.lo; d <= A.hi; ++d) {
            const int j = i + d;
            if (j < 0 || j >= A.cols) continue;
            T.set(j, i, A.get(i, j));
        }
    return T;
}

Band band_flip_transpose(const Band& A) {
    if (A.rows != A.cols) throw std::logic_error("band_flip_transpose: matrix is not square");
    const int N = A.rows;
    Band F(N, N, A.lo, A.hi);
    for (int i = 0; i < N; ++i)
        for (int d = -A.lo; d <= A.hi; ++d) {
            const int j = i + d;
            if (j < 0 || j >= N) continue;
            F.set(i, j, A.get(N - 1 - j, N - 1 - i));
        }
    return F;
}

Band band_parity(const Band& A, int p) {
    for (int i = 0; i < A.rows; ++i)
        for (int d = -A.lo; d <= A.hi; ++d) {
            if ((d & 1) == 0) continue;
            if (A.get(i, i + d) != 0.0) throw std::logic_error("operator couples index parities");
        }
    Band P((A.rows - p + 1) / 2, (A.cols - p + 1) / 2, A.lo / 2, A.hi / 2);
    for (int i = 0; i < P.rows; ++i)
        for (int d = -P.lo; d <= P.hi; ++d) {
            const int j = i + d;
            if (j < 0 || j >= P.cols) continue;
            P.set(i, j, A.get(2 * i + p, 2 * j + p));
        }
    return P;
}

// ----------------------------------------------------------------------------
// operators of Section 3 (built 6 larger, then cut: rows < n-2 are exact)
// ----------------------------------------------------------------------------

namespace {

constexpr int kPad = 6;

Band op_T_to_U(int N) {          // C_01: T_0 = U_0, T_k = (U_k - U_{k-2}) / 2
    Band M(N, N, 0, 2);
    M.set(0, 0, 1.0);
    for (int k = 1; k < N; ++k) M.set(k, k, 0.5);
    for (int k = 2; k < N; ++k) M.set(k - 2, k, -0.5);
    return M;
}
Band op_U_to_C2(int N) {         // C_12: U_k = (C2_k - C2_{k-2}) / (k + 1)
    Band M(N, N, 0, 2);
    for (int i = 0; i < N; ++i) M.set(i, i, 1.0 / (i + 1));
    for (int i = 0; i + 2 < N; ++i) M.set(i, i + 2, -1.0 / (i + 3));
    return M;
}
Band op_mul_r(int N) {           // R: x C2_k = ((k+1) C2_{k+1} + (k+3) C2_{k-1}) / (2(k+2))
    Band M(N, N, 1, 1);
    for (int i = 0; i + 1 < N; ++i) M.set(i, i + 1, (i + 4.0) / (2.0 * (i + 3)));
    for (int i = 1; i < N; ++i) M.set(i, i - 1, i / (2.0 * (i + 1)));
    return M;
}
Band op_d1(int N) {              // D_1: T_k' = k U_{k-1}
    Band M(N, N, 0, 1);
    for (int i = 0; i + 1 < N; ++i) M.set(i, i + 1, i + 1.0);
    return M;
}
Band op_d2(int N) {              // D_2: T_k'' = 2k C2_{k-2}
    Band M(N, N, 0, 2);
    for (int i = 0; i + 2 < N; ++i) M.set(i, i + 2, 2.0 * (i + 2));
    return M;
}
Band op_dirichlet(int N, int n) { // Q: phi_j = T_{j+2} - T_j
    Band Q(N, n - 2, 2, 0);
    for (int j = 0; j < n - 2; ++j) {
        Q.set(j, j, -1.0);
        Q.set(j + 2, j, 1.0);
    }
    return Q;
}

}  // namespace

DirOps build_dir_ops(int n) {
    const int N = n + kPad;
    DirOps o;
    o.n = n;
    const Band S0 = op_T_to_U(N), S1 = op_U_to_C2(N), R = op_mul_r(N);
    const Band D1 = op_d1(N), D2 = op_d2(N), Q = op_dirichlet(N, n);
    const Band S10 = band_mul(S1, S0);
    const Band RR = band_mul(R, R);
    const Band Rad0 = band_axpby(1.0, band_mul(band_mul(R, S1), D1), 1.0, band_mul(RR, D2));
    o.A0 = band_cut(band_mul(Rad0, Q), n - 2, n - 2);
    o.Cc = band_cut(band_mul(S10, Q), n - 2, n - 2);
    o.R2Q = band_cut(band_mul(band_mul(RR, S10), Q), n - 2, n - 2);
    o.C02Q = o.Cc;
    o.D2Q = band_cut(band_mul(D2, Q), n - 2, n - 2);
    o.R2f = band_cut(band_mul(RR, S10), n, n);
    o.C02f = band_cut(S10, n, n);
    o.A0f = band_cut(Rad0, n, n);
    o.S10f = o.C02f;
    o.D2f = band_cut(D2, n, n);
    o.PTa = band_cut(band_mul(R, band_axpby(1.0, S10, 1.0, band_mul(R, band_mul(S1, D1)))), n, n);
    o.PTb = band_cut(band_mul(R, S10), n, n);
    return o;
}

// ----------------------------------------------------------------------------
// host banded LU with partial pivoting (for the eigenvalue iterations only)
// ----------------------------------------------------------------------------

namespace {

struct HostLU {
    int n = 0, lo = 0, hi = 0;   // U has bandwidth hi + lo after pivoting
    std::vector<double> a;       // dense-band rows of width lo + (hi + lo) + 1
    std::vector<int> piv;
    int w() const { return 2 * lo + hi + 1; }
    double& at(int i, int j) { return a[static_cast<size_t>(i) * w() + (j - i + lo)]; }

    explicit HostLU(const Band& M) : n(M.rows), lo(M.lo), hi(M.hi),
        a(static_cast<size_t>(M.rows) * (2 * M.lo + M.hi + 1), 0.0), piv(M.rows) {
        for (int i = 0; i < n; ++i)
            for (int j = std::max(0, i - lo); j <= std::min(n - 1, i + hi); ++j) at(i, j) = M.get(i, j);
        const int uh = hi + lo;
        for (int k = 0; k < n; ++k) {
            int p = k;
            double best = std::fabs(at(k, k));
            for (int i = k + 1; i <= std::min(n - 1, k + lo); ++i)
                if (std::fabs(at(i, k)) > best) { best = std::fabs(at(i, k)); p = i; }
            piv[k] = p;
            if (best == 0.0) throw std::runtime_error("singular pencil in bound estimation");
            if (p != k)
                for (int j = k; j <= std::min(n - 1, k + uh); ++j) std::swap(at(k, j), at(p, j));
            const double inv = 1.0 / at(k, k);
            for (int i = k + 1; i <= std::min(n - 1, k + lo); ++i) {
                const double l = at(i, k) * inv;
                at(i, k) = l;
                if (l == 0.0) continue;
                for (int j = k + 1; j <= std::min(n - 1, k + uh); ++j) at(i, j) -= l * at(k, j);
            }
        }
    }
    void solve(std::vector<double>& x) {
        const int uh = hi + lo;
        for (int k = 0; k < n; ++k) {
            if (piv[k] != k) std::swap(x[k], x[piv[k]]);
            for (int i = k + 1; i <= std::min(n - 1, k + lo); ++i) x[i] -= at(i, k) * x[k];
        }
        for (int k = n - 1; k >= 0; --k) {
            double s = x[k];
            for (int j = k + 1; j <= std::min(n - 1, k + uh); ++j) s -= at(k, j) * x[j];
            x[k] = s / at(k, k);
        }
    }
};

void band_apply(const Band& M, const std::vector<double>& x, std::vector<double>& y) {
    y.assign(M.rows, 0.0);
    for (int i = 0; i < M.rows; ++i) {
        double s = 0.0;
        for (int j = std::max(0, i - M.lo); j <= std::min(M.cols - 1, i + M.hi); ++j) s += M.get(i, j) * x[j];
        y[i] = s;
    }
}

// Extreme eigenvalue of solve(Den, Num x) by power iteration (Rayleigh estimate).
double power_estimate(const Band& Num, const Band& Den, int iters) {
    const int n = Num.rows;
    HostLU lu(Den);
    std::vector<double> x(n), y;
    for (int i = 0; i < n; ++i) x[i] = std::sin(1.37 * i + 0.71) + 0.05;
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        double nx = 0.0;
        for (double t : x) nx += t * t;
        nx = std::sqrt(nx);
        for (double& t : x) t /= nx;
        band_apply(Num, x, y);
        lu.solve(y);
        double xy = 0.0;
        for (int i = 0; i < n; ++i) xy += x[i] * y[i];
        lam = xy;
        x.swap(y);
    }
    return lam;
}

}  // namespace

void pencil_bounds_r(const Band& A, const Band& C, double* a, double* b) {
    double amin = 0.0, bmax = -1e300;
    for (int par = 0; par < 2; ++par) {
        const Band Ap = band_parity(A, par), Cp = band_parity(C, par);
        if (Ap.rows == 0) continue;
        const double top = power_estimate(Ap, Cp, 300);          // most negative
        const double mu = power_estimate(Cp, Ap, 60);            // 1 / (closest to zero)
        amin = std::min(amin, top);
        bmax = std::max(bmax, 1.0 / mu);
    }
    // widen to enclose: a further from zero, b closer to zero
    *a = 1.02 * amin;
    *b = 0.98 * bmax;
}

void pencil_bounds_z(const Band& B, const Band& D, double* c, double* d) {
    // spectrum of -D B^-1 equals that of the pencil (-D^T, B^T)
    const Band Bt = band_transpose(B), mDt = band_axpby(-1.0, band_transpose(D), 0.0, band_transpose(D));
    double cmin = 1e300, dmax = 0.0;
    for (int par = 0; par < 2; ++par) {
        const Band Np = band_parity(mDt, par), Dp = band_parity(Bt, par);
        if (Np.rows == 0) continue;
        const double top = power_estimate(Np, Dp, 300);
        const double mu = power_estimate(Dp, Np, 60);
        dmax = std::max(dmax, top);
        cmin = std::min(cmin, 1.0 / mu);
    }
    *c = 0.98 * cmin;
    *d = 1.02 * dmax;
}

// ----------------------------------------------------------------------------
// elliptic functions and Zolotarev shifts
// ----------------------------------------------------------------------------

namespace {

// Arithmetic-geometric mean AGM(1, b0) together with the c_n sequence.
int agm(double b0, double* a, double* c, int cap) {
    a[0] = 1.0;
    double b = b0;
    c[0] = std::sqrt((1.0 - b0) * (1.0 + b0));
    int N = 0;
    while (N + 1 < cap && std::fabs(c[N]) > std::ldexp(a[N], -60)) {
        const double an = a[N];
        a[N + 1] = 0.5 * (an + b);
        c[N + 1] = 0.5 * (an - b);
        b = std::sqrt(an * b);
        ++N;
    }
    return N;
}

// dn by the descending AGM recursion on the amplitude (moderate k').
double dn_descending(double u, double kp) {
    double a[64], c[64];
    const int N = agm(kp, a, c, 64);
    if (N == 0) return 1.0;
    double phi[65];
    phi[N] = std::ldexp(a[N] * u, N);
    for (int k = N; k >= 1; --k) phi[k - 1] = 0.5 * (phi[k] + std::asin(c[k] * std::sin(phi[k]) / a[k]));
    return std::cos(phi[0]) / std::cos(phi[1] - phi[0]);
}

// dn from theta functions of the complementary nome q' = exp(-pi K / K')
// (Jacobi's imaginary transformation); positive series, no cancellation.
double dn_theta(double u, double kp) {
    const double k = std::sqrt((1.0 - kp) * (1.0 + kp));
    const double K = ellip_K_from_kp(kp);
    const double Kc = ellip_K_from_kp(k);
    const double lnq = -M_PI * K / Kc;
    const double y = M_PI * u / (2.0 * Kc);
    auto ch = [](double e, double x) { return 0.5 * (std::exp(e + x) + std::exp(e - x)); };
    double t3 = 1.0;
    for (int n = 1; n <= 60; ++n) {
        const double term = 2.0 * ch(n * n * lnq, 2.0 * n * y);
        t3 += term;
        if (term < 1e-18 * t3) break;
    }
    double t2 = 0.0;
    for (int n = 0; n <= 60; ++n) {
        const double h = n + 0.5;
        const double term = 2.0 * ch(h * h * lnq, (2 * n + 1) * y);
        t2 += term;
        if (n > 0 && term < 1e-18 * t2) break;
    }
    return std::sqrt(kp) * t3 / t2;
}

double dn_plain(double u, double kp) { return kp >= 0.5 ? dn_descending(u, kp) : dn_theta(u, kp); }

}  // namespace

double ellip_K_from_kp(double kp) {
    double a[64], c[64];
    const int N = agm(kp, a, c, 64);
    return M_PI / (2.0 * a[N]);
}

double jacobi_dn_frac(double t, double kp) {
    const double K = ellip_K_from_kp(kp);
    if (t <= 0.5) return dn_plain(t * K, kp);
    return kp / dn_plain((1.0 - t) * K, kp);      // dn(K - x) = k' / dn(x)
}

int adi_num_iterations(double a, double b, double c, double d, double eps) {
    const double gamma = std::fabs(c - a) * std::fabs(d - b) / (std::fabs(c - b) * std::fabs(d - a));
    const double J = std::ceil(std::log(16.0 * gamma) * std::log(4.0 / eps) / (M_PI * M_PI));
    return std::max(1, static_cast<int>(J));
}

void adi_shifts(double a, double b, double c, double d, int J, double* u, double* v) {
    const double gamma = std::fabs(c - a) * std::fabs(d - b) / (std::fabs(c - b) * std::fabs(d - a));
    const double az = -1.0 + 2.0 * gamma + 2.0 * std::sqrt(gamma * (gamma - 1.0));
    const double kp = 1.0 / az;
    // Moebius map (-az, -1, 1, az) -> (a, b, c, d) through the cross-ratio.
    auto T = [&](double z) {
        const double rho = (z + az) * (-2.0) / ((z - 1.0) * (az - 1.0));
        const double s = rho * (b - a) / (b - c);
        return (a - s * c) / (1.0 - s);
    };
    for (int j = 0; j < J; ++j) {
        const double dn = jacobi_dn_frac((2.0 * j + 1.0) / (2.0 * J), kp);
        u[j] = T(az * dn);
        v[j] = T(-az * dn);
    }
}

// ----------------------------------------------------------------------------
// geometry, per-mode parameters and ADI tables
// ----------------------------------------------------------------------------

Geometry make_geometry(int m, int n, int p) {
    Geometry g;
    g.m = m; g.n = n; g.p = p;
    g.nw = p / 2 + 1;
    g.me[0] = (m - 1) / 2; g.me[1] = (m - 2) / 2;    // ceil((m-2)/2), floor((m-2)/2)
    g.ne[0] = (n - 1) / 2; g.ne[1] = (n - 2) / 2;
    for (int par = 0; par < 2; ++par) {
        g.mp[par] = (g.me[par] + 7) / 8 * 8;
        g.np[par] = (g.ne[par] + 7) / 8 * 8;
    }
    for (int w = 0; w < g.nw; ++w) {
        g.plane_w.push_back(w); g.plane_part.push_back(0);
        const bool real_only = (w == 0) || (p % 2 == 0 && w == p / 2);
        if (!real_only) { g.plane_w.push_back(w); g.plane_part.push_back(1); }
    }
    g.nplanes = static_cast<int>(g.plane_w.size());
    g.plane_elems = static_cast<int64_t>(m - 2) * (n - 2);
    g.total_elems = g.plane_elems * g.nplanes;
    g.eplane_elems = static_cast<int64_t>(g.mp[0] + g.mp[1]) * (g.ne[0] + g.ne[1]);
    g.etotal_elems = g.eplane_elems * g.nplanes;
    return g;
}

namespace {

Band radial_A(const DirOps& r, int w) {
    return band_axpby(1.0, r.A0, -static_cast<double>(w) * w, r.Cc);
}

// No-pivot banded LU of M (rows of the parity block): fills L (lo entries),
// inverse pivots and dinv-scaled U (hi entries).
void nopivot_lu(const Band& M, std::vector<double>& L, std::vector<double>& dinv,
                std::vector<double>& Us) {
    const int n = M.rows, lo = M.lo, hi = M.hi;
    std::vector<double> a(static_cast<size_t>(n) * (lo + hi + 1));
    auto at = [&](int i, int j) -> double& { return a[static_cast<size_t>(i) * (lo + hi + 1) + (j - i + lo)]; };
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - lo); j <= std::min(n - 1, i + hi); ++j) at(i, j) = M.get(i, j);
    L.assign(static_cast<size_t>(n) * lo, 0.0);
    dinv.assign(n, 0.0);
    Us.assign(static_cast<size_t>(n) * hi, 0.0);
    for (int k = 0; k < n; ++k) {
        const double piv = at(k, k);
        if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv)) throw std::runtime_error("zero pivot in ADI factorisation");
        for (int i = k + 1; i <= std::min(n - 1, k + lo); ++i) {
            const double l = at(i, k) / piv;
            at(i, k) = l;
            for (int j = k + 1; j <= std::min(n - 1, k + hi); ++j) at(i, j) -= l * at(k, j);
        }
    }
    for (int i = 0; i < n; ++i) {
        for (int t = 1; t <= lo; ++t) if (i - t >= 0) L[static_cast<size_t>(i) * lo + (lo - t)] = at(i, i - t);
        dinv[i] = 1.0 / at(i, i);
        for (int t = 1; t <= hi; ++t) if (i + t < n) Us[static_cast<size_t>(i) * hi + (t - 1)] = dinv[i] * at(i, i + t);
    }
}

// No-pivot UL of M (eliminating the upper band from the last row up):
// M = U' L' with U' unit upper (hi multipliers per row) and L' lower.  Per row:
// Up = U'(i, i+t) for t = 1..hi, dinv = 1 / L'(i, i), Ls = dinv L'(i, i-t) for t = 1..lo.
void nopivot_ul(const Band& M, std::vector<double>& Up, std::vector<double>& dinv,
                std::vector<double>& Ls) {
    const int n = M.rows, lo = M.lo, hi = M.hi;
    std::vector<double> a(static_cast<size_t>(n) * (lo + hi + 1));
    auto at = [&](int i, int j) -> double& { return a[static_cast<size_t>(i) * (lo + hi + 1) + (j - i + lo)]; };
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - lo); j <= std::min(n - 1, i + hi); ++j) at(i, j) = M.get(i, j);
    for (int k = n - 1; k >= 0; --k) {
        const double piv = at(k, k);
        if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv)) throw std::runtime_error("zero pivot in ADI factorisation");
        for (int i = k - 1; i >= std::max(0, k - hi); --i) {
            const double f = at(i, k) / piv;
            at(i, k) = f;
            for (int j = std::max(0, k - lo); j < k; ++j) at(i, j) -= f * at(k, j);
        }
    }
    Up.assign(static_cast<size_t>(n) * hi, 0.0);
    dinv.assign(n, 0.0);
    Ls.assign(static_cast<size_t>(n) * lo, 0.0);
    for (int i = 0; i < n; ++i) {
        for (int t = 1; t <= hi; ++t) if (i + t < n) Up[static_cast<size_t>(i) * hi + (t - 1)] = at(i, i + t);
        dinv[i] = 1.0 / at(i, i);
        for (int t = 1; t <= lo; ++t) if (i - t >= 0) Ls[static_cast<size_t>(i) * lo + (t - 1)] = dinv[i] * at(i, i - t);
    }
}

// Coupling of the split sweeps for a line of bandwidths (lo, hi) cut at t:
// the unknowns x_{t-lo} .. x_{t+hi-1} satisfy the normalised last lo rows of
// the LU part and first hi rows of the UL part,
//   x_i + sum_s dinv_i U_{i,i+s} x_{i+s} = dinv_i g_i        (t-lo <= i < t)
//   x_i + sum_s dinv'_i L'_{i,i-s} x_{i-s} = dinv'_i g'_i    (t <= i < t+hi),
// so x = K (g_{t-lo}, .., g_{t-1}, g'_t, .., g'_{t+hi-1}) with
// K = C^-1 diag(dinv, dinv').  K is written row-major (K x K doubles).
void split_coupling(int lo, int hi, int t, const std::vector<double>& Us, const std::vector<double>& dinv,
                    const std::vector<double>& Ls, const std::vector<double>& dinvp, double* out) {
    const int K = lo + hi, x0 = t - lo;
    std::vector<long double> C(static_cast<size_t>(K) * K, 0.0L), inv(static_cast<size_t>(K) * K, 0.0L);
    std::vector<long double> d(K);
    for (int r = 0; r < K; ++r) {
        const int i = x0 + r;
        C[r * K + r] = 1.0L;
        if (i < t) {
            for (int s = 1; s <= hi; ++s) C[r * K + (r + s)] = Us[static_cast<size_t>(i) * hi + (s - 1)];
            d[r] = dinv[i];
        } else {
            for (int s = 1; s <= lo; ++s) C[r * K + (r - s)] = Ls[static_cast<size_t>(i) * lo + (s - 1)];
            d[r] = dinvp[i];
        }
        inv[r * K + r] = 1.0L;
    }
    for (int c = 0; c < K; ++c) {                 // Gauss-Jordan, partial pivoting
        int p = c;
        for (int r = c + 1; r < K; ++r) if (std::fabs(C[r * K + c]) > std::fabs(C[p * K + c])) p = r;
        if (!(std::fabs(C[p * K + c]) > 0.0L)) throw std::runtime_error("singular split coupling");
        if (p != c)
            for (int q = 0; q < K; ++q) { std::swap(C[p * K + q], C[c * K + q]); std::swap(inv[p * K + q], inv[c * K + q]); }
        const long double piv = C[c * K + c];
        for (int q = 0; q < K; ++q) { C[c * K + q] /= piv; inv[c * K + q] /= piv; }
        for (int r = 0; r < K; ++r) {
            if (r == c) continue;
            const long double f = C[r * K + c];
            if (f == 0.0L) continue;
            for (int q = 0; q < K; ++q) { C[r * K + q] -= f * C[c * K + q]; inv[r * K + q] -= f * inv[c * K + q]; }
        }
    }
    for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) out[r * K + c] = static_cast<double>(inv[r * K + c] * d[c]);
}

}  // namespace

// Run f(i) for i in [0, n) on up to 16 host threads; the first exception
// thrown by any f(i) is rethrown in the caller.
template <typename F>
void parallel_for(int n, F&& f) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = std::min(n, static_cast<int>(std::min(hw, 16u)));
    if (T <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::exception_ptr> errs(T);
    std::vector<std::thread> pool;
    pool.reserve(T);
    for (int t = 0; t < T; ++t)
        pool.emplace_back([&, t] {
            try {
                for (int i = next++; i < n; i = next++) f(i);
            } catch (...) {
                errs[t] = std::current_exception();
                next = n;
            }
        });
    for (auto& th : pool) th.join();
    for (auto& e : errs)
        if (e) std::rethrow_exception(e);
}

int adi_split_row(int n) { return std::max(8, (n / 2 + 4) / 8 * 8); }

bool adi_split_fits(int me_min, int ne_min) {
    return me_min - adi_split_row(me_min) >= 3 && ne_min - adi_split_row(ne_min) >= 2 &&
           adi_split_row(me_min) >= 8 && adi_split_row(ne_min) >= 8;
}

void mode_parameters(const DirOps& r, const DirOps& z, int w, double ka, double eps,
                     double zc, double zd, double* bounds4, int* J,
                     std::vector<double>* u, std::vector<double>* v, double a_scale) {
    double a, b;
    pencil_bounds_r(radial_A(r, w), r.R2Q, &a, &b);
    if (ka > 0.0) { a -= 1.0 / ka; b -= 1.0 / ka; }
    if (a_scale != 1.0) a = std::min(a * a_scale, 1.5 * b);   // test only: no longer encloses
    bounds4[0] = a; bounds4[1] = b; bounds4[2] = zc; bounds4[3] = zd;
    *J = adi_num_iterations(a, b, zc, zd, eps);
    if (u && v) {
        u->assign(*J, 0.0); v->assign(*J, 0.0);
        adi_shifts(a, b, zc, zd, *J, u->data(), v->data());
    }
}

AdiSetup build_adi_setup(const Geometry& g, const DirOps& r, const DirOps& z, double ka, double eps,
                         bool flip, bool split, double a_scale) {
    AdiSetup s;
    s.kappa_alpha = ka; s.eps = eps; s.nw = g.nw;
    s.split = split;
    for (int par = 0; par < 2; ++par) {
        s.rrows[par] = g.mp[par] + (split ? kRCouple : 0);
        s.zrows[par] = g.np[par] + (split ? kZCouple : 0);
        s.tr[par] = split ? adi_split_row(g.me[par]) : 0;
        s.tz[par] = split ? adi_split_row(g.ne[par]) : 0;
    }
    if (split && !adi_split_fits(std::min(g.me[0], g.me[1]), std::min(g.ne[0], g.ne[1])))
        throw std::logic_error("parity blocks too small for the split sweeps");
    double zc, zd;
    pencil_bounds_z(band_transpose(z.C02Q), band_transpose(z.D2Q), &zc, &zd);

    const Band Bt = band_transpose(z.C02Q), Dt = band_transpose(z.D2Q);
    Band Bp[2], Dp[2];
    for (int par = 0; par < 2; ++par) {
        Bp[par] = band_parity(Bt, par); Dp[par] = band_parity(Dt, par);
        if (flip) { Bp[par] = band_flip_transpose(Bp[par]); Dp[par] = band_flip_transpose(Dp[par]); }
    }
    // records per shift: both parity blocks, rows padded to a multiple of 8
    // (plus the coupling rows of the split layout)
    const int me_sum = s.rrows[0] + s.rrows[1], ne_sum = s.zrows[0] + s.zrows[1];

    s.J.resize(g.nw); s.bounds.resize(4 * g.nw);
    s.roff.resize(g.nw); s.zoff.resize(g.nw); s.soff.resize(g.nw);
    int64_t rsz = 0, zsz = 0, ssz = 0;
    std::vector<std::vector<double>> U(g.nw), V(g.nw);
    parallel_for(g.nw, [&](int w) {
        mode_parameters(r, z, w, ka, eps, zc, zd, &s.bounds[4 * w], &s.J[w], &U[w], &V[w], a_scale);
    });
    for (int w = 0; w < g.nw; ++w) {
        s.roff[w] = rsz; s.zoff[w] = zsz; s.soff[w] = ssz;
        rsz += static_cast<int64_t>(s.J[w]) * me_sum * kRRec;
        zsz += static_cast<int64_t>(s.J[w]) * ne_sum * kZRec;
        ssz += s.J[w];
    }
    s.rtab.assign(rsz, 0.0); s.ztab.assign(zsz, 0.0); s.vmu.assign(ssz, 0.0);

    parallel_for(g.nw, [&](int w) {
        std::vector<double> L, dinv, Us, Up, dinvp, Ls;
        const Band Aw = radial_A(r, w);
        // pencil (A, C): Poisson (A_w, C~); heat (C~ - ka A_w, -ka C~)
        const Band A = ka > 0.0 ? band_axpby(1.0, r.R2Q, -ka, Aw) : Aw;
        const Band C = ka > 0.0 ? band_axpby(-ka, r.R2Q, 0.0, r.R2Q) : r.R2Q;
        Band Ap[2], Cp[2];
        for (int par = 0; par < 2; ++par) {
            Ap[par] = band_parity(A, par); Cp[par] = band_parity(C, par);
            if (flip) { Ap[par] = band_flip_transpose(Ap[par]); Cp[par] = band_flip_transpose(Cp[par]); }
        }
        const int J = s.J[w];
        for (int j = 0; j < J; ++j) {
            const double uj = U[w][j], vj = V[w][j];
            const double un = (j + 1 < J) ? U[w][j + 1] : 0.0;
            s.vmu[s.soff[w] + j] = vj - uj;
            // r-direction records
            int64_t base = s.roff[w] + static_cast<int64_t>(j) * me_sum * kRRec;
            for (int par = 0; par < 2; ++par) {
                const Band Mu = band_axpby(uj, Cp[par], -1.0, Ap[par]);
                const Band Mv = band_axpby(vj, Cp[par], -1.0, Ap[par]);
                if (Mu.lo != 2 || Mu.hi != 3) throw std::logic_error("unexpected r-band widths");
                nopivot_lu(Mu, L, dinv, Us);
                const int t_split = split ? s.tr[par] : Mu.rows;
                if (split) nopivot_ul(Mu, Up, dinvp, Ls);
                for (int i = 0; i < Mu.rows; ++i) {
                    double* rec = &s.rtab[base + static_cast<int64_t>(i) * kRRec];
                    for (int t = 0; t < 6; ++t) rec[t] = Mv.get(i, i - 2 + t);
                    if (i < t_split) {
                        rec[6] = L[2 * i + 0];   // multiplier of g_{i-2}
                        rec[7] = L[2 * i + 1];   // multiplier of g_{i-1}
                        rec[8] = dinv[i];
                        rec[9] = Us[3 * i + 0]; rec[10] = Us[3 * i + 1]; rec[11] = Us[3 * i + 2];
                    } else {
                        rec[6] = Up[3 * i + 0];  // multiplier of g'_{i+1}
                        rec[7] = Up[3 * i + 1];  // multiplier of g'_{i+2}
                        rec[8] = Up[3 * i + 2];  // multiplier of g'_{i+3}
                        rec[9] = dinvp[i];
                        rec[10] = Ls[2 * i + 0]; rec[11] = Ls[2 * i + 1];   // x_{i-1}, x_{i-2}
                    }
                }
                if (split)
                    split_coupling(2, 3, t_split, Us, dinv, Ls, dinvp,
                                   &s.rtab[base + static_cast<int64_t>(g.mp[par]) * kRRec]);
                base += static_cast<int64_t>(s.rrows[par]) * kRRec;
            }
            // z-direction records: solve x (v B + D) = z, then w = x (u' B + D)
            base = s.zoff[w] + static_cast<int64_t>(j) * ne_sum * kZRec;
            for (int par = 0; par < 2; ++par) {
                const Band M = band_axpby(vj, Bp[par], 1.0, Dp[par]);
                const Band N = band_transpose(M);
                const Band Mn = band_axpby(un, Bp[par], 1.0, Dp[par]);
                if (N.lo != 1 || N.hi != 2) throw std::logic_error("unexpected z-band widths");
                nopivot_lu(N, L, dinv, Us);
                const int t_split = split ? s.tz[par] : N.rows;
                if (split) nopivot_ul(N, Up, dinvp, Ls);
                for (int k = 0; k < N.rows; ++k) {
                    double* rec = &s.ztab[base + static_cast<int64_t>(k) * kZRec];
                    if (k < t_split) {
                        rec[0] = L[k];
                        rec[1] = dinv[k];
                        rec[2] = Us[2 * k + 0]; rec[3] = Us[2 * k + 1];
                    } else {
                        rec[0] = Up[2 * k + 0]; rec[1] = Up[2 * k + 1];   // g'_{k+1}, g'_{k+2}
                        rec[2] = dinvp[k];
                        rec[3] = Ls[k];                                    // x_{k-1}
                    }
                    if (j + 1 < J)
                        for (int t = 0; t < 4; ++t) rec[4 + t] = Mn.get(k - 1 + t, k);
                }
                if (split)
                    split_coupling(1, 2, t_split, Us, dinv, Ls, dinvp,
                                   &s.ztab[base + static_cast<int64_t>(g.np[par]) * kZRec]);
                base += static_cast<int64_t>(s.zrows[par]) * kZRec;
            }
        }
    });
    s.J_max = *std::max_element(s.J.begin(), s.J.end());
    s.J_min = *std::min_element(s.J.begin(), s.J.end());
    double sum = 0.0;
    for (int pl = 0; pl < g.nplanes; ++pl) sum += s.J[g.plane_w[pl]];
    s.J_mean = sum / g.nplanes;
    return s;
}

// ----------------------------------------------------------------------------
// DFT tables (Bluestein when the length is not a power of two)
// ----------------------------------------------------------------------------

namespace {

using cld = std::complex<long double>;

void host_fft(std::vector<cld>& x) {      // forward, sign -1, length power of two
    const size_t N = x.size();
    for (size_t i = 1, j = 0; i < N; ++i) {
        size_t bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    for (size_t len = 2; len <= N; len <<= 1) {
        for (size_t i = 0; i < N; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const long double ang = -2.0L * pi * static_cast<long double>(k) / static_cast<long double>(len);
                const cld wk(std::cos(ang), std::sin(ang));
                const cld a = x[i + k], b = x[i + k + len / 2] * wk;
                x[i + k] = a + b;
                x[i + k + len / 2] = a - b;
            }
    }
}

}  // namespace

bool dft_radix_plan(int N, std::vector<int>* radices) {
    radices->clear();
    if (N < 1) return false;
    int n = N, p2 = 1;
    while (n % 2 == 0) { n /= 2; p2 *= 2; }
    int big = 0, nbig = 0;                 // the odd prime factor 7, 11, 13 or 17
    for (int q : {17, 13, 11, 7})
        while (n % q == 0) { n /= q; big = q; ++nbig; }
    int c3 = 0, c5 = 0;
    while (n % 3 == 0) { n /= 3; ++c3; }
    while (n % 5 == 0) { n /= 5; ++c5; }
    // one prime factor above 17 (at most kMaxPrimeRadix) is computed directly,
    // as the first pass, by all threads of a line together (prime_pass)
    int prime = 0;
    if (n > 17 && n <= kMaxPrimeRadix) {
        bool isp = true;
        for (int d = 2; d * d <= n; ++d)
            if (n % d == 0) { isp = false; break; }
        if (isp) { prime = n; n = 1; }
    }
    // the kernels run a factor 7, 11, 13 or 17 only as the first pass (no
    // twiddles), or 7 as the second pass after a prime pass
    if (n != 1 || nbig > 1 || (prime && big && big != 7)) return false;
    if (prime) radices->push_back(prime);
    if (big) radices->push_back(big);
    for (int Ls = 1; Ls < p2;) {
        const int rem = p2 / Ls;
        const int R = rem >= 16 ? 16 : rem;
        radices->push_back(R);
        Ls *= R;
    }
    for (; c3 > 0 && c5 > 0; --c3, --c5) radices->push_back(15);
    for (; c5 > 0; --c5) radices->push_back(5);
    for (; c3 > 0; --c3) radices->push_back(3);
    return static_cast<int>(radices->size()) <= kMaxRadixPasses;
}

int dft_threads_per_line(int N, const std::vector<int>& radices, int pts) {
    int lo = std::max(1, (N + pts - 1) / pts);
    for (int R : radices) {
        if (R > 17) {                               // prime pass: one work item per thread
            const int ng = (R / 2 + kPrimeOutputs - 1) / kPrimeOutputs;
            lo = std::max(lo, (N / R) * (ng + 1));
        } else if (R >= 11) {
            lo = std::max(lo, N / R);               // one butterfly per thread
        }
    }
    int best = lo;
    long long best_cost = -1;
    for (int T = lo; T <= std::max(lo, std::min(N, 2 * lo)); ++T) {
        long long c = 0;
        for (int R : radices) c += R > 17 ? 0 : static_cast<long long>((N / R + T - 1) / T) * R;
        c *= T;
        if (best_cost < 0 || c < best_cost) { best_cost = c; best = T; }
    }
    return best;
}

DftTables build_dft_tables(int L, bool mixed, int pts) {
    DftTables t;
    t.L = L;
    const long double pi = 3.141592653589793238462643383279502884L;
    const bool pow2 = (L & (L - 1)) == 0;
    std::vector<int> rad;
    t.bluestein = !(pow2 || (mixed && dft_radix_plan(L, &rad)));
    int Nb = 1;
    if (!t.bluestein) Nb = L;
    else while (Nb < 2 * L - 1) Nb <<= 1;
    t.Nb = Nb;
    if (!dft_radix_plan(Nb, &t.radices)) throw std::runtime_error("DFT radix plan");
    // 8 points per thread (twice the threads of 16, a third fewer registers
    // with the prime pass in its own instance) for direct FFTs up to 256
    // points without a prime pass; longer lines and Bluestein measured as fast
    // or faster with 16
    t.pts = (pts == 8 && !t.bluestein && Nb <= 256 && !(t.radices.size() > 0 && t.radices[0] > 17)) ? 8 : 16;
    t.tpl = dft_threads_per_line(Nb, t.radices, t.pts);
    // Per-pass twiddles of the Stockham FFT, in pass order: for the pass of
    // radix R on sub-transforms of length Ls, entries
    // [k (R-1) + q - 1] = exp(-2 pi i k q / (R Ls)), k < Ls, 1 <= q < R
    // (Nb - 1 entries in total; the table is padded to Nb).
    t.tw.assign(2 * static_cast<size_t>(Nb), 0.0);
    {
        size_t off = 0;
        int Ls = 1;
        for (int R : t.radices) {
            for (int k = 0; k < Ls; ++k)
                for (int q = 1; q < R; ++q) {
                    const long double ang = -2.0L * pi * static_cast<long double>(k) * q /
                                            (static_cast<long double>(R) * Ls);
                    t.tw[2 * off] = static_cast<double>(std::cos(ang));
                    t.tw[2 * off + 1] = static_cast<double>(std::sin(ang));
                    ++off;
                }
            Ls *= R;
        }
    }
    // a prime first pass needs no twiddles; its slots hold the roots
    // (cos, sin)(2 pi m / R), m = 1 .. R-1, that the pass reads
    if (!t.radices.empty() && t.radices[0] > 17) {
        const int R = t.radices[0];
        for (int m = 1; m < R; ++m) {
            const long double ang = 2.0L * pi * static_cast<long double>(m) / static_cast<long double>(R);
            t.tw[2 * (m - 1)] = static_cast<double>(std::cos(ang));
            t.tw[2 * (m - 1) + 1] = static_cast<double>(std::sin(ang));
        }
    }
    if (t.bluestein) {
        t.chirp.resize(2 * static_cast<size_t>(L));
        std::vector<cld> h(Nb, cld(0, 0));
        for (int nn = 0; nn < L; ++nn) {
            const long long q = (static_cast<long long>(nn) * nn) % (2LL * L);
            const long double ang = pi * static_cast<long double>(q) / L;
            t.chirp[2 * nn] = static_cast<double>(std::cos(ang));
            t.chirp[2 * nn + 1] = static_cast<double>(-std::sin(ang));
            h[nn] = cld(std::cos(ang), std::sin(ang));
            if (nn > 0) h[Nb - nn] = h[nn];
        }
        host_fft(h);
        t.bhat.resize(2 * static_cast<size_t>(Nb));
        for (int k = 0; k < Nb; ++k) {
            t.bhat[2 * k] = static_cast<double>(h[k].real() / Nb);
            t.bhat[2 * k + 1] = static_cast<double>(h[k].imag() / Nb);
        }
    }
    return t;
}

// ----------------------------------------------------------------------------
// horizontal (disk) Poisson tables
// ----------------------------------------------------------------------------

DiskTables build_disk_tables(const DirOps& ops, int nw) {
    DiskTables t;
    const int m = ops.n;
    const Band R2tau = band_cut(ops.R2f, m - 2, m);
    Band Rp[2];
    for (int par = 0; par < 2; ++par) {
        Rp[par] = band_parity(R2tau, par);
        t.rows[par] = Rp[par].rows;
        t.cols[par] = Rp[par].cols;
        for (int i = 0; i < Rp[par].rows; ++i)
            for (int j = 0; j < Rp[par].cols; ++j)
                if ((j < i - 1 || j > i + 3) && Rp[par].get(i, j) != 0.0)
                    throw std::logic_error("disk right side wider than its taps");
    }
    t.rmax = std::max(t.rows[0], t.rows[1]);
    t.taps.assign(2 * static_cast<size_t>(t.rmax) * kDiskTaps, 0.0);
    for (int par = 0; par < 2; ++par)
        for (int i = 0; i < t.rows[par]; ++i)
            for (int s = 0; s < kDiskTaps; ++s)
                t.taps[(static_cast<size_t>(par) * t.rmax + i) * kDiskTaps + s] = Rp[par].get(i, i - 1 + s);
    // PT curl right side: row i = 2q + par reads the other parity's
    // coefficients j = 2q' + 1 - par with q' = q - 1 + s, s < kDiskTaps
    t.pt_taps.assign(2 * static_cast<size_t>(t.rmax) * 2 * kDiskTaps, 0.0);
    for (int op = 0; op < 2; ++op) {
        const Band M = band_cut(op == 0 ? ops.PTa : ops.PTb, m - 2, m);
        for (int i = 0; i < m - 2; ++i)
            for (int j = 0; j < m; ++j) {
                const double v = M.get(i, j);
                if (v == 0.0) continue;
                const int par = i & 1, q = i >> 1, s = (j >> 1) - (q - 1);
                if ((j & 1) == par || s < 0 || s >= kDiskTaps)
                    throw std::logic_error("PT curl right side wider than its taps");
                t.pt_taps[((static_cast<size_t>(par) * t.rmax + q) * 2 + op) * kDiskTaps + s] = v;
            }
    }
    t.lu.assign(static_cast<size_t>(nw) * 2 * t.rmax * kDiskRec, 0.0);
    for (int w = 0; w < nw; ++w) {
        const Band Aw = band_axpby(1.0, ops.A0, -static_cast<double>(w) * w, ops.Cc);
        for (int par = 0; par < 2; ++par) {
            const Band A = band_parity(Aw, par);
            const int nr = A.rows;
            for (int i = 0; i < nr; ++i)
                for (int j = 0; j < nr; ++j)
                    if ((j < i - 1 || j > i + 2) && A.get(i, j) != 0.0)
                        throw std::logic_error("disk operator wider than (1, 2)");
            double* rec = &t.lu[((static_cast<size_t>(w) * 2 + par) * t.rmax) * kDiskRec];
            long double u0p = 0, u1p = 0, u2p = 0;    // previous row of U: d, U(i,i+1), U(i,i+2)
            for (int i = 0; i < nr; ++i) {
                const long double l = i > 0 ? static_cast<long double>(A.get(i, i - 1)) / u0p : 0.0L;
                const long double d = static_cast<long double>(A.get(i, i)) - l * u1p;
                const long double e1 = static_cast<long double>(A.get(i, i + 1)) - l * u2p;
                const long double e2 = static_cast<long double>(A.get(i, i + 2));
                if (d == 0.0L) throw std::runtime_error("zero pivot in the disk operator");
                rec[i * kDiskRec + 0] = static_cast<double>(l);
                rec[i * kDiskRec + 1] = static_cast<double>(1.0L / d);
                rec[i * kDiskRec + 2] = static_cast<double>(e1 / d);
                rec[i * kDiskRec + 3] = static_cast<double>(e2 / d);
                u0p = d; u1p = e1; u2p = e2;
            }
        }
    }
    return t;
}

}  // namespace cyl
