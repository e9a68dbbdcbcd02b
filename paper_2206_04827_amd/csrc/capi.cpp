// C ABI of the cylinder solver (declared in include/cylspec.h).
#include "../../include/cylspec.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <tuple>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include <unistd.h>

#include "kernels.hpp"
#include "plan.hpp"

namespace cyl {

namespace {

thread_local std::string g_last_error;

struct Failure {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw Failure{code, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            fail(CYL_E_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
        fail(CYL_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

template <typename F>
int guarded(F&& body) {
    try {
        body();
        return CYL_OK;
    } catch (const Failure& f) {
        g_last_error = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return CYL_E_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        g_last_error = std::string("internal error: ") + e.what();
        return CYL_E_INTERNAL;
    }
}

// Owned device allocation.
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 8;
        hip_check(hipMalloc(&p, b), "hipMalloc");
        bytes = b;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

template <typename T>
void upload(DevMem& m, const std::vector<T>& v) {
    m.alloc(v.size() * sizeof(T));
    if (!v.empty()) hip_check(hipMemcpy(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
}

int env_int(const char* name, int dflt);
static_assert(kMaxDftPasses == kMaxRadixPasses, "radix plan fits the device view");
static_assert(kPrimePassOutputs == kPrimeOutputs, "prime pass thread count matches the kernel");

struct DftOwned {
    DftTables t;
    DevMem tw, chirp, bhat;
    DftDev view{};
    void build(int L) {
        t = build_dft_tables(L, env_int("CYLSPEC_DFT_MIXED", 1) != 0, env_int("CYLSPEC_DFT_POINTS", 8) == 16 ? 16 : 8);
        upload(tw, t.tw);
        if (t.bluestein) { upload(chirp, t.chirp); upload(bhat, t.bhat); }
        view.L = t.L; view.Nb = t.Nb; view.tpl = t.tpl; view.pts = t.pts; view.bluestein = t.bluestein ? 1 : 0;
        view.nrad = static_cast<int>(t.radices.size());
        for (int i = 0; i < kMaxDftPasses; ++i) view.rad[i] = i < view.nrad ? t.radices[i] : 0;
        view.tw = tw.as<double2>();
        view.chirp = t.bluestein ? chirp.as<double2>() : nullptr;
        view.bhat = t.bluestein ? bhat.as<double2>() : nullptr;
    }
};

// ADI tables, block descriptors and operator-apply records of one pencil.
// flip: the transposed pencil in flipped block orientation (the adjoint).
struct Setup {
    AdiSetup h;
    int passes = 1;
    bool flip = false;
    DevMem rtab, ztab, vmu, blocks, atab, ztabA_own;
    const double* ztabA = nullptr;   // B/D column records of this orientation
    std::vector<BlockDesc> hblocks;
    // physical parity: the blocks with r-parity = w (mod 2), and the others
    DevMem blocks_phys, blocks_skip;
    int n_phys = 0, n_skip = 0;
    bool g16 = false;                // every block's halves are multiples of 16
    bool z16 = false;                // every block's z halves are multiples of 16
};

enum Phase { PH_FWD, PH_RHS, PH_ADI, PH_RES, PH_REC, PH_INV, PH_HRHS, PH_PROJ, PH_ADJ, PH_COUNT };

}  // namespace
}  // namespace cyl

using namespace cyl;

struct cyl_plan_s {
    int m = 0, n = 0, p = 0;
    hipStream_t stream = nullptr;
    Geometry geo;
    DirOps rops, zops;
    DftOwned dr, dz, dth;
    DevMem pre_fr, post_fr, pre_ir, post_ir, pre_fz, post_fz, pre_iz, post_iz, fold_r, fold_z;
    DevMem t_r2, t_a0, t_s10, t_c02, t_d2;
    RhsTables rhs{};
    DevMem plane_of, ztabA, atab_proj;
    DevMem planesA, planesB, E, X, R, state, acc;
    bool use_lds = false;
    bool adi_split = false;        // split-sweep kernel (two threads per line)
    bool split_gs = false;         //   with the block state in global memory
    int fused_res = 0;             //   emitting the first pass's residual itself (0 never,
                                   //   1 with enough blocks per compute unit, 2 always)
    int num_cus = 0;               // compute units of the device
    int dct_lines = 0;             // z-direction DCT: lines per workgroup at most (tuned; 0: default)
    int device = 0;                // the device current when the plan was created
    int64_t state_stride = 0;
    int adi_threads = 64;
    size_t lds_bytes = 0;
    std::map<double, std::unique_ptr<Setup>> setups;   // Poisson tables per prepared tolerance
    bool profiling = false;
    bool physical = false;         // Poisson solves keep the j = w (mod 2) blocks only
    std::unique_ptr<DiskTables> disk;   // horizontal Poisson records (built with the plan)
    DevMem disk_lu, disk_taps, disk_pt_taps;
    DevMem planesC;                // third coefficient-plane buffer (the PT decomposition)
    DevMem lift_ra, lift_zb;       // (1 + r_j)/2, (1 + z_k)/2 of the boundary-trace lift
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> recs;
};

struct cyl_heat_s {
    cyl_plan_t plan = nullptr;
    hipStream_t stream = nullptr;   // copy of the plan's stream: destroy needs no parent handle
    std::unique_ptr<Setup> setup;
    double alpha = 0, dt = 0, kappa = 0, tol = 0;
    int order = 1;
    double beta[4] = {0, 0, 0, 0};
    DevMem P[4], Econst, Xt, lift, T0;
    bool has_lift = false;
    bool physical = false; // steps solve the j = w (mod 2) blocks only (the plan's flag at creation)
    int head = 0;          // index of the newest history level
    long long steps = 0;
};

// Reverse-mode state of a BDF1 heat run: checkpoints of the projected state
// P_s = C~ X_s B~ every `every` steps (P_0 from T_0), the solutions X_k of the
// segment being differentiated, and the adjoint work buffers.
struct cyl_heat_grad_s {
    cyl_heat_t heat = nullptr;
    hipStream_t stream = nullptr;       // copy of the plan's stream (see cyl_heat_s)
    int steps = 0, every = 0, nseg = 0;
    int seg_holds = -1;                 // segment whose solutions X_k are in seg
    bool ready = false;                 // a forward run has filled the checkpoints
    std::unique_ptr<Setup> adj;         // transposed heat pencil, flipped orientation
    DevMem atab_pois, proj_flip;        // Poisson apply rows; flipped projection rows
    DevMem ckpt, seg, Pw, Xh, Et, Gsum, partials, planes, vals;
    int64_t ck_stride = 0, n_partials = 0;
};

// One launch of a batched ADI pass: every block of the group, cost-sorted.
struct BatchLaunch {
    int kind = 0;                 // 0 split sweeps, 1 LDS one thread per line, 2 HBM state
    int np = 0, threads = 0;
    size_t lds = 0;
    int nblocks = 0;
    int64_t state_stride = 0;
    bool g16 = false;             // 16-row groups: LDS split (kind 0) or forward z of the global-state split (kind 3)
    bool queue = false;           // split kinds: persistent workgroups over a work queue
    int grid = 0;                 //   and their number (resident at once)
    std::unique_ptr<cyl::DevMem> blocks, state, counter;
};

// Launch configuration of a batch's ADI passes (chosen by the tuner).
struct BatchCfg {
    int grouping = 0;             // 0 per (kernel, threads), 1 per (kernel, threads, width), 2 per kernel
    bool queue = false;           // work-queue launches of the split kernels
    bool g16 = true;              // 16-row groups where every block allows them
    std::string str() const {
        return "g" + std::to_string(grouping) + (queue ? "q1" : "q0") + (g16 ? "s16" : "s8");
    }
    static bool parse(const std::string& t, BatchCfg* c) {
        int g = -1, q = -1, sz = -1;
        if (std::sscanf(t.c_str(), "g%dq%ds%d", &g, &q, &sz) != 3 || g < 0 || g > 2 || (q != 0 && q != 1) ||
            (sz != 8 && sz != 16))
            return false;
        c->grouping = g;
        c->queue = q == 1;
        c->g16 = sz == 16;
        return true;
    }
};

// Batched heat stepping over independent problems (uneven sizes).
struct cyl_batch_s {
    hipStream_t user = nullptr;          // the stream of every member's plan
    hipStream_t stream = nullptr;        // the batch's own stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<cyl_heat_t> heats;
    std::vector<int> head0;              // heads the cycle tables were built for
    std::vector<long long> steps0;
    int L = 1, pos = 0;                  // steps per cycle; position of the next step
    long long taken = 0;                 // steps advanced by the batch
    std::vector<std::unique_ptr<cyl::DevMem>> E, R;   // per-problem right side / residual
    std::vector<BatchLaunch> adi1, adi2; // pass 1 (all), pass 2 (two-pass problems)
    cyl::DevMem ptr1, ptr2;              // AdiPtrs per problem for the two passes
    cyl::DevMem blocks_all;              // every block, prob set (apply items index it)
    cyl::DevMem res_items, res_ptrs;
    int n_res = 0;
    cyl::DevMem proj_items;
    int n_proj = 0;
    std::vector<std::unique_ptr<cyl::DevMem>> proj_ptrs, rhs_items;   // per cycle position
    cyl::DevMem rhs_wg;
    int64_t rhs_nwg = 0;
    std::string grouping;
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~cyl_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace cyl {
namespace {

// ---------------------------------------------------------------------------
// profiling scopes
// ---------------------------------------------------------------------------
struct Scope {
    cyl_plan_t pl;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    Scope(cyl_plan_t p, int ph) : pl(p), phase(ph) {
        if (!pl->profiling) return;
        hip_check(hipEventCreate(&a), "hipEventCreate");
        hip_check(hipEventCreate(&b), "hipEventCreate");
        hip_check(hipEventRecord(a, pl->stream), "hipEventRecord");
    }
    ~Scope() {
        if (!pl->profiling || !a) return;
        if (hipEventRecord(b, pl->stream) == hipSuccess) pl->recs.push_back({phase, a, b});
    }
};

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

// Passes and per-pass tolerance: for large grids a tight tolerance is reached
// in two passes of sqrt(eps), with the FP64 residual in between, because one
// long pass stalls at the rounding floor of the shifted solves.
void pass_policy(int m, int n, double eps, int* passes, double* eps_pass) {
    int ps = (eps < 1e-8 && std::max(m, n) >= 192) ? 2 : 1;
    const int forced = env_int("CYLSPEC_PASSES", 0);
    if (forced == 1 || forced == 2) ps = forced;
    *passes = ps;
    *eps_pass = ps == 2 ? std::sqrt(eps) : eps;
}

// Operator-apply records of a pencil (residuals): per w, per r parity, rows of
// 12 (A row i at i-2..i+3, then C row i at i-2..i+3).  ka == 0: Poisson pencil
// (A_w, C~); otherwise the heat pencil (C~ - ka A_w, -ka C~).
std::vector<double> apply_rows(const cyl_plan_s* pl, double ka, bool flip) {
    const Geometry& g = pl->geo;
    const int me0 = g.me[0], me1 = g.me[1];
    std::vector<double> at(static_cast<size_t>(g.nw) * (me0 + me1) * 12, 0.0);
    for (int w = 0; w < g.nw; ++w) {
        const Band Aw = band_axpby(1.0, pl->rops.A0, -static_cast<double>(w) * w, pl->rops.Cc);
        const Band A = ka > 0.0 ? band_axpby(1.0, pl->rops.R2Q, -ka, Aw) : Aw;
        const Band C = ka > 0.0 ? band_axpby(-ka, pl->rops.R2Q, 0.0, pl->rops.R2Q) : pl->rops.R2Q;
        size_t base = static_cast<size_t>(w) * (me0 + me1) * 12;
        for (int pr = 0; pr < 2; ++pr) {
            Band Ap = band_parity(A, pr), Cp = band_parity(C, pr);
            if (flip) { Ap = band_flip_transpose(Ap); Cp = band_flip_transpose(Cp); }
            for (int i = 0; i < Ap.rows; ++i) {
                for (int t = 0; t < 6; ++t) {
                    at[base + i * 12 + t] = Ap.get(i, i - 2 + t);
                    at[base + i * 12 + 6 + t] = Cp.get(i, i - 2 + t);
                }
            }
            base += static_cast<size_t>(Ap.rows) * 12;
        }
    }
    return at;
}

// z apply records: per z parity, columns of 8 (B column k at rows k-1..k+2,
// then D column k likewise), B = C02Q^T and D = D2Q^T.
std::vector<double> z_columns(const cyl_plan_s* pl, bool flip) {
    const Geometry& g = pl->geo;
    const Band Bt = band_transpose(pl->zops.C02Q), Dt = band_transpose(pl->zops.D2Q);
    std::vector<double> za(static_cast<size_t>(g.ne[0] + g.ne[1]) * 8, 0.0);
    size_t base = 0;
    for (int pz = 0; pz < 2; ++pz) {
        Band Bp = band_parity(Bt, pz), Dp = band_parity(Dt, pz);
        if (flip) { Bp = band_flip_transpose(Bp); Dp = band_flip_transpose(Dp); }
        for (int k = 0; k < Bp.cols; ++k)
            for (int t = 0; t < 4; ++t) {
                za[base + k * 8 + t] = Bp.get(k - 1 + t, k);
                za[base + k * 8 + 4 + t] = Dp.get(k - 1 + t, k);
            }
        base += static_cast<size_t>(Bp.cols) * 8;
    }
    return za;
}

// Projection records (heat history C~ X B~): A = R2Q rows, C = 0, shared by all w.
std::vector<double> projection_rows(const cyl_plan_s* pl, bool flip) {
    const Geometry& g = pl->geo;
    std::vector<double> ap(static_cast<size_t>(g.me[0] + g.me[1]) * 12, 0.0);
    size_t base = 0;
    for (int pr = 0; pr < 2; ++pr) {
        Band Cp = band_parity(pl->rops.R2Q, pr);
        if (flip) Cp = band_flip_transpose(Cp);
        for (int i = 0; i < Cp.rows; ++i)
            for (int t = 0; t < 6; ++t) ap[base + i * 12 + t] = Cp.get(i, i - 2 + t);
        base += static_cast<size_t>(Cp.rows) * 12;
    }
    return ap;
}

std::unique_ptr<Setup> make_setup(cyl_plan_t pl, double ka, double eps, bool flip = false) {
    auto s = std::make_unique<Setup>();
    double eps_pass;
    pass_policy(pl->m, pl->n, eps, &s->passes, &eps_pass);
    // test only: CYLSPEC_TEST_BOUNDS_SCALE in (0, 1) shrinks the eigenvalue
    // bounds so that they no longer enclose the spectrum (drives the residual
    // check to CYL_E_NOT_CONVERGED without any fault)
    double a_scale = 1.0;
    if (const char* t = std::getenv("CYLSPEC_TEST_BOUNDS_SCALE")) {
        const double v = std::atof(t);
        if (v > 0.0 && v < 1.0) a_scale = v;
    }
    s->h = build_adi_setup(pl->geo, pl->rops, pl->zops, ka, eps_pass, flip, pl->adi_split, a_scale);
    s->flip = flip;
    const Geometry& g = pl->geo;
    const int me0 = g.me[0], me1 = g.me[1], ne0 = g.ne[0], ne1 = g.ne[1];
    // block offsets inside a plane: (pr, pz) = (0,0), (0,1), (1,0), (1,1)
    const int64_t eblk[4] = {0, static_cast<int64_t>(g.mp[0]) * ne0,
                             static_cast<int64_t>(g.mp[0]) * (ne0 + ne1),
                             static_cast<int64_t>(g.mp[0]) * (ne0 + ne1) + static_cast<int64_t>(g.mp[1]) * ne0};
    const int64_t xblk[4] = {0, static_cast<int64_t>(me0) * ne0, static_cast<int64_t>(me0) * (ne0 + ne1),
                             static_cast<int64_t>(me0) * (ne0 + ne1) + static_cast<int64_t>(me1) * ne0};
    for (int pl_i = 0; pl_i < g.nplanes; ++pl_i) {
        const int w = g.plane_w[pl_i];
        for (int pr = 0; pr < 2; ++pr)
            for (int pz = 0; pz < 2; ++pz) {
                BlockDesc b{};
                b.w = w; b.J = s->h.J[w]; b.me = g.me[pr]; b.ne = g.ne[pz];
                b.mp = g.mp[pr]; b.np = g.np[pz];
                b.pr = pr; b.pz = pz; b.part = g.plane_part[pl_i]; b.plane = pl_i;
                b.eoff = pl_i * g.eplane_elems + eblk[2 * pr + pz];
                b.xoff = pl_i * g.plane_elems + xblk[2 * pr + pz];
                b.rstride = static_cast<int64_t>(s->h.rrows[0] + s->h.rrows[1]) * kRRec;
                b.zstride = static_cast<int64_t>(s->h.zrows[0] + s->h.zrows[1]) * kZRec;
                b.rbase = s->h.roff[w] + (pr ? static_cast<int64_t>(s->h.rrows[0]) * kRRec : 0);
                b.zbase = s->h.zoff[w] + (pz ? static_cast<int64_t>(s->h.zrows[0]) * kZRec : 0);
                b.tr = s->h.tr[pr];
                b.tz = s->h.tz[pz];
                b.soff = s->h.soff[w];
                s->hblocks.push_back(b);
            }
    }
    // the ADI kernel copies records in 128-double chunks: keep read slack
    s->h.rtab.resize(s->h.rtab.size() + 256, 0.0);
    s->h.ztab.resize(s->h.ztab.size() + 256, 0.0);
    upload(s->rtab, s->h.rtab);
    upload(s->ztab, s->h.ztab);
    upload(s->vmu, s->h.vmu);
    upload(s->blocks, s->hblocks);
    s->g16 = env_int("CYLSPEC_ADI_G16", 1) != 0 && !s->hblocks.empty() &&
             std::all_of(s->hblocks.begin(), s->hblocks.end(), [](const BlockDesc& b) { return adi_split_g16(b); });
    s->z16 = env_int("CYLSPEC_ADI_G16", 1) != 0 && !s->hblocks.empty() &&
             std::all_of(s->hblocks.begin(), s->hblocks.end(), [](const BlockDesc& b) { return adi_split_gs_z16(b); });
    if (env_int("CYLSPEC_LOG", 0) > 0 && pl->adi_split && !pl->split_gs)
        std::fprintf(stderr, "[cylspec] ADI tables: %zu blocks, %d rows per group in the backward r and the z sweeps\n",
                     s->hblocks.size(), s->g16 ? 16 : 8);
    if (env_int("CYLSPEC_LOG", 0) > 0 && pl->split_gs)
        std::fprintf(stderr, "[cylspec] ADI tables: %zu blocks, %d rows per group in the forward z sweeps (state in "
                             "global memory)\n", s->hblocks.size(), s->z16 ? 16 : 8);
    {
        std::vector<BlockDesc> keep, skip;
        for (const BlockDesc& b : s->hblocks) (b.pr == (std::abs(b.w) & 1) ? keep : skip).push_back(b);
        s->n_phys = static_cast<int>(keep.size());
        s->n_skip = static_cast<int>(skip.size());
        upload(s->blocks_phys, keep);
        upload(s->blocks_skip, skip);
    }
    upload(s->atab, apply_rows(pl, ka, flip));
    if (flip) {
        upload(s->ztabA_own, z_columns(pl, true));
        s->ztabA = s->ztabA_own.as<double>();
    } else {
        s->ztabA = pl->ztabA.as<double>();
    }
    return s;
}

// The Poisson tables of a tolerance: built (host work, device allocation)
// by cyl_plan_prepare only; a solve finds them or fails.
Setup* poisson_setup(cyl_plan_t pl, double eps, bool build) {
    auto it = pl->setups.find(eps);
    if (it != pl->setups.end()) return it->second.get();
    if (!build) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "adi_tol %.17g is not prepared on this plan (call cyl_plan_prepare "
                                        "first; solves allocate nothing)", eps);
        fail(CYL_E_INVALID_ARG, buf);
    }
    auto s = make_setup(pl, 0.0, eps);
    Setup* raw = s.get();
    pl->setups[eps] = std::move(s);
    return raw;
}

// E-layout buffer: zero padding rows, plus read-ahead slack after the end.
void alloc_elayout(DevMem& m, const Geometry& g) {
    const size_t bytes = (static_cast<size_t>(g.etotal_elems) + 64) * sizeof(double);
    m.alloc(bytes);
    hip_check(hipMemset(m.p, 0, bytes), "hipMemset");
}

// ---------------------------------------------------------------------------
// transform sequences
// ---------------------------------------------------------------------------
LineSet r_lines(const Geometry& g) {
    LineSet ls{};
    ls.outer = static_cast<int64_t>(g.n) * g.m; ls.inner = g.m; ls.elem = 1;
    ls.n_outer = g.nw; ls.n_inner = g.n;
    return ls;
}
LineSet z_lines(const Geometry& g) {
    LineSet ls{};
    ls.outer = static_cast<int64_t>(g.n) * g.m; ls.inner = 1; ls.elem = g.m;
    ls.n_outer = g.nw; ls.n_inner = g.m;
    return ls;
}

void transform_fwd(cyl_plan_t pl, const double* values, double2* coeffs) {
    Scope sc(pl, PH_FWD);
    const Geometry& g = pl->geo;
    hip_check(launch_theta_fwd(values, coeffs, g.m, g.n, g.p, pl->dth.view, pl->stream), "theta_fwd");
    hip_check(launch_dct(coeffs, coeffs, z_lines(g), g.n, false, pl->dz.view, pl->pre_fz.as<double>(),
                         pl->post_fz.as<double>(), pl->fold_z.as<double2>(), pl->stream, pl->dct_lines),
              "dct_z_fwd");
    hip_check(launch_dct(coeffs, coeffs, r_lines(g), g.m, true, pl->dr.view, pl->pre_fr.as<double>(),
                         pl->post_fr.as<double>(), pl->fold_r.as<double2>(), pl->stream), "dct_r_fwd");
}

// W: coefficient-plane workspace (nullptr: the plan's planesA); coeffs may
// equal W (in place) and is not modified otherwise.
void transform_inv(cyl_plan_t pl, const double2* coeffs, double* values, double2* W = nullptr) {
    Scope sc(pl, PH_INV);
    const Geometry& g = pl->geo;
    if (!W) W = pl->planesA.as<double2>();
    hip_check(launch_dct(coeffs, W, r_lines(g), g.m, true, pl->dr.view, pl->pre_ir.as<double>(),
                         pl->post_ir.as<double>(), pl->fold_r.as<double2>(), pl->stream), "dct_r_inv");
    hip_check(launch_dct(W, W, z_lines(g), g.n, false, pl->dz.view, pl->pre_iz.as<double>(),
                         pl->post_iz.as<double>(), pl->fold_z.as<double2>(), pl->stream, pl->dct_lines),
              "dct_z_inv");
    hip_check(launch_theta_inv(W, values, g.m, g.n, g.p, pl->dth.view, pl->stream), "theta_inv");
}

// values = F^T coeffs (the transpose of transform_fwd with respect to the real
// inner products of both arrays).  U is overwritten; it must not be planesA.
void transform_fwd_adjoint(cyl_plan_t pl, double2* U, double* values) {
    const Geometry& g = pl->geo;
    {
        Scope sc(pl, PH_ADJ);
        hip_check(launch_scale_planes(U, g.m, g.n, g.p, 0, pl->stream), "scale planes");
    }
    transform_inv(pl, U, values);
    Scope sc(pl, PH_ADJ);
    hip_check(launch_scale_values(values, values, g.m, g.n, g.p, 0, pl->stream), "scale values");
}

// coeffs = F^-T values (the transpose of transform_inv); tmp holds p n m doubles.
void transform_inv_adjoint(cyl_plan_t pl, const double* values, double* tmp, double2* coeffs) {
    const Geometry& g = pl->geo;
    {
        Scope sc(pl, PH_ADJ);
        hip_check(launch_scale_values(values, tmp, g.m, g.n, g.p, 1, pl->stream), "scale values");
    }
    transform_fwd(pl, tmp, coeffs);
    Scope sc(pl, PH_ADJ);
    hip_check(launch_scale_planes(coeffs, g.m, g.n, g.p, 1, pl->stream), "scale planes");
}

// Device workspace of one solve: the plan's own buffers, or (the
// allocation-free entry point) a carve-out of the static scratch.
struct Work {
    double2* planesA = nullptr;   // coefficient planes
    double2* planesB = nullptr;   //   (the lift's, Poisson with bc_lift only)
    double* E = nullptr;          // right side, E-layout
    double* X = nullptr;          // solution blocks, X-layout
    double* R = nullptr;          // residual, E-layout
    double* acc = nullptr;        // 4 reduction slots
    double* state = nullptr;      // block state of the HBM/global-state ADI kernels
};

Work plan_work(cyl_plan_s* pl) {
    Work w;
    w.planesA = pl->planesA.as<double2>();
    w.planesB = pl->planesB.as<double2>();
    w.E = pl->E.as<double>();
    w.X = pl->X.as<double>();
    w.R = pl->R.as<double>();
    w.acc = pl->acc.as<double>();
    w.state = pl->state.as<double>();
    return w;
}

// LDS of a global-state split launch: everything a workgroup may use when
// the LDS band is on (its rows around the r split stay on the chip), else
// what the records, the exchange area (and the residual epilogue) need.
size_t gs_launch_lds(size_t needed) {
    if (env_int("CYLSPEC_ADI_GS_BAND", 1) == 0) return needed;
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return needed;
    int per_cu = 0;
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
        lim = std::max(lim, per_cu);
    // 1 KB below the limit: room for the work-queue instances' static LDS
    return std::max(needed, static_cast<size_t>(lim) - 1024);
}

// Two passes with split kernels: the first pass writes the residual of its
// own solution (no separate residual launch).  Every round of resident blocks
// then ends in a burst of E and R traffic; measured, this pays only with at
// least four blocks per compute unit (one block per unit fits in LDS), the
// separate full-occupancy launch otherwise.
bool fuse_residual(const cyl_plan_s* pl, const Setup* s, bool physical) {
    const int nblk = physical ? s->n_phys : static_cast<int>(s->hblocks.size());
    return s->passes == 2 && (pl->fused_res == 2 ||
                              (pl->fused_res == 1 && pl->num_cus > 0 && nblk >= 4 * pl->num_cus));
}

// ADI solve of all blocks (physical: the j = w (mod 2) blocks only):
// X <- solution of A X B + C X D = E (setup pencil).  Residuals go to R,
// the block state of the global-state kernels to `state` (nullptr: the
// plan's buffers).
void adi_solve(cyl_plan_t pl, Setup* s, const double* E, double* X, bool physical = false,
               double* R = nullptr, double* state = nullptr) {
    const Geometry& g = pl->geo;
    if (!R) R = pl->R.as<double>();
    if (!state) state = pl->state.as<double>();
    const int nblk = physical ? s->n_phys : static_cast<int>(s->hblocks.size());
    DevMem& blocks = physical ? s->blocks_phys : s->blocks;
    const int64_t a_wstride = static_cast<int64_t>(g.me[0] + g.me[1]) * 12;
    const bool fuse = fuse_residual(pl, s, physical);
    const ResArgs res{R, s->atab.as<double>(), s->ztabA, a_wstride, g.me[0], g.ne[0]};
    for (int pass = 0; pass < s->passes; ++pass) {
        const double* rhs = E;
        if (pass > 0 && fuse) {
            rhs = R;
        } else if (pass > 0) {
            Scope sc(pl, PH_RES);
            hip_check(launch_apply2(blocks.as<BlockDesc>(), nblk, g.me[0], g.ne[0], E, 1.0, X, 1.0, 1.0,
                                    R, s->atab.as<double>(), a_wstride,
                                    s->ztabA, pl->stream), "residual");
            rhs = R;
        }
        Scope sc(pl, PH_ADI);
        const ResArgs* rp = fuse && pass == 0 ? &res : nullptr;
        if (pl->adi_split && pl->split_gs)
            hip_check(launch_adi_split_gs(blocks.as<BlockDesc>(), nblk, pl->adi_threads, g.np[0], rhs, X,
                                          state, pl->state_stride, s->rtab.as<double>(),
                                          s->ztab.as<double>(), s->vmu.as<double>(), pass > 0, pl->lds_bytes,
                                          pl->stream, nullptr, rp, s->z16),
                      "adi");
        else if (pl->adi_split)
            hip_check(launch_adi_split(blocks.as<BlockDesc>(), nblk, pl->adi_threads, g.np[0], rhs, X,
                                       s->rtab.as<double>(), s->ztab.as<double>(), s->vmu.as<double>(),
                                       pass > 0, pl->lds_bytes, pl->stream, nullptr, rp, s->g16),
                      "adi");
        else
            hip_check(launch_adi(blocks.as<BlockDesc>(), nblk, pl->adi_threads, g.np[0], rhs, X,
                                 state, pl->state_stride, s->rtab.as<double>(),
                                 s->ztab.as<double>(),
                                 s->vmu.as<double>(), pass > 0, pl->use_lds, pl->lds_bytes, pl->stream),
                      "adi");
    }
}

// Residual check of a solve (synchronises): R and acc are workspace.
void check_residual(cyl_plan_t pl, Setup* s, const double* E, const double* X, double* R, double* acc,
                    double eps, cyl_solve_info* info) {
    const Geometry& g = pl->geo;
    const int nblk = static_cast<int>(s->hblocks.size());
    {
        Scope sc(pl, PH_RES);
        hip_check(launch_apply2(s->blocks.as<BlockDesc>(), nblk, g.me[0], g.ne[0], E, 1.0, X, 1.0, 1.0,
                                R, s->atab.as<double>(),
                                static_cast<int64_t>(g.me[0] + g.me[1]) * 12,
                                s->ztabA, pl->stream), "residual");
    }
    hip_check(launch_fill_zero(acc, 3, pl->stream), "clear norms");
    hip_check(launch_norms(R, E, g.etotal_elems, X, g.total_elems, acc, pl->stream), "norms");
    double h[3];
    hip_check(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, pl->stream), "copy norms");
    hip_check(hipStreamSynchronize(pl->stream), "sync");
    info->J_max = s->h.J_max;
    info->J_min = s->h.J_min;
    info->passes = s->passes;
    info->fused_residual = fuse_residual(pl, s, pl->physical) ? 1 : 0;
    info->adi_iterations_mean = s->h.J_mean;
    info->resid_ratio = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
    const double lim = 1e3 * std::max(eps, 1e-12);
    if (h[2] > 0.0 || !std::isfinite(info->resid_ratio) || info->resid_ratio > lim)
        fail(CYL_E_NOT_CONVERGED, "ADI result not finite or residual ratio " +
                                      std::to_string(info->resid_ratio) + " above " + std::to_string(lim));
}

void validate_tol(double eps) {
    if (!(eps >= 1e-15 && eps <= 1e-2)) fail(CYL_E_INVALID_ARG, "adi_tol must lie in [1e-15, 1e-2]");
}
void validate_space(int space) {
    if (space != CYL_SPACE_VALUE && space != CYL_SPACE_COEFF) fail(CYL_E_INVALID_ARG, "space must be CYL_SPACE_VALUE or CYL_SPACE_COEFF");
}

// Lines per workgroup of the z-direction DCT, chosen by timing: more lines
// mean fewer, larger workgroups; the best count depends on the length
// (measured: 32 at 256^3, 16 at 192^3 and 512^3).  Timed on the plan's own
// coefficient planes (zero-filled) for plans of at least 2^20 complex
// coefficients; CYLSPEC_DCT_LINES fixes the count instead.
void tune_dct_lines(cyl_plan_t pl) {
    const Geometry& g = pl->geo;
    const int64_t elems = static_cast<int64_t>(g.nw) * g.n * g.m;
    if (env_int("CYLSPEC_DCT_LINES", 0) > 0 || env_int("CYLSPEC_TUNE_DCT", 1) == 0 || elems < (1 << 20)) return;
    double2* A = pl->planesA.as<double2>();
    hip_check(launch_fill_zero(reinterpret_cast<double*>(A), 2 * elems, pl->stream), "zero planes");
    struct Ev {
        hipEvent_t a = nullptr, b = nullptr;
        ~Ev() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    hip_check(hipEventCreate(&ev.a), "hipEventCreate");
    hip_check(hipEventCreate(&ev.b), "hipEventCreate");
    int best = 0;
    float best_ms = 1e30f;
    for (int lines : {8, 16, 32}) {
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hip_check(hipEventRecord(ev.a, pl->stream), "hipEventRecord");
            hip_check(launch_dct(A, A, z_lines(g), g.n, false, pl->dz.view, pl->pre_fz.as<double>(),
                                 pl->post_fz.as<double>(), pl->fold_z.as<double2>(), pl->stream, lines),
                      "dct tuning");
            hip_check(hipEventRecord(ev.b, pl->stream), "hipEventRecord");
            hip_check(hipEventSynchronize(ev.b), "hipEventSynchronize");
            float t = 0.0f;
            hip_check(hipEventElapsedTime(&t, ev.a, ev.b), "hipEventElapsedTime");
            if (rep > 0) ms = std::min(ms, t);      // the first run warms the instance up
        }
        if (ms < best_ms) { best_ms = ms; best = lines; }
    }
    pl->dct_lines = best;
}

void build_plan(cyl_plan_t pl) {
    const int m = pl->m, n = pl->n, p = pl->p;
    pl->geo = make_geometry(m, n, p);
    pl->rops = build_dir_ops(m);
    pl->zops = build_dir_ops(n);
    pl->dr.build(m - 1);
    pl->dz.build(n - 1);
    // fold table of the length-(M) DCT-I: (cos(pi j / M), sin(pi j / M)), j = 0..M
    auto fold_tab = [](int len, DevMem& f) {
        const int M = len - 1;
        const long double pi = 3.141592653589793238462643383279502884L;
        std::vector<double> v(2 * static_cast<size_t>(M + 1));
        for (int j = 0; j <= M; ++j) {
            const long double a = pi * static_cast<long double>(j) / static_cast<long double>(M);
            v[2 * j] = static_cast<double>(std::cos(a));
            v[2 * j + 1] = static_cast<double>(std::sin(a));
        }
        upload(f, v);
    };
    fold_tab(m, pl->fold_r);
    // (1 + r_j)/2 and (1 + z_k)/2 of the doubled grid, r_j = cos((m - 1 - j) pi / (m - 1))
    auto unit_tab = [](int len, DevMem& t) {
        const double pi = 3.14159265358979323846;
        std::vector<double> v(static_cast<size_t>(len));
        for (int j = 0; j < len; ++j) v[j] = 0.5 * (1.0 + std::cos((len - j - 1) * pi / (len - 1)));
        upload(t, v);
    };
    unit_tab(m, pl->lift_ra);
    unit_tab(n, pl->lift_zb);
    fold_tab(n, pl->fold_z);
    pl->dth.build(p);
    // DCT pre/post factors: forward c_k = (-1)^k s_k / M * DCT-I(f)_k with
    // s_0 = s_M = 1/2; inverse f = DCT-I(g), g_k = (-1)^k c_k (halved inside).
    auto dct_tabs = [](int len, DevMem& pf, DevMem& qf, DevMem& pi, DevMem& qi) {
        const int M = len - 1;
        std::vector<double> pre_f(len, 1.0), post_f(len), pre_i(len), post_i(len, 1.0);
        for (int k = 0; k < len; ++k) {
            const double sg = (k & 1) ? -1.0 : 1.0;
            const double half = (k == 0 || k == M) ? 0.5 : 1.0;
            post_f[k] = sg * half / M;
            pre_i[k] = sg * ((k == 0 || k == M) ? 1.0 : 0.5);
        }
        upload(pf, pre_f); upload(qf, post_f); upload(pi, pre_i); upload(qi, post_i);
    };
    dct_tabs(m, pl->pre_fr, pl->post_fr, pl->pre_ir, pl->post_ir);
    dct_tabs(n, pl->pre_fz, pl->post_fz, pl->pre_iz, pl->post_iz);
    // tau right-hand-side tables (full T-coefficient operators)
    std::vector<double> r2(static_cast<size_t>(m - 2) * 5), a0(static_cast<size_t>(m - 2) * 4),
        s10(static_cast<size_t>(m - 2) * 4), c02(static_cast<size_t>(n - 2) * 3), d2(n - 2);
    for (int i = 0; i < m - 2; ++i) {
        for (int t = 0; t < 5; ++t) r2[i * 5 + t] = pl->rops.R2f.get(i, i - 2 + 2 * t);
        for (int t = 0; t < 4; ++t) {
            a0[i * 4 + t] = pl->rops.A0f.get(i, i - 2 + 2 * t);
            s10[i * 4 + t] = pl->rops.S10f.get(i, i - 2 + 2 * t);
        }
    }
    for (int k = 0; k < n - 2; ++k) {
        for (int t = 0; t < 3; ++t) c02[k * 3 + t] = pl->zops.C02f.get(k, k + 2 * t);
        d2[k] = pl->zops.D2f.get(k, k + 2);
    }
    upload(pl->t_r2, r2); upload(pl->t_a0, a0); upload(pl->t_s10, s10);
    upload(pl->t_c02, c02); upload(pl->t_d2, d2);
    pl->rhs.r2 = pl->t_r2.as<double>(); pl->rhs.a0 = pl->t_a0.as<double>();
    pl->rhs.s10 = pl->t_s10.as<double>(); pl->rhs.c02 = pl->t_c02.as<double>();
    pl->rhs.d2 = pl->t_d2.as<double>();
    const Geometry& g = pl->geo;
    std::vector<int> pof(2 * g.nw, -1);
    for (int i = 0; i < g.nplanes; ++i) pof[2 * g.plane_w[i] + g.plane_part[i]] = i;
    upload(pl->plane_of, pof);
    upload(pl->ztabA, z_columns(pl, false));
    upload(pl->atab_proj, projection_rows(pl, false));
    // workspace
    const size_t planes_bytes = static_cast<size_t>(g.nw) * n * m * sizeof(double2);
    const size_t blk_bytes = static_cast<size_t>(g.total_elems) * sizeof(double);
    pl->planesA.alloc(planes_bytes);
    pl->planesB.alloc(planes_bytes);
    pl->planesC.alloc(planes_bytes);
    alloc_elayout(pl->E, g);
    pl->X.alloc(blk_bytes);
    alloc_elayout(pl->R, g);
    pl->acc.alloc(4 * sizeof(double));
    // ADI variant: LDS-resident when the largest block and its records fit
    pl->adi_threads = ((std::max(g.me[0], g.ne[0]) + 63) / 64) * 64;
    pl->state_stride = static_cast<int64_t>(g.mp[0] + 4) * (g.np[0] + 1);
    auto chunks = [](int x) { return static_cast<size_t>((x + 127) / 128 * 128); };
    pl->lds_bytes = (static_cast<size_t>(pl->state_stride) + chunks(kRRec * g.mp[0]) +
                     chunks(kZRec * g.np[0])) * sizeof(double);
    int dev = 0, max_lds = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) max_lds = 65536;
    int max_lds_sm = 0;
    if (hipDeviceGetAttribute(&max_lds_sm, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
        max_lds = std::max(max_lds, max_lds_sm);
    if (hipDeviceGetAttribute(&pl->num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        pl->num_cus = 0;
    pl->device = dev;
    hip_check(scratch_init(dev), "static scratch address");
    // horizontal (disk) Poisson records: small, built here so that the disk
    // solve allocates nothing
    {
        auto t = std::make_unique<DiskTables>(build_disk_tables(pl->rops, g.nw));
        upload(pl->disk_lu, t->lu);
        upload(pl->disk_taps, t->taps);
        upload(pl->disk_pt_taps, t->pt_taps);
        pl->disk = std::move(t);
    }
    const int mode = env_int("CYLSPEC_ADI_GLOBAL", 0);
    pl->use_lds = mode == 0 && pl->adi_threads <= 256 && g.np[0] <= 128 &&
                  pl->lds_bytes <= static_cast<size_t>(max_lds);
    if (pl->use_lds && pl->lds_bytes > 65536) {
        if (adi_set_lds_limit(g.np[0], pl->lds_bytes) != hipSuccess) {
            (void)hipGetLastError();
            pl->use_lds = false;
        }
    }
    // split sweeps (two threads per line) when every parity block is long enough
    if (env_int("CYLSPEC_ADI_SPLIT", 1) != 0 && mode == 0 && g.np[0] <= 128 && g.mp[0] <= 128 &&
        adi_split_fits(std::min(g.me[0], g.me[1]), std::min(g.ne[0], g.ne[1]))) {
        const size_t sb = adi_split_lds_bytes(g.mp[0], g.np[0]);
        bool ok = sb <= static_cast<size_t>(max_lds);
        if (ok && sb > 65536 && adi_split_set_lds_limit(g.np[0], sb) != hipSuccess) {
            (void)hipGetLastError();
            ok = false;
        }
        if (ok) {
            pl->adi_split = true;
            pl->adi_threads = 2 * (((std::max(g.me[0], g.ne[0]) + 63) / 64) * 64);
            pl->lds_bytes = sb;
            pl->use_lds = true;
        }
    } else if (env_int("CYLSPEC_ADI_SPLIT", 1) != 0 && mode == 0 && g.np[0] > 128 && g.np[0] <= 256 &&
               g.mp[0] <= 256 && adi_split_fits(std::min(g.me[0], g.me[1]), std::min(g.ne[0], g.ne[1]))) {
        // blocks too large for LDS: split sweeps with the state in global memory
        const int lines = ((std::max(g.me[0], g.ne[0]) + 63) / 64) * 64;
        pl->adi_split = true;
        pl->split_gs = true;
        pl->adi_threads = 2 * lines;
        pl->fused_res = env_int("CYLSPEC_ADI_FUSED_RES", 1);
        pl->lds_bytes = gs_launch_lds(adi_split_gs_lds_bytes(g.mp[0], g.np[0], lines, pl->fused_res != 0));
        if (pl->lds_bytes > 65536 && adi_split_gs_set_lds_limit(g.np[0], pl->lds_bytes) != hipSuccess) {
            (void)hipGetLastError();
            pl->fused_res = 0;
            pl->lds_bytes = adi_split_gs_lds_bytes(g.mp[0], g.np[0], lines, false);
        }
        pl->state_stride = adi_split_gs_state_stride(g.mp[0], g.np[0]);
        pl->state.alloc(static_cast<size_t>(4 * g.nplanes) * pl->state_stride * sizeof(double));
        pl->use_lds = true;        // no HBM-state one-thread kernel
    }
    if (pl->adi_split && !pl->split_gs) pl->fused_res = env_int("CYLSPEC_ADI_FUSED_RES", 1);
    if (!pl->use_lds) {
        pl->adi_threads = std::min(512, pl->adi_threads);
        pl->state.alloc(static_cast<size_t>(4 * g.nplanes) * pl->state_stride * sizeof(double));
    }
    tune_dct_lines(pl);
    if (env_int("CYLSPEC_LOG", 0) > 0)
        std::fprintf(stderr, "[cylspec] plan %dx%dx%d: blocks me=(%d,%d) ne=(%d,%d), ADI %s, %d threads, "
                             "LDS %zu of %d bytes, DFT Nb r/z/theta = %d/%d/%d, z-DCT lines per workgroup <= %d\n",
                     m, n, p, g.me[0], g.me[1], g.ne[0], g.ne[1],
                     pl->split_gs ? "split, global state" : pl->adi_split ? "LDS-resident split"
                                                           : pl->use_lds ? "LDS-resident" : "HBM-resident",
                     pl->adi_threads, pl->lds_bytes, max_lds, pl->dr.t.Nb, pl->dz.t.Nb, pl->dth.t.Nb,
                     pl->dct_lines > 0 ? pl->dct_lines : 8);
}

// One BDF1 step of the handle's pencil: X = S^-1 (Pin + Econst), Pout = C~ X B~.
void heat_step_bdf1(cyl_heat_t h, const double* Pin, double* X, double* Pout) {
    cyl_plan_s* pl = h->plan;
    const Geometry& g = pl->geo;
    Setup* s = h->setup.get();
    const double* P[1] = {Pin};
    const double one = 1.0;
    {
        Scope sc(pl, PH_HRHS);
        hip_check(launch_heat_rhs(pl->E.as<double>(), P, &one, 1, h->Econst.as<double>(), g.etotal_elems,
                                  pl->stream), "heat rhs");
    }
    adi_solve(pl, s, pl->E.as<double>(), X);
    Scope sc(pl, PH_PROJ);
    hip_check(launch_apply2(s->blocks.as<BlockDesc>(), static_cast<int>(s->hblocks.size()), g.me[0], g.ne[0],
                            nullptr, 0.0, X, -1.0, 0.0, Pout, pl->atab_proj.as<double>(), 0,
                            pl->ztabA.as<double>(), pl->stream), "project");
}

// ---------------------------------------------------------------------------
// batched heat stepping
// ---------------------------------------------------------------------------
int adi_kind(const cyl_plan_s* pl) {
    return pl->split_gs ? 3 : pl->adi_split ? 0 : (pl->use_lds ? 1 : 2);
}

struct BlockRef {
    BlockDesc b;
    double cost;
    int kind, threads, np, mp;
    int64_t sstride;
};

// Launch groups of one ADI pass.  grouping 0: one launch per (kernel, threads);
// 1: one per (kernel, threads, padded width); 2: one per kernel.  Blocks of a
// launch are sorted by cost (J me ne) so that the dispatcher hands the
// longest blocks out first.
std::vector<BatchLaunch> build_launches(const std::vector<BlockRef>& refs, const BatchCfg& cfg) {
    const int grouping = cfg.grouping;
    std::map<std::tuple<int, int, int>, std::vector<const BlockRef*>> groups;
    for (const auto& r : refs) {
        const std::tuple<int, int, int> key =
            grouping == 0 ? std::make_tuple(r.kind, r.threads, 0)
                          : grouping == 1 ? std::make_tuple(r.kind, r.threads, r.np) : std::make_tuple(r.kind, 0, 0);
        groups[key].push_back(&r);
    }
    auto chunks = [](int x) { return static_cast<size_t>((x + 127) / 128 * 128); };
    std::vector<BatchLaunch> out;
    for (auto& kv : groups) {
        auto& v = kv.second;
        std::stable_sort(v.begin(), v.end(), [](const BlockRef* a, const BlockRef* b) { return a->cost > b->cost; });
        BatchLaunch l;
        l.kind = v.front()->kind;
        int mp = 0;
        for (const BlockRef* r : v) {
            l.threads = std::max(l.threads, r->threads);
            l.np = std::max(l.np, r->np);
            mp = std::max(mp, r->mp);
            l.state_stride = std::max(l.state_stride, r->sstride);
        }
        l.nblocks = static_cast<int>(v.size());
        if (l.kind == 0) {
            l.lds = adi_split_lds_bytes(mp, l.np);
            if (l.lds > 65536) hip_check(adi_split_set_lds_limit(l.np, l.lds), "LDS limit");
        } else if (l.kind == 1) {
            l.lds = (static_cast<size_t>(mp + 4) * (l.np + 1) + chunks(kRRec * mp) + chunks(kZRec * l.np)) * sizeof(double);
            if (l.lds > 65536) hip_check(adi_set_lds_limit(l.np, l.lds), "LDS limit");
        } else if (l.kind == 3) {
            // the kernel's row stride follows the group's np: size every slot
            // for the group's largest mp at that stride
            l.lds = gs_launch_lds(adi_split_gs_lds_bytes(mp, l.np, l.threads / 2, false));
            if (l.lds > 65536) hip_check(adi_split_gs_set_lds_limit(l.np, l.lds), "LDS limit");
            l.state_stride = adi_split_gs_state_stride(mp, l.np);
            l.state = std::make_unique<DevMem>();
            l.state->alloc(static_cast<size_t>(l.nblocks) * l.state_stride * sizeof(double));
        } else {
            l.state = std::make_unique<DevMem>();
            l.state->alloc(static_cast<size_t>(l.nblocks) * l.state_stride * sizeof(double));
        }
        std::vector<BlockDesc> hb;
        hb.reserve(v.size());
        for (const BlockRef* r : v) hb.push_back(r->b);
        const bool g16_ok = cfg.g16 && env_int("CYLSPEC_ADI_G16", 1) != 0;
        l.g16 = l.kind == 0 && g16_ok && std::all_of(hb.begin(), hb.end(), [](const BlockDesc& b) { return adi_split_g16(b); });
        if (l.kind == 3)
            l.g16 = g16_ok && std::all_of(hb.begin(), hb.end(), [](const BlockDesc& b) { return adi_split_gs_z16(b); });
        if (cfg.queue && (l.kind == 0 || l.kind == 3)) {
            l.queue = true;
            hip_check(adi_split_queue_grid(l.np, l.threads, l.lds, l.kind == 3, l.g16, &l.grid), "queue grid");
            l.grid = std::max(1, std::min(l.grid, l.nblocks));
            l.counter = std::make_unique<DevMem>();
            l.counter->alloc(sizeof(double));
            if (l.kind == 3) {      // one state slot per persistent workgroup
                l.state = std::make_unique<DevMem>();
                l.state->alloc(static_cast<size_t>(l.grid) * l.state_stride * sizeof(double));
            }
        }
        l.blocks = std::make_unique<DevMem>();
        upload(*l.blocks, hb);
        out.push_back(std::move(l));
    }
    return out;
}

void run_adi_launches(hipStream_t st, const std::vector<BatchLaunch>& ls, const AdiPtrs* pp, bool acc) {
    for (const auto& l : ls) {
        const BlockDesc* bl = l.blocks->as<BlockDesc>();
        BlockQueue q{nullptr, l.grid};
        if (l.queue) {
            // the counter starts at zero (a fill kernel: capturable, unlike a memset node)
            hip_check(launch_fill_zero(l.counter->as<double>(), 1, st), "queue reset");
            q.counter = l.counter->as<int>();
        }
        if (l.kind == 0)
            hip_check(launch_adi_split(bl, l.nblocks, l.threads, l.np, nullptr, nullptr, nullptr, nullptr, nullptr,
                                       acc, l.lds, st, pp, nullptr, l.g16, l.queue ? &q : nullptr), "batched adi");
        else if (l.kind == 3)
            hip_check(launch_adi_split_gs(bl, l.nblocks, l.threads, l.np, nullptr, nullptr, l.state->as<double>(),
                                          l.state_stride, nullptr, nullptr, nullptr, acc, l.lds, st, pp, nullptr,
                                          l.g16, l.queue ? &q : nullptr),
                      "batched adi");
        else
            hip_check(launch_adi(bl, l.nblocks, l.threads, l.np, nullptr, nullptr,
                                 l.state ? l.state->as<double>() : nullptr, l.state_stride, nullptr, nullptr,
                                 nullptr, acc, l.kind == 1, l.lds, st, pp), "batched adi");
    }
}

// One batched BDF step at cycle position c (enqueue only).
void batch_step_once(cyl_batch_s* B, int c) {
    const int nprob = static_cast<int>(B->heats.size());
    hip_check(launch_heat_rhs_batch(B->rhs_items[c]->as<HeatRhsItem>(), nprob, B->rhs_wg.as<int64_t>(),
                                    B->rhs_nwg, B->stream), "batched heat rhs");
    run_adi_launches(B->stream, B->adi1, B->ptr1.as<AdiPtrs>(), false);
    if (B->n_res > 0) {
        hip_check(launch_apply_batch(B->res_items.as<ApplyItem>(), B->n_res, B->blocks_all.as<BlockDesc>(),
                                     B->res_ptrs.as<ApplyPtrs>(), 1.0, 1.0, 1.0, B->stream), "batched residual");
        run_adi_launches(B->stream, B->adi2, B->ptr2.as<AdiPtrs>(), true);
    }
    hip_check(launch_apply_batch(B->proj_items.as<ApplyItem>(), B->n_proj, B->blocks_all.as<BlockDesc>(),
                                 B->proj_ptrs[c]->as<ApplyPtrs>(), 0.0, -1.0, 0.0, B->stream), "batched projection");
}

// Host bookkeeping of the members after one step.
void batch_advance(cyl_batch_s* B) {
    for (cyl_heat_t h : B->heats) {
        h->head = (h->head + h->order - 1) % h->order;
        ++h->steps;
    }
    B->pos = (B->pos + 1) % B->L;
    ++B->taken;
}

std::mutex g_tune_mutex;
std::map<std::string, std::string> g_tune_cache;   // batch signature -> BatchCfg::str()
bool g_tune_file_read = false;

// The on-disk tuning cache (CYLSPEC_TUNE_CACHE = path; none when unset):
// one "signature<TAB>configuration" line per tuned batch.  Read once per
// process; rewritten whole (temporary file, then rename) when an entry is
// added.  Callers hold g_tune_mutex.
std::string tune_file() {
    const char* f = std::getenv("CYLSPEC_TUNE_CACHE");
    return f ? std::string(f) : std::string();
}
void tune_file_read() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const std::string path = tune_file();
    if (path.empty()) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        BatchCfg c;
        if (tab != std::string::npos && BatchCfg::parse(line.substr(tab + 1), &c))
            g_tune_cache.emplace(line.substr(0, tab), c.str());
    }
}
void tune_file_write() {
    const std::string path = tune_file();
    if (path.empty()) return;
    const std::string tmp = path + ".tmp" + std::to_string(static_cast<long long>(getpid()));
    {
        std::ofstream out(tmp, std::ios::trunc);
        for (const auto& kv : g_tune_cache) out << kv.first << '\t' << kv.second << '\n';
        if (!out) {
            std::remove(tmp.c_str());
            return;       // the cache is an optimisation: an unwritable path only loses it
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

// Time pass-1 ADI launches of candidate configurations on the batch's own
// buffers (the members' states are not touched) and keep the fastest:
// coordinate descent over the launch grouping, then work-queue launches,
// then the 16-row groups (each candidate the best of two runs).
BatchCfg autotune_cfg(cyl_batch_s* B, const std::vector<BlockRef>& refs, const std::string& key) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        tune_file_read();
        auto it = g_tune_cache.find(key);
        BatchCfg c;
        if (it != g_tune_cache.end() && BatchCfg::parse(it->second, &c)) return c;
    }
    const int nprob = static_cast<int>(B->heats.size());
    std::vector<AdiPtrs> tp(nprob);
    for (int q = 0; q < nprob; ++q) {
        Setup* s = B->heats[q]->setup.get();
        tp[q] = AdiPtrs{B->E[q]->as<double>(), B->R[q]->as<double>(), s->rtab.as<double>(), s->ztab.as<double>(),
                        s->vmu.as<double>()};
    }
    DevMem tpd;
    upload(tpd, tp);
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "hipEventCreate");
    hip_check(hipEventCreate(&b), "hipEventCreate");
    auto time_cfg = [&](const BatchCfg& c) {
        const auto ls = build_launches(refs, c);
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            hip_check(hipEventRecord(a, B->stream), "hipEventRecord");
            run_adi_launches(B->stream, ls, tpd.as<AdiPtrs>(), false);
            hip_check(hipEventRecord(b, B->stream), "hipEventRecord");
            hip_check(hipEventSynchronize(b), "hipEventSynchronize");
            float t = 0.0f;
            hip_check(hipEventElapsedTime(&t, a, b), "hipEventElapsedTime");
            ms = std::min(ms, t);
        }
        return ms;
    };
    BatchCfg best;
    float best_ms = time_cfg(best);
    auto consider = [&](BatchCfg c) {
        const float ms = time_cfg(c);
        if (ms < best_ms) { best_ms = ms; best = c; }
    };
    for (int g = 1; g < 3; ++g) { BatchCfg c = best; c.grouping = g; consider(c); }
    { BatchCfg c = best; c.queue = true; consider(c); }
    { BatchCfg c = best; c.g16 = false; consider(c); }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (env_int("CYLSPEC_LOG", 0) > 0)
        std::fprintf(stderr, "[cylspec] batch tuned: %s (pass-1 ADI %.3f ms)\n", best.str().c_str(), best_ms);
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_tune_cache[key] = best.str();
    tune_file_write();
    return best;
}

void batch_build(cyl_batch_s* B, int flags) {
    const int nprob = static_cast<int>(B->heats.size());
    int L = 1;
    for (cyl_heat_t h : B->heats) L = std::max(L, h->order);      // orders are 1 or 4
    B->L = L;
    hip_check(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming), "hipEventCreate");
    hip_check(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming), "hipEventCreate");
    std::vector<BlockRef> refs1, refs2;
    std::vector<BlockDesc> all;
    std::vector<ApplyItem> res_items, proj_items;
    std::vector<AdiPtrs> p1(nprob), p2(nprob);
    std::vector<ApplyPtrs> rp(nprob);
    std::vector<std::vector<ApplyPtrs>> pp(L, std::vector<ApplyPtrs>(nprob));
    std::vector<std::vector<HeatRhsItem>> ri(L, std::vector<HeatRhsItem>(nprob));
    std::vector<int64_t> wg(nprob + 1, 0);
    std::ostringstream key;
    for (int q = 0; q < nprob; ++q) {
        cyl_heat_t h = B->heats[q];
        cyl_plan_s* pl = h->plan;
        const Geometry& g = pl->geo;
        Setup* s = h->setup.get();
        B->E.push_back(std::make_unique<DevMem>());
        B->R.push_back(std::make_unique<DevMem>());
        alloc_elayout(*B->E.back(), g);
        alloc_elayout(*B->R.back(), g);
        double* Eq = B->E.back()->as<double>();
        double* Rq = B->R.back()->as<double>();
        double* Xq = h->Xt.as<double>();
        p1[q] = AdiPtrs{Eq, Xq, s->rtab.as<double>(), s->ztab.as<double>(), s->vmu.as<double>()};
        p2[q] = AdiPtrs{Rq, Xq, s->rtab.as<double>(), s->ztab.as<double>(), s->vmu.as<double>()};
        rp[q] = ApplyPtrs{Eq, Xq, Rq, s->atab.as<double>(), s->ztabA,
                          static_cast<int64_t>(g.me[0] + g.me[1]) * 12, g.me[0], g.ne[0]};
        const int kind = adi_kind(pl);
        const int lines = ((std::max(g.me[0], g.ne[0]) + 63) / 64) * 64;
        const int threads = (kind == 0 || kind == 3) ? 2 * lines : std::min(512, lines);
        const int64_t sstride = kind == 3 ? adi_split_gs_state_stride(g.mp[0], g.np[0])
                                          : static_cast<int64_t>(g.mp[0] + 4) * (g.np[0] + 1);
        key << kind << ':' << g.np[0] << ':' << g.mp[0] << ':' << s->hblocks.size() << ':' << s->passes << ';';
        for (const BlockDesc& b0 : s->hblocks) {
            BlockDesc b = b0;
            b.prob = q;
            const int bi = static_cast<int>(all.size());
            all.push_back(b);
            BlockRef r{b, static_cast<double>(b.J) * b.me * b.ne, kind, threads, g.np[0], g.mp[0], sstride};
            refs1.push_back(r);
            if (s->passes == 2) refs2.push_back(r);
            for (int ti = 0; ti * 32 < b.me; ++ti)
                for (int tk = 0; tk * 32 < b.ne; ++tk) {
                    proj_items.push_back(ApplyItem{bi, ti, tk, 0});
                    if (s->passes == 2) res_items.push_back(ApplyItem{bi, ti, tk, 0});
                }
        }
        // cycle tables: the head moves down by one (mod order) every step
        for (int c = 0; c < L; ++c) {
            const int hc = ((h->head - c) % h->order + h->order) % h->order;
            HeatRhsItem it{};
            it.E = Eq;
            for (int i = 0; i < h->order; ++i) {
                it.P[i] = h->P[(hc + i) % h->order].as<double>();
                it.beta[i] = h->beta[i];
            }
            it.nb = h->order;
            it.Ec = h->Econst.as<double>();
            it.total = g.etotal_elems;
            ri[c][q] = it;
            const int slot = (hc + h->order - 1) % h->order;
            pp[c][q] = ApplyPtrs{nullptr, Xq, h->P[slot].as<double>(), pl->atab_proj.as<double>(),
                                 pl->ztabA.as<double>(), 0, g.me[0], g.ne[0]};
        }
        wg[q + 1] = wg[q] + (g.etotal_elems + 1023) / 1024;
        B->head0.push_back(h->head);
        B->steps0.push_back(h->steps);
    }
    B->rhs_nwg = wg[nprob];
    upload(B->rhs_wg, wg);
    for (int c = 0; c < L; ++c) {
        B->rhs_items.push_back(std::make_unique<DevMem>());
        upload(*B->rhs_items.back(), ri[c]);
        B->proj_ptrs.push_back(std::make_unique<DevMem>());
        upload(*B->proj_ptrs.back(), pp[c]);
    }
    upload(B->ptr1, p1);
    upload(B->ptr2, p2);
    upload(B->res_ptrs, rp);
    upload(B->blocks_all, all);
    upload(B->res_items, res_items);
    upload(B->proj_items, proj_items);
    B->n_res = static_cast<int>(res_items.size());
    B->n_proj = static_cast<int>(proj_items.size());
    // launch configuration: tuned (cached per batch signature, in the process
    // and in CYLSPEC_TUNE_CACHE), or the default; CYLSPEC_BATCH_GROUPING and
    // CYLSPEC_BATCH_QUEUE fix those parts
    BatchCfg cfg;
    const int fg = env_int("CYLSPEC_BATCH_GROUPING", -1), fq = env_int("CYLSPEC_BATCH_QUEUE", -1);
    if (!(flags & CYL_BATCH_NO_TUNE) && (fg < 0 || fg > 2 || fq < 0)) {
        int dev = 0;
        hipDeviceProp_t prop;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        cfg = autotune_cfg(B, refs1, std::string(prop.gcnArchName) + "/" +
                                         std::to_string(prop.multiProcessorCount) + "|" + key.str());
    }
    if (fg >= 0 && fg <= 2) cfg.grouping = fg;
    if (fq >= 0) cfg.queue = fq != 0;
    static const char* names[3] = {"per kernel and thread count", "per kernel, thread count and width",
                                   "per kernel"};
    B->grouping = std::string(names[cfg.grouping]) + (cfg.queue ? ", work-queue launches" : "") +
                  (cfg.g16 ? "" : ", 8-row groups");
    B->adi1 = build_launches(refs1, cfg);
    if (!refs2.empty()) B->adi2 = build_launches(refs2, cfg);
    B->use_graph = (flags & CYL_BATCH_NO_GRAPH) == 0;
    if (B->use_graph) {
        hip_check(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        for (int c = 0; c < L; ++c) batch_step_once(B, c);
        hip_check(hipStreamEndCapture(B->stream, &B->graph), "hipStreamEndCapture");
        hip_check(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
}

// The Poisson solve of Section 3 (eq. HelmholtzMatEqn without time terms) on
// workspace w: forward transforms, tau right side, ADI (and the residual
// correction), optional residual check, recombination, inverse transform.
// Per-phase times of one solve for cyl_solve_info: the solve's phases are
// recorded (as when profiling) and read back after the stream has finished;
// the records stay for cyl_plan_get_profile only if profiling was on.
struct PhaseTimer {
    cyl_plan_t pl;
    cyl_solve_info* info;
    bool was = false;
    size_t rec0 = 0;
    PhaseTimer(cyl_plan_t p, cyl_solve_info* i) : pl(p), info(i) {
        if (!info) return;
        was = pl->profiling;
        rec0 = pl->recs.size();
        pl->profiling = true;
    }
    void finish() {
        if (!info) return;
        pl->profiling = was;
        hip_check(hipStreamSynchronize(pl->stream), "sync");
        double ms[PH_COUNT] = {0};
        for (size_t i = rec0; i < pl->recs.size(); ++i) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, pl->recs[i].a, pl->recs[i].b) == hipSuccess) ms[pl->recs[i].phase] += t;
        }
        drop();
        info->ms_transform = ms[PH_FWD];
        info->ms_rhs = ms[PH_RHS];
        info->ms_adi = ms[PH_ADI] + ms[PH_RES];
        info->ms_inverse = ms[PH_REC] + ms[PH_INV];
        info = nullptr;
    }
    void drop() {
        if (was) return;
        for (size_t i = rec0; i < pl->recs.size(); ++i) {
            (void)hipEventDestroy(pl->recs[i].a);
            (void)hipEventDestroy(pl->recs[i].b);
        }
        pl->recs.resize(rec0);
    }
    ~PhaseTimer() {           // an error left the solve: restore the flag
        if (!info) return;
        pl->profiling = was;
        (void)hipStreamSynchronize(pl->stream);
        drop();
    }
};

void poisson_run(cyl_plan_t pl, Setup* s, int space, const double* f, const double* bc_lift, double* u,
                 double adi_tol, cyl_solve_info* info, const Work& w) {
    PhaseTimer timer(pl, info);
    const Geometry& g = pl->geo;
    const double2* F = reinterpret_cast<const double2*>(f);
    const double2* Lc = reinterpret_cast<const double2*>(bc_lift);
    if (space == CYL_SPACE_VALUE) {
        transform_fwd(pl, f, w.planesA);
        F = w.planesA;
        if (bc_lift) {
            transform_fwd(pl, bc_lift, w.planesB);
            Lc = w.planesB;
        }
    }
    {
        Scope sc(pl, PH_RHS);
        hip_check(launch_rhs3(F, Lc, 1.0, 0.0, -1.0, w.E, s->blocks.as<BlockDesc>(),
                              pl->plane_of.as<int>(), g.nw, g.m, g.n, pl->rhs, pl->stream), "rhs");
    }
    if (pl->physical)
        hip_check(launch_zero_blocks(s->blocks_skip.as<BlockDesc>(), s->n_skip, g.me[0], g.ne[0], w.X,
                                     pl->stream), "zero blocks");
    adi_solve(pl, s, w.E, w.X, pl->physical, w.R, w.state);
    if (env_int("CYLSPEC_LOG", 0) >= 2)
        std::fprintf(stderr, "[cylspec] poisson %dx%dx%d tol %.3g: %d blocks, J %d..%d (mean %.2f), %d pass(es)%s%s\n",
                     pl->m, pl->n, pl->p, adi_tol, pl->physical ? s->n_phys : static_cast<int>(s->hblocks.size()),
                     s->h.J_min, s->h.J_max, s->h.J_mean, s->passes,
                     fuse_residual(pl, s, pl->physical) ? ", residual formed by the first pass" : "",
                     w.E == pl->E.as<double>() ? "" : ", static scratch");
    if (info) check_residual(pl, s, w.E, w.X, w.R, w.acc, adi_tol, info);
    double2* out = space == CYL_SPACE_COEFF ? reinterpret_cast<double2*>(u) : w.planesA;
    {
        Scope sc(pl, PH_REC);
        hip_check(launch_recombine(w.X, Lc, out, pl->plane_of.as<int>(), s->blocks.as<BlockDesc>(), g.nw,
                                   g.m, g.n, g.p, pl->stream), "recombine");
    }
    if (space == CYL_SPACE_VALUE) transform_inv(pl, w.planesA, u, w.planesA);
    timer.finish();
}

double* ckpt_slot(cyl_heat_grad_s* a, int j) { return a->ckpt.as<double>() + j * a->ck_stride; }
double* seg_slot(cyl_heat_grad_s* a, int t) { return a->seg.as<double>() + t * a->heat->plan->geo.total_elems; }

}  // namespace
}  // namespace cyl

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

const char* cyl_status_string(int status) {
    switch (status) {
        case CYL_OK: return "ok";
        case CYL_E_INVALID_ARG: return "invalid argument";
        case CYL_E_UNSUPPORTED: return "unsupported size or option";
        case CYL_E_OUT_OF_MEMORY: return "out of memory";
        case CYL_E_HIP: return "HIP runtime error";
        case CYL_E_NOT_CONVERGED: return "ADI did not converge";
        case CYL_E_INTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* cyl_last_error(void) { return g_last_error.c_str(); }

int cyl_plan_create(cyl_plan_t* plan, int n_r, int n_z, int n_theta, void* hip_stream) {
    return guarded([&] {
        if (!plan) fail(CYL_E_INVALID_ARG, "plan pointer is NULL");
        *plan = nullptr;
        if (n_r < 4 || n_z < 4 || n_theta < 1) fail(CYL_E_INVALID_ARG, "need n_r >= 4, n_z >= 4, n_theta >= 1");
        if (n_r > 1025 || n_z > 1025 || n_theta > 4096) fail(CYL_E_UNSUPPORTED, "need n_r, n_z <= 1025 and n_theta <= 4096");
        auto nb_of = [](int L) { if ((L & (L - 1)) == 0) return L; int N = 1; while (N < 2 * L - 1) N <<= 1; return N; };
        if (nb_of(n_theta) > 4096) fail(CYL_E_UNSUPPORTED, "n_theta that is not a power of two must be <= 2048");
        auto pl = std::make_unique<cyl_plan_s>();
        pl->m = n_r; pl->n = n_z; pl->p = n_theta;
        pl->stream = static_cast<hipStream_t>(hip_stream);
        build_plan(pl.get());
        *plan = pl.release();
    });
}

int cyl_plan_destroy(cyl_plan_t plan) {
    return guarded([&] {
        if (!plan) fail(CYL_E_INVALID_ARG, "plan is NULL");
        (void)hipStreamSynchronize(plan->stream);
        for (auto& r : plan->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        delete plan;
    });
}

int cyl_transform_fwd(cyl_plan_t plan, const double* values, double* coeffs) {
    return guarded([&] {
        if (!plan || !values || !coeffs) fail(CYL_E_INVALID_ARG, "NULL argument");
        transform_fwd(plan, values, reinterpret_cast<double2*>(coeffs));
    });
}

int cyl_transform_inv(cyl_plan_t plan, const double* coeffs, double* values) {
    return guarded([&] {
        if (!plan || !values || !coeffs) fail(CYL_E_INVALID_ARG, "NULL argument");
        transform_inv(plan, reinterpret_cast<const double2*>(coeffs), values);
    });
}

int cyl_plan_prepare(cyl_plan_t plan, double adi_tol) {
    return guarded([&] {
        if (!plan) fail(CYL_E_INVALID_ARG, "plan is NULL");
        validate_tol(adi_tol);
        (void)poisson_setup(plan, adi_tol, true);
    });
}

int cyl_poisson_solve(cyl_plan_t plan, int space, const double* f, const double* bc_lift, double* u,
                      double adi_tol, cyl_solve_info* info) {
    return guarded([&] {
        if (!plan || !f || !u) fail(CYL_E_INVALID_ARG, "NULL argument");
        validate_space(space);
        validate_tol(adi_tol);
        poisson_run(plan, poisson_setup(plan, adi_tol, false), space, f, bc_lift, u, adi_tol, info,
                    plan_work(plan));
    });
}

int cyl_poisson_solve_noalloc(cyl_plan_t plan, int space, const double* f, const double* bc_lift, double* u,
                              double adi_tol, cyl_solve_info* info) {
    return guarded([&] {
        if (!plan || !f || !u) fail(CYL_E_INVALID_ARG, "NULL argument");
        validate_space(space);
        validate_tol(adi_tol);
        cyl_plan_s* pl = plan;
        Setup* s = poisson_setup(pl, adi_tol, false);
        const Geometry& g = pl->geo;
        const size_t planes_bytes = static_cast<size_t>(g.nw) * g.n * g.m * sizeof(double2);
        const size_t e_bytes = (static_cast<size_t>(g.etotal_elems) + 64) * sizeof(double);
        const size_t x_bytes = static_cast<size_t>(g.total_elems) * sizeof(double);
        auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t need = up(planes_bytes) * (bc_lift ? 2 : 1) + 2 * up(e_bytes) + up(x_bytes) +
                            up(4 * sizeof(double)) + up(pl->state.bytes);
        if (need > kScratchBytes) {
            char buf[200];
            std::snprintf(buf, sizeof(buf), "a %dx%dx%d solve needs %zu bytes of workspace; the static scratch of "
                                            "cyl_poisson_solve_noalloc holds %zu",
                          pl->m, pl->n, pl->p, need, kScratchBytes);
            fail(CYL_E_UNSUPPORTED, buf);
        }
        char* base = static_cast<char*>(scratch_device_ptr(pl->device));
        if (!base) fail(CYL_E_INTERNAL, "static scratch address not initialised");
        Work w;
        size_t off = 0;
        auto take = [&](size_t b) { char* q = base + off; off += up(b); return q; };
        w.planesA = reinterpret_cast<double2*>(take(planes_bytes));
        if (bc_lift) w.planesB = reinterpret_cast<double2*>(take(planes_bytes));
        w.E = reinterpret_cast<double*>(take(e_bytes));
        w.R = reinterpret_cast<double*>(take(e_bytes));
        w.X = reinterpret_cast<double*>(take(x_bytes));
        w.acc = reinterpret_cast<double*>(take(4 * sizeof(double)));
        if (pl->state.bytes) w.state = reinterpret_cast<double*>(take(pl->state.bytes));
        // the scratch keeps the previous call's contents: the E-layout padding
        // rows (read by the sweeps, never written) must start at zero
        hip_check(launch_fill_zero(w.E, static_cast<int64_t>(e_bytes / sizeof(double)), pl->stream), "clear E");
        hip_check(launch_fill_zero(w.R, static_cast<int64_t>(e_bytes / sizeof(double)), pl->stream), "clear R");
        poisson_run(pl, s, space, f, bc_lift, u, adi_tol, info, w);
    });
}

int cyl_heat_create(cyl_heat_t* h, cyl_plan_t plan, double alpha, double dt, int bdf_order,
                    double adi_tol, int space, const double* const* history, const double* g,
                    const double* bc_lift) {
    return guarded([&] {
        if (!h) fail(CYL_E_INVALID_ARG, "heat handle pointer is NULL");
        *h = nullptr;
        if (!plan || !history || !g) fail(CYL_E_INVALID_ARG, "NULL argument");
        if (!(alpha > 0.0) || !std::isfinite(alpha)) fail(CYL_E_INVALID_ARG, "alpha must be > 0");
        if (!(dt > 0.0) || !std::isfinite(dt)) fail(CYL_E_INVALID_ARG, "dt must be > 0");
        if (bdf_order != 1 && bdf_order != 4) fail(CYL_E_UNSUPPORTED, "bdf_order must be 1 or 4");
        validate_space(space);
        validate_tol(adi_tol);
        for (int i = 0; i < bdf_order; ++i)
            if (!history[i]) fail(CYL_E_INVALID_ARG, "NULL history level");
        cyl_plan_s* pl = plan;
        const Geometry& geo = pl->geo;
        auto H = std::make_unique<cyl_heat_s>();
        H->plan = pl;
        H->stream = pl->stream;
        H->alpha = alpha; H->dt = dt; H->order = bdf_order; H->tol = adi_tol;
        if (bdf_order == 1) { H->kappa = dt; H->beta[0] = 1.0; }
        else {
            H->kappa = 12.0 * dt / 25.0;
            H->beta[0] = 48.0 / 25.0; H->beta[1] = -36.0 / 25.0; H->beta[2] = 16.0 / 25.0; H->beta[3] = -3.0 / 25.0;
        }
        const double ka = H->kappa * alpha;
        H->setup = make_setup(pl, ka, adi_tol);
        const size_t blk_bytes = static_cast<size_t>(geo.total_elems) * sizeof(double);
        const size_t planes_bytes = static_cast<size_t>(geo.nw) * geo.n * geo.m * sizeof(double2);
        for (int i = 0; i < bdf_order; ++i) alloc_elayout(H->P[i], geo);
        alloc_elayout(H->Econst, geo);
        H->Xt.alloc(blk_bytes);
        H->T0.alloc(planes_bytes);
        const BlockDesc* blocks = H->setup->blocks.as<BlockDesc>();
        const double2* Lc = nullptr;
        if (bc_lift) {
            H->lift.alloc(planes_bytes);
            H->has_lift = true;
            if (space == CYL_SPACE_VALUE) transform_fwd(pl, bc_lift, H->lift.as<double2>());
            else hip_check(hipMemcpyAsync(H->lift.p, bc_lift, planes_bytes, hipMemcpyDeviceToDevice, pl->stream), "copy lift");
            Lc = H->lift.as<double2>();
        }
        // history levels -> P_i = [R2 (T_i - L) C02^T]_tau
        for (int i = 0; i < bdf_order; ++i) {
            const double2* C;
            if (space == CYL_SPACE_VALUE) {
                double2* dst = (i == 0) ? H->T0.as<double2>() : pl->planesA.as<double2>();
                transform_fwd(pl, history[i], dst);
                C = dst;
            } else {
                if (i == 0) hip_check(hipMemcpyAsync(H->T0.p, history[0], planes_bytes, hipMemcpyDeviceToDevice, pl->stream), "copy T0");
                C = reinterpret_cast<const double2*>(history[i]);
            }
            Scope sc(pl, PH_RHS);
            hip_check(launch_rhs3(C, Lc, 1.0, -1.0, 0.0, H->P[i].as<double>(), blocks, pl->plane_of.as<int>(),
                                  geo.nw, geo.m, geo.n, pl->rhs, pl->stream), "history rhs");
        }
        // constant part: kappa [R2 G C02^T]_tau + kappa alpha [r^2 nabla^2 L]_tau
        const double2* G;
        if (space == CYL_SPACE_VALUE) {
            transform_fwd(pl, g, pl->planesA.as<double2>());
            G = pl->planesA.as<double2>();
        } else {
            G = reinterpret_cast<const double2*>(g);
        }
        {
            Scope sc(pl, PH_RHS);
            hip_check(launch_rhs3(G, Lc, H->kappa, 0.0, ka, H->Econst.as<double>(), blocks,
                                  pl->plane_of.as<int>(), geo.nw, geo.m, geo.n, pl->rhs, pl->stream),
                      "forcing rhs");
        }
        H->physical = pl->physical;
        if (H->physical)      // the skipped blocks' solutions are never written: zero them once
            hip_check(launch_zero_blocks(H->setup->blocks_skip.as<BlockDesc>(), H->setup->n_skip, geo.me[0],
                                         geo.ne[0], H->Xt.as<double>(), pl->stream), "zero blocks");
        H->head = 0;
        *h = H.release();
    });
}

int cyl_heat_step(cyl_heat_t h, int n_steps) {
    return guarded([&] {
        if (!h) fail(CYL_E_INVALID_ARG, "heat handle is NULL");
        if (n_steps < 0) fail(CYL_E_INVALID_ARG, "n_steps must be >= 0");
        cyl_plan_s* pl = h->plan;
        const Geometry& g = pl->geo;
        Setup* s = h->setup.get();
        const int nblk = h->physical ? s->n_phys : static_cast<int>(s->hblocks.size());
        const BlockDesc* blocks = (h->physical ? s->blocks_phys : s->blocks).as<BlockDesc>();
        for (int st = 0; st < n_steps; ++st) {
            const double* P[4];
            for (int i = 0; i < h->order; ++i) P[i] = h->P[(h->head + i) % h->order].as<double>();
            {
                Scope sc(pl, PH_HRHS);
                hip_check(launch_heat_rhs(pl->E.as<double>(), P, h->beta, h->order, h->Econst.as<double>(),
                                          g.etotal_elems, pl->stream), "heat rhs");
            }
            adi_solve(pl, s, pl->E.as<double>(), h->Xt.as<double>(), h->physical);
            if (env_int("CYLSPEC_LOG", 0) >= 2)
                std::fprintf(stderr, "[cylspec] heat step %lld of %dx%dx%d: %d blocks, J %d..%d, %d pass(es)\n",
                             h->steps + 1, pl->m, pl->n, pl->p, nblk, s->h.J_min, s->h.J_max, s->passes);
            // the oldest slot becomes the newest: P_new = C~ Xt B~
            const int slot = (h->head + h->order - 1) % h->order;
            {
                Scope sc(pl, PH_PROJ);
                hip_check(launch_apply2(blocks, nblk, g.me[0], g.ne[0], nullptr, 0.0,
                                        h->Xt.as<double>(), -1.0, 0.0, h->P[slot].as<double>(),
                                        pl->atab_proj.as<double>(), 0, pl->ztabA.as<double>(),
                                        pl->stream), "project");
            }
            h->head = slot;
            ++h->steps;
        }
    });
}

int cyl_heat_read(cyl_heat_t h, int space, double* T_out) {
    return guarded([&] {
        if (!h || !T_out) fail(CYL_E_INVALID_ARG, "NULL argument");
        validate_space(space);
        cyl_plan_s* pl = h->plan;
        const Geometry& g = pl->geo;
        const size_t planes_bytes = static_cast<size_t>(g.nw) * g.n * g.m * sizeof(double2);
        if (h->steps == 0) {
            if (space == CYL_SPACE_COEFF)
                hip_check(hipMemcpyAsync(T_out, h->T0.p, planes_bytes, hipMemcpyDeviceToDevice, pl->stream), "copy");
            else
                transform_inv(pl, h->T0.as<double2>(), T_out);
            return;
        }
        double2* out = space == CYL_SPACE_COEFF ? reinterpret_cast<double2*>(T_out) : pl->planesA.as<double2>();
        {
            Scope sc(pl, PH_REC);
            hip_check(launch_recombine(h->Xt.as<double>(), h->has_lift ? h->lift.as<double2>() : nullptr, out,
                                       pl->plane_of.as<int>(), h->setup->blocks.as<BlockDesc>(), g.nw, g.m, g.n,
                                       g.p, pl->stream), "recombine");
        }
        if (space == CYL_SPACE_VALUE) transform_inv(pl, pl->planesA.as<double2>(), T_out);
    });
}

int cyl_heat_destroy(cyl_heat_t h) {
    return guarded([&] {
        if (!h) fail(CYL_E_INVALID_ARG, "heat handle is NULL");
        (void)hipStreamSynchronize(h->stream);
        delete h;
    });
}

int cyl_adi_parameters(int n_r, int n_z, int w, double kappa_alpha, double adi_tol, double* bounds4,
                       int* J, double* u, double* v, int cap) {
    return guarded([&] {
        if (n_r < 4 || n_z < 4 || w < 0 || kappa_alpha < 0.0 || !bounds4 || !J)
            fail(CYL_E_INVALID_ARG, "invalid argument");
        if (n_r > 1025 || n_z > 1025) fail(CYL_E_UNSUPPORTED, "n_r, n_z <= 1025");
        validate_tol(adi_tol);
        const DirOps r = build_dir_ops(n_r), z = build_dir_ops(n_z);
        double zc, zd;
        pencil_bounds_z(band_transpose(z.C02Q), band_transpose(z.D2Q), &zc, &zd);
        std::vector<double> uu, vv;
        mode_parameters(r, z, w, kappa_alpha, adi_tol, zc, zd, bounds4, J, &uu, &vv);
        if (u && v) {
            if (cap < *J) fail(CYL_E_INVALID_ARG, "shift capacity smaller than J");
            std::copy(uu.begin(), uu.end(), u);
            std::copy(vv.begin(), vv.end(), v);
        }
    });
}

int cyl_disk_poisson_solve(cyl_plan_t plan, int space, const double* f, double* u) {
    return guarded([&] {
        if (!plan || !f || !u) fail(CYL_E_INVALID_ARG, "NULL argument");
        validate_space(space);
        if (space == CYL_SPACE_COEFF && f == u) fail(CYL_E_INVALID_ARG, "u must not alias f in coefficient space");
        cyl_plan_s* pl = plan;
        const Geometry& g = pl->geo;
        const DiskTables& t = *pl->disk;
        const double2* F = reinterpret_cast<const double2*>(f);
        double2* U = reinterpret_cast<double2*>(u);
        if (space == CYL_SPACE_VALUE) {
            transform_fwd(pl, f, pl->planesA.as<double2>());
            F = pl->planesA.as<double2>();
            U = pl->planesB.as<double2>();
        }
        {
            Scope sc(pl, PH_ADI);
            hip_check(launch_disk(F, U, pl->disk_lu.as<double>(), pl->disk_taps.as<double>(), g.m, g.n, g.nw,
                                  t.rmax, t.rows[0], t.rows[1], pl->stream),
                      "disk solve");
        }
        if (space == CYL_SPACE_VALUE) transform_inv(pl, pl->planesB.as<double2>(), u);
    });
}

int cyl_pt_decompose(cyl_plan_t plan, int space, const double* v_r, const double* v_theta,
                     const double* v_z, double* lambda, double* gamma) {
    return guarded([&] {
        if (!plan || !v_r || !v_theta || !v_z || !lambda || !gamma) fail(CYL_E_INVALID_ARG, "NULL argument");
        validate_space(space);
        if (lambda == gamma) fail(CYL_E_INVALID_ARG, "lambda and gamma must be different arrays");
        if (space == CYL_SPACE_COEFF)
            for (const double* out : {static_cast<const double*>(lambda), static_cast<const double*>(gamma)})
                if (out == v_r || out == v_theta || out == v_z)
                    fail(CYL_E_INVALID_ARG, "in coefficient space lambda and gamma must not alias an input");
        cyl_plan_s* pl = plan;
        const Geometry& g = pl->geo;
        const DiskTables& t = *pl->disk;
        const int wnyq = g.p % 2 == 0 ? g.p / 2 : -1;
        auto disk = [&](const double2* F, double2* U) {
            Scope sc(pl, PH_ADI);
            hip_check(launch_disk(F, U, pl->disk_lu.as<double>(), pl->disk_taps.as<double>(), g.m, g.n, g.nw,
                                  t.rmax, t.rows[0], t.rows[1], pl->stream, -1.0),
                      "disk solve (gamma)");
        };
        auto curl = [&](const double2* Vt, const double2* Vr, double2* U) {
            Scope sc(pl, PH_ADI);
            hip_check(launch_disk_pt(Vt, Vr, U, pl->disk_lu.as<double>(), pl->disk_pt_taps.as<double>(), g.m, g.n,
                                     g.nw, t.rmax, t.rows[0], t.rows[1], wnyq, pl->stream),
                      "disk solve (lambda)");
        };
        if (space == CYL_SPACE_COEFF) {
            disk(reinterpret_cast<const double2*>(v_z), reinterpret_cast<double2*>(gamma));
            curl(reinterpret_cast<const double2*>(v_theta), reinterpret_cast<const double2*>(v_r),
                 reinterpret_cast<double2*>(lambda));
            return;
        }
        double2* A = pl->planesA.as<double2>();
        double2* B = pl->planesB.as<double2>();
        double2* C = pl->planesC.as<double2>();
        // every input is read before an output is written (outputs may alias inputs)
        transform_fwd(pl, v_r, A);
        transform_fwd(pl, v_theta, B);
        curl(B, A, C);
        transform_fwd(pl, v_z, A);
        disk(A, B);
        transform_inv(pl, B, gamma, B);
        transform_inv(pl, C, lambda, C);
    });
}

int cyl_device_peaks(void* hip_stream, const double* src, double* dst, int64_t n, int reps,
                     double* fp64_tflops, double* copy_gbs) {
    return guarded([&] {
        if (reps < 1 || reps > 1000) fail(CYL_E_INVALID_ARG, "reps must lie in [1, 1000]");
        if (copy_gbs) {
            if (!src || !dst || n <= 0) fail(CYL_E_INVALID_ARG, "the copy needs src, dst and n > 0");
            if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
                fail(CYL_E_INVALID_ARG, "src and dst must be 16-byte aligned");
            if (src < dst + n && dst < src + n) fail(CYL_E_INVALID_ARG, "src and dst overlap");
        }
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        int dev = 0, cus = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
        struct Events {
            hipEvent_t a = nullptr, b = nullptr;
            ~Events() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } ev;
        hip_check(hipEventCreate(&ev.a), "event");
        hip_check(hipEventCreate(&ev.b), "event");
        // one warm-up launch, then the fastest of reps timed launches (ms)
        auto best_ms = [&](auto&& launch) {
            launch();
            float best = 0.0f;
            for (int r = 0; r < reps; ++r) {
                hip_check(hipEventRecord(ev.a, s), "event record");
                launch();
                hip_check(hipEventRecord(ev.b, s), "event record");
                hip_check(hipEventSynchronize(ev.b), "event sync");
                float ms = 0.0f;
                hip_check(hipEventElapsedTime(&ms, ev.a, ev.b), "elapsed");
                if (r == 0 || ms < best) best = ms;
            }
            return static_cast<double>(best);
        };
        if (fp64_tflops) {
            double flops = 0.0;
            const double ms = best_ms([&] {
                hip_check(launch_fma_peak(dst, 8 * cus, 4096, s, &flops), "fma peak");
            });
            *fp64_tflops = flops / (ms * 1e-3) / 1e12;
        }
        if (copy_gbs) {
            const double ms = best_ms([&] {
                hip_check(launch_copy_peak(src, dst, n, 16 * cus, s), "copy peak");
            });
            *copy_gbs = 2.0 * 8.0 * static_cast<double>(n) / (ms * 1e-3) / 1e9;
        }
    });
}

int cyl_plan_set_physical(cyl_plan_t plan, int enable) {
    return guarded([&] {
        if (!plan) fail(CYL_E_INVALID_ARG, "plan is NULL");
        if (enable && plan->p % 2 != 0)
            fail(CYL_E_UNSUPPORTED, "physical parity needs an even n_theta (theta + pi on the grid)");
        plan->physical = enable != 0;
    });
}

int cyl_trace_lift(cyl_plan_t plan, const double* rface, const double* zface, double* lift) {
    return guarded([&] {
        if (!plan || !rface || !zface || !lift) fail(CYL_E_INVALID_ARG, "NULL argument");
        hip_check(launch_trace_lift(rface, zface, plan->lift_ra.as<double>(), plan->lift_zb.as<double>(), lift,
                                    plan->m, plan->n, plan->p, plan->stream),
                  "trace lift");
    });
}

int cyl_plan_set_profiling(cyl_plan_t plan, int enable) {
    return guarded([&] {
        if (!plan) fail(CYL_E_INVALID_ARG, "plan is NULL");
        plan->profiling = enable != 0;
    });
}

int cyl_plan_get_profile(cyl_plan_t plan, cyl_profile* out) {
    return guarded([&] {
        if (!plan || !out) fail(CYL_E_INVALID_ARG, "NULL argument");
        hip_check(hipStreamSynchronize(plan->stream), "sync");
        double ms[PH_COUNT] = {0};
        int cnt[PH_COUNT] = {0};
        for (auto& r : plan->recs) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) { ms[r.phase] += t; cnt[r.phase] += 1; }
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        plan->recs.clear();
        out->ms_transform_fwd = ms[PH_FWD]; out->n_transform_fwd = cnt[PH_FWD];
        out->ms_rhs = ms[PH_RHS]; out->n_rhs = cnt[PH_RHS];
        out->ms_adi = ms[PH_ADI]; out->n_adi = cnt[PH_ADI];
        out->ms_residual = ms[PH_RES]; out->n_residual = cnt[PH_RES];
        out->ms_recombine = ms[PH_REC]; out->n_recombine = cnt[PH_REC];
        out->ms_transform_inv = ms[PH_INV]; out->n_transform_inv = cnt[PH_INV];
        out->ms_heat_rhs = ms[PH_HRHS]; out->n_heat_rhs = cnt[PH_HRHS];
        out->ms_project = ms[PH_PROJ]; out->n_project = cnt[PH_PROJ];
        out->ms_adjoint = ms[PH_ADJ]; out->n_adjoint = cnt[PH_ADJ];
    });
}

int cyl_transform_fwd_adjoint(cyl_plan_t plan, const double* coeffs_bar, double* values_bar) {
    return guarded([&] {
        if (!plan || !coeffs_bar || !values_bar) fail(CYL_E_INVALID_ARG, "NULL argument");
        const Geometry& g = plan->geo;
        const size_t bytes = static_cast<size_t>(g.nw) * g.n * g.m * sizeof(double2);
        hip_check(hipMemcpyAsync(plan->planesB.p, coeffs_bar, bytes, hipMemcpyDeviceToDevice, plan->stream), "copy");
        transform_fwd_adjoint(plan, plan->planesB.as<double2>(), values_bar);
    });
}

int cyl_transform_inv_adjoint(cyl_plan_t plan, const double* values_bar, double* coeffs_bar) {
    return guarded([&] {
        if (!plan || !coeffs_bar || !values_bar) fail(CYL_E_INVALID_ARG, "NULL argument");
        // planesA holds (p/2 + 1) n m complex >= p n m doubles: room for the scaled values
        transform_inv_adjoint(plan, values_bar, plan->planesA.as<double>(), reinterpret_cast<double2*>(coeffs_bar));
    });
}

int cyl_heat_grad_create(cyl_heat_grad_t* out, cyl_heat_t h, int n_steps, int checkpoint_every) {
    return guarded([&] {
        if (!out) fail(CYL_E_INVALID_ARG, "handle pointer is NULL");
        *out = nullptr;
        if (!h) fail(CYL_E_INVALID_ARG, "heat handle is NULL");
        if (n_steps < 1) fail(CYL_E_INVALID_ARG, "n_steps must be >= 1");
        if (checkpoint_every < 1) fail(CYL_E_INVALID_ARG, "checkpoint_every must be >= 1");
        if (h->order != 1) fail(CYL_E_UNSUPPORTED, "differentiation supports BDF1 only");
        if (h->has_lift) fail(CYL_E_UNSUPPORTED, "differentiation supports homogeneous Dirichlet data only");
        if (h->physical) fail(CYL_E_UNSUPPORTED, "differentiation solves all parity blocks (physical heat handle)");
        cyl_plan_s* pl = h->plan;
        const Geometry& g = pl->geo;
        auto a = std::make_unique<cyl_heat_grad_s>();
        a->heat = h;
        a->stream = pl->stream;
        a->steps = n_steps;
        a->every = std::min(checkpoint_every, n_steps);
        a->nseg = (n_steps + a->every - 1) / a->every;
        a->adj = make_setup(pl, h->kappa * h->alpha, h->tol, true);
        upload(a->atab_pois, apply_rows(pl, 0.0, false));
        upload(a->proj_flip, projection_rows(pl, true));
        // checkpoints: E-layout slots, zero padding rows
        a->ck_stride = g.etotal_elems + 64;
        const size_t ck_bytes = static_cast<size_t>(a->nseg) * a->ck_stride * sizeof(double);
        a->ckpt.alloc(ck_bytes);
        hip_check(hipMemset(a->ckpt.p, 0, ck_bytes), "hipMemset");
        a->seg.alloc(static_cast<size_t>(a->every) * g.total_elems * sizeof(double));
        alloc_elayout(a->Pw, g);
        alloc_elayout(a->Xh, g);
        a->Et.alloc(static_cast<size_t>(g.total_elems) * sizeof(double));
        a->Gsum.alloc(static_cast<size_t>(g.total_elems) * sizeof(double));
        a->n_partials = apply_dot_partials(static_cast<int>(a->adj->hblocks.size()), g.me[0], g.ne[0]);
        a->partials.alloc(static_cast<size_t>(a->n_partials) * sizeof(double));
        a->planes.alloc(static_cast<size_t>(g.nw) * g.n * g.m * sizeof(double2));
        a->vals.alloc(static_cast<size_t>(g.p) * g.n * g.m * sizeof(double));
        *out = a.release();
    });
}

int cyl_heat_grad_forward(cyl_heat_grad_t a) {
    return guarded([&] {
        if (!a) fail(CYL_E_INVALID_ARG, "handle is NULL");
        cyl_heat_t h = a->heat;
        cyl_plan_s* pl = h->plan;
        const Geometry& g = pl->geo;
        const int N = a->steps, K = a->every, s_last = (a->nseg - 1) * K;
        // P_0 = [R2 T_0 C02^T]_tau from the handle's initial temperature
        {
            Scope sc(pl, PH_RHS);
            hip_check(launch_rhs3(h->T0.as<double2>(), nullptr, 1.0, 0.0, 0.0, ckpt_slot(a, 0),
                                  h->setup->blocks.as<BlockDesc>(), pl->plane_of.as<int>(), g.nw, g.m, g.n,
                                  pl->rhs, pl->stream), "initial projection");
        }
        const double* cur = ckpt_slot(a, 0);
        for (int k = 1; k <= N; ++k) {
            double* X = k > s_last ? seg_slot(a, k - s_last - 1) : h->Xt.as<double>();
            double* Pout = (k % K == 0 && k < N) ? ckpt_slot(a, k / K) : a->Pw.as<double>();
            heat_step_bdf1(h, cur, X, Pout);
            cur = Pout;
        }
        // leave the heat handle at step N
        const size_t eb = static_cast<size_t>(g.etotal_elems) * sizeof(double);
        hip_check(hipMemcpyAsync(h->P[0].p, cur, eb, hipMemcpyDeviceToDevice, pl->stream), "copy state");
        hip_check(hipMemcpyAsync(h->Xt.p, seg_slot(a, N - s_last - 1),
                                 static_cast<size_t>(g.total_elems) * sizeof(double), hipMemcpyDeviceToDevice,
                                 pl->stream), "copy state");
        h->head = 0;
        h->steps = N;
        a->seg_holds = a->nseg - 1;
        a->ready = true;
    });
}

int cyl_heat_grad_backward(cyl_heat_grad_t a, int space, const double* T_bar, double* T0_bar,
                           double* g_bar, double* alpha_bar) {
    return guarded([&] {
        if (!a || !T_bar || !T0_bar || !g_bar || !alpha_bar) fail(CYL_E_INVALID_ARG, "NULL argument");
        validate_space(space);
        if (!a->ready) fail(CYL_E_INVALID_ARG, "cyl_heat_grad_forward has not been run");
        cyl_heat_t h = a->heat;
        cyl_plan_s* pl = h->plan;
        const Geometry& g = pl->geo;
        Setup* adj = a->adj.get();
        const BlockDesc* fblocks = h->setup->blocks.as<BlockDesc>();
        const BlockDesc* ablocks = adj->blocks.as<BlockDesc>();
        const int nblk = static_cast<int>(adj->hblocks.size());
        const int N = a->steps, K = a->every;
        const double kappa = h->kappa;
        const int64_t xb = g.total_elems;
        hip_check(hipMemsetAsync(a->Gsum.p, 0, static_cast<size_t>(xb) * sizeof(double), pl->stream), "memset");
        hip_check(hipMemsetAsync(a->partials.p, 0, static_cast<size_t>(a->n_partials) * sizeof(double), pl->stream),
                  "memset");
        // seed: Xbar_N = Q^T Ubar_N Q, Ubar_N = F^-T T_bar
        const double2* Ubar = reinterpret_cast<const double2*>(T_bar);
        if (space == CYL_SPACE_VALUE) {
            transform_inv_adjoint(pl, T_bar, a->vals.as<double>(), a->planes.as<double2>());
            Ubar = a->planes.as<double2>();
        }
        {
            Scope sc(pl, PH_ADJ);
            hip_check(launch_recombine_t(Ubar, 1.0, a->Xh.as<double>(), ablocks, nblk,
                                         static_cast<int64_t>(g.me[0]) * g.ne[0], g.m, g.n, pl->stream),
                      "recombine_t");
        }
        const int64_t awstride = static_cast<int64_t>(g.me[0] + g.me[1]) * 12;
        for (int j = a->nseg - 1; j >= 0; --j) {
            const int s0 = j * K, len = std::min(K, N - s0);
            if (a->seg_holds != j) {                     // recompute X_{s0+1..s0+len}
                const double* cur = ckpt_slot(a, j);
                for (int t = 1; t <= len; ++t) {
                    heat_step_bdf1(h, cur, seg_slot(a, t - 1), a->Pw.as<double>());
                    cur = a->Pw.as<double>();
                }
                a->seg_holds = j;
            }
            for (int t = len; t >= 1; --t) {
                const int k = s0 + t;
                // Ebar_k = S^-T Xbar_k (flipped: the ordinary ADI on the flipped pencil)
                adi_solve(pl, adj, a->Xh.as<double>(), a->Et.as<double>());
                Scope sc(pl, PH_ADJ);
                hip_check(launch_apply_dot(fblocks, nblk, g.me[0], g.ne[0], seg_slot(a, t - 1), a->Et.as<double>(),
                                           a->atab_pois.as<double>(), awstride, pl->ztabA.as<double>(),
                                           a->partials.as<double>(), pl->stream), "alpha term");
                hip_check(launch_axpy(a->Gsum.as<double>(), a->Et.as<double>(), 1.0, xb, pl->stream), "accumulate");
                if (k > 1)                                // Xbar_{k-1} = C~^T Ebar_k B~^T
                    hip_check(launch_apply2(ablocks, nblk, g.me[0], g.ne[0], nullptr, 0.0, a->Et.as<double>(), -1.0,
                                            0.0, a->Xh.as<double>(), a->proj_flip.as<double>(), 0, adj->ztabA,
                                            pl->stream), "project_t");
            }
        }
        // T0_bar = F^T [R2^T Ebar_1 C02], g_bar = F^T kappa [R2^T (sum_k Ebar_k) C02]
        const double* srcs[2] = {a->Et.as<double>(), a->Gsum.as<double>()};
        const double scales[2] = {1.0, kappa};
        double* outs[2] = {T0_bar, g_bar};
        for (int q = 0; q < 2; ++q) {
            double2* U = space == CYL_SPACE_COEFF ? reinterpret_cast<double2*>(outs[q]) : a->planes.as<double2>();
            {
                Scope sc(pl, PH_ADJ);
                hip_check(launch_rhs_t(srcs[q], scales[q], U, pl->plane_of.as<int>(), ablocks, g.nw, g.m, g.n,
                                       pl->rhs, pl->stream), "rhs_t");
            }
            if (space == CYL_SPACE_VALUE) transform_fwd_adjoint(pl, U, outs[q]);
        }
        Scope sc(pl, PH_ADJ);
        hip_check(launch_sum(a->partials.as<double>(), a->n_partials, kappa, alpha_bar, pl->stream), "alpha sum");
    });
}

int cyl_heat_grad_destroy(cyl_heat_grad_t a) {
    return guarded([&] {
        if (!a) fail(CYL_E_INVALID_ARG, "handle is NULL");
        (void)hipStreamSynchronize(a->stream);
        delete a;
    });
}

int cyl_batch_create(cyl_batch_t* out, int count, const cyl_heat_t* heats, int flags) {
    cyl_batch_s* raw = nullptr;
    const int st = guarded([&] {
        if (!out) fail(CYL_E_INVALID_ARG, "batch pointer is NULL");
        *out = nullptr;
        if (count < 1 || !heats) fail(CYL_E_INVALID_ARG, "need count >= 1 heat handles");
        if (flags & ~(CYL_BATCH_NO_GRAPH | CYL_BATCH_NO_TUNE)) fail(CYL_E_INVALID_ARG, "unknown flags");
        auto B = std::make_unique<cyl_batch_s>();
        for (int i = 0; i < count; ++i) {
            if (!heats[i]) fail(CYL_E_INVALID_ARG, "NULL heat handle");
            for (int j = 0; j < i; ++j)
                if (heats[j] == heats[i]) fail(CYL_E_INVALID_ARG, "a heat handle appears twice");
            if (heats[i]->stream != heats[0]->stream) fail(CYL_E_INVALID_ARG, "member plans use different streams");
            if (heats[i]->physical) fail(CYL_E_UNSUPPORTED, "batches step all parity blocks (physical heat handle)");
            B->heats.push_back(heats[i]);
        }
        B->user = heats[0]->stream;
        batch_build(B.get(), flags);
        raw = B.release();
    });
    if (st == CYL_OK) *out = raw;
    return st;
}

int cyl_batch_step(cyl_batch_t b, int n_steps) {
    return guarded([&] {
        if (!b) fail(CYL_E_INVALID_ARG, "batch is NULL");
        if (n_steps < 0) fail(CYL_E_INVALID_ARG, "n_steps must be >= 0");
        const int nprob = static_cast<int>(b->heats.size());
        for (int q = 0; q < nprob; ++q) {
            cyl_heat_t h = b->heats[q];
            const int expect = static_cast<int>(((b->head0[q] - b->taken) % h->order + h->order) % h->order);
            if (h->steps != b->steps0[q] + b->taken || h->head != expect)
                fail(CYL_E_INVALID_ARG, "a member was stepped outside the batch");
        }
        if (n_steps == 0) return;
        hip_check(hipEventRecord(b->ev_in, b->user), "hipEventRecord");
        hip_check(hipStreamWaitEvent(b->stream, b->ev_in, 0), "hipStreamWaitEvent");
        int left = n_steps;
        while (left > 0 && (b->pos != 0 || !b->use_graph || left < b->L)) {
            batch_step_once(b, b->pos);
            batch_advance(b);
            --left;
        }
        while (left >= b->L) {
            hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
            for (int c = 0; c < b->L; ++c) batch_advance(b);
            left -= b->L;
        }
        while (left > 0) {
            batch_step_once(b, b->pos);
            batch_advance(b);
            --left;
        }
        hip_check(hipEventRecord(b->ev_out, b->stream), "hipEventRecord");
        hip_check(hipStreamWaitEvent(b->user, b->ev_out, 0), "hipStreamWaitEvent");
    });
}

int cyl_batch_describe(cyl_batch_t b, int* launches_per_pass, int* uses_graph, const char** grouping) {
    return guarded([&] {
        if (!b) fail(CYL_E_INVALID_ARG, "batch is NULL");
        if (launches_per_pass) *launches_per_pass = static_cast<int>(b->adi1.size());
        if (uses_graph) *uses_graph = b->use_graph ? 1 : 0;
        if (grouping) *grouping = b->grouping.c_str();
    });
}

int cyl_batch_destroy(cyl_batch_t b) {
    return guarded([&] {
        if (!b) fail(CYL_E_INVALID_ARG, "batch is NULL");
        (void)hipStreamSynchronize(b->stream);
        delete b;
    });
}

}  // extern "C"
