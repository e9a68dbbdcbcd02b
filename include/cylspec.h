/*
 * cylspec -- spectral Poisson and heat solver in the closed cylinder on MI355X.
 *
 * Method: D. Darrow, "A Quasi-Optimal Spectral Solver for the Heat and Poisson
 * Equations in a Closed Cylinder" (arXiv 2206.04827).  A field on the doubled
 * Chebyshev-Chebyshev-Fourier grid (Section 2, Definition "grid") is moved to
 * CCF coefficients by DCT-I in r, DCT-I in z and a DFT in theta (Section 2);
 * each Fourier mode then obeys its own sparse Sylvester equation
 * (Section 3, eq. HelmholtzMatEqn), which is solved by ADI with Zolotarev
 * shifts (Section 3, Algorithm 1 and the shift formulas after it).
 *
 * Conventions for every call below:
 *  - All array arguments are DEVICE pointers to FP64 data, used on the plan's
 *    HIP stream.  The caller allocates and frees them; inputs and outputs must
 *    not alias.  Every call returns after enqueueing work; results are valid
 *    after the stream has synchronised.
 *  - Value space: real array [n_theta][n_z][n_r], r fastest.  Element (l,k,j)
 *    is the value at the grid point of Definition "grid":
 *        r_j = cos((n_r - j - 1) pi / (n_r - 1)),  z_k likewise,
 *        theta_l = (2 l - n_theta) pi / n_theta.
 *  - Coefficient space: complex interleaved (re, im) array
 *    [floor(n_theta/2) + 1][n_z][n_r], r fastest.  Slot (w,k,j) holds the
 *    coefficient of T_j(r) T_k(z) e^{i w theta} (Section 2, the CCF
 *    polynomial) of a REAL field, w = 0..floor(n_theta/2); negative w follow by
 *    conjugation.  For even n_theta the slot w = n_theta/2 holds the paper's
 *    w = -n_theta/2 coefficient (the same function on the grid).  Imaginary
 *    parts of the w = 0 and Nyquist slots are ignored on input and written as 0.
 *  - Boundary data: homogeneous Dirichlet at r = +-1 and z = +-1 unless a lift
 *    field is given.  A lift is any field (same space as the data) whose values
 *    on the boundary grid points are the Dirichlet data; only those boundary
 *    values affect the result.  The paper states no boundary closure for these
 *    two problems; this tau/Dirichlet closure is the library's reading.
 *  - Errors: argument checks are synchronous and enqueue nothing.  A failed
 *    call returns a CYL_E_* code; cyl_last_error() gives a thread-local
 *    description.  HIP runtime failures map to CYL_E_HIP.
 *  - Handles are not thread safe.
 */
#ifndef CYLSPEC_H
#define CYLSPEC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cyl_plan_s* cyl_plan_t;
typedef struct cyl_heat_s* cyl_heat_t;
typedef struct cyl_heat_grad_s* cyl_heat_grad_t;
typedef struct cyl_batch_s* cyl_batch_t;

enum {
    CYL_OK = 0,
    CYL_E_INVALID_ARG = 1,
    CYL_E_UNSUPPORTED = 2,
    CYL_E_OUT_OF_MEMORY = 3,
    CYL_E_HIP = 4,
    CYL_E_NOT_CONVERGED = 5,
    CYL_E_INTERNAL = 6
};

enum { CYL_SPACE_VALUE = 0, CYL_SPACE_COEFF = 1 };

/* Filled by cyl_poisson_solve when a host pointer is given (this synchronises
 * the stream).  resid_ratio = ||E - L(X)||_2 / ||E||_2 over all modes, where
 * L(X) = A X B + C X D is the per-mode operator of eq. (HelmholtzMatEqn).
 * The ms_ fields are this solve's phases, timed with HIP events on the
 * plan's stream (the residual check itself is not in them). */
typedef struct {
    int J_max;          /* most ADI iterations of any mode (per pass)        */
    int J_min;          /* fewest ADI iterations of any mode (per pass)      */
    int passes;         /* 1, or 2 when a residual-correction pass was run   */
    int fused_residual; /* 1: the first pass's ADI launch also formed the
                           residual for the second (no separate launch)      */
    double resid_ratio;
    double adi_iterations_mean; /* mean J over real mode planes, per pass   */
    double ms_transform;  /* forward transforms (value space; 0 otherwise)   */
    double ms_rhs;        /* tau right side                                  */
    double ms_adi;        /* ADI passes and the residual between them        */
    double ms_inverse;    /* recombination and inverse transforms            */
} cyl_solve_info;

/* Accumulated device time per phase since profiling was enabled (ms), and the
 * number of launches recorded for each.  Filled by cyl_plan_get_profile. */
typedef struct {
    double ms_transform_fwd, ms_rhs, ms_adi, ms_residual, ms_recombine,
           ms_transform_inv, ms_heat_rhs, ms_project, ms_adjoint;
    int n_transform_fwd, n_rhs, n_adi, n_residual, n_recombine,
        n_transform_inv, n_heat_rhs, n_project, n_adjoint;
} cyl_profile;

/* Create a plan for an n_r x n_z x n_theta grid (Definition "grid").
 * Requires 4 <= n_r, n_z <= 1025 and 1 <= n_theta <= 4096.  The plan owns the
 * operator bands of Section 3 for every wavenumber and a device workspace;
 * hip_stream (a hipStream_t, NULL = the default stream) is used for all work.
 * Ownership: the caller destroys the plan with cyl_plan_destroy. */
int cyl_plan_create(cyl_plan_t* plan, int n_r, int n_z, int n_theta, void* hip_stream);
int cyl_plan_destroy(cyl_plan_t plan);

/* Values -> coefficients (Section 2: DCT-I along r, DCT-I along z, DFT along
 * theta).  values: [n_theta][n_z][n_r]; coeffs: complex [n_theta/2+1][n_z][n_r]. */
int cyl_transform_fwd(cyl_plan_t plan, const double* values, double* coeffs);
/* Coefficients -> values on the grid (the inverse of cyl_transform_fwd). */
int cyl_transform_inv(cyl_plan_t plan, const double* coeffs, double* values);

/* Transposes of the two transforms with respect to the real inner products
 * sum x_i y_i of the stored arrays (complex arrays as interleaved doubles; the
 * imaginary parts of the w = 0 and Nyquist slots are not part of the
 * coefficient space: ignored on input, written as 0).  The chain rule needs
 * them to move gradients between value and coefficient space:
 *   cyl_transform_fwd_adjoint: values_bar = F^T coeffs_bar,
 *   cyl_transform_inv_adjoint: coeffs_bar = (F^-1)^T values_bar,
 * with F the map of cyl_transform_fwd.  Both use the plan's workspace. */
int cyl_transform_fwd_adjoint(cyl_plan_t plan, const double* coeffs_bar, double* values_bar);
int cyl_transform_inv_adjoint(cyl_plan_t plan, const double* values_bar, double* coeffs_bar);

/* Build and upload the ADI tables of the Poisson pencil for one tolerance
 * (Section 3: the eigenvalue bounds, J and the Zolotarev shifts after
 * Algorithm 1, and the per-shift banded factors).  adi_tol: the ADI tolerance
 * eps, 1e-15 <= eps <= 1e-2; the number of ADI iterations per mode is
 * J = ceil(ln(16 gamma) ln(4/eps) / pi^2).  Host work and device allocation;
 * synchronous.  Preparing a tolerance twice does nothing the second time.
 * The one- or two-pass policy of the tolerance is fixed here. */
int cyl_plan_prepare(cyl_plan_t plan, double adi_tol);

/* Solve nabla^2 u = f in the cylinder (Section 3, eq. HelmholtzMatEqn without
 * time terms), u = bc on the boundary (bc_lift == NULL: homogeneous).
 * space: CYL_SPACE_VALUE or CYL_SPACE_COEFF for f, bc_lift and u alike.
 * adi_tol: a tolerance prepared with cyl_plan_prepare (CYL_E_INVALID_ARG
 * otherwise).  Allocates nothing and, with info == NULL, only enqueues
 * kernels on the plan's stream, so it may be captured into a HIP graph.
 * Uses the plan's workspace: calls on one plan must not overlap.
 * info: NULL, or a host struct to fill (synchronises; CYL_E_NOT_CONVERGED if
 * the result is not finite or resid_ratio > 1e3 * max(adi_tol, 1e-12)). */
int cyl_poisson_solve(cyl_plan_t plan, int space, const double* f, const double* bc_lift,
                      double* u, double adi_tol, cyl_solve_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as cyl_poisson_solve, same arguments and results, but its workspace
 * (coefficient planes, right side, residual, solution blocks and reduction
 * slots) is carved from a static device array of 64 MiB that the library
 * holds on every device it runs on until the process ends, instead of the
 * plan's own buffers.  The call allocates nothing; the plan and the prepared
 * tolerance must exist beforehand (cyl_plan_create, cyl_plan_prepare).
 * A grid whose workspace exceeds 64 MiB (about 100^3 values; the lift doubles
 * the planes) fails with CYL_E_UNSUPPORTED and enqueues nothing.  Every call
 * on one device shares that device's array, whatever the plan: calls that
 * may overlap on one device (other streams, other threads) race and must be
 * ordered by the caller.  The array keeps the last call's contents; the call
 * clears what it needs cleared itself, with kernels. */
int cyl_poisson_solve_noalloc(cyl_plan_t plan, int space, const double* f, const double* bc_lift,
                              double* u, double adi_tol, cyl_solve_info* info);

/* Physical-parity fast path for cyl_poisson_solve on this plan (enable != 0)
 * or the general solve (0, the default).  On the doubled grid (r in [-1, 1])
 * a function that is single-valued and smooth on the cylinder satisfies
 * f(-r, theta) = f(r, theta + pi), so its coefficient of T_j(r) e^{i w theta}
 * vanishes unless j = w (mod 2), and the Poisson operator keeps that subspace
 * (the parity restriction the paper's introduction cites for the doubled
 * discretization).  Enabled, a solve runs the ADI and the residual
 * correction on the j = w (mod 2) parity blocks only (half of the blocks)
 * and returns a solution whose other coefficients are exactly zero; the
 * other-parity part of f (rounding for physical forcing) is discarded.  The
 * residual ratio reported in cyl_solve_info still covers all of f.  Needs an
 * even n_theta (CYL_E_UNSUPPORTED otherwise: for odd n_theta theta + pi is no
 * grid angle and the sampled parities mix).  Heat handles created while the
 * flag is set step the same way (BDF keeps the subspace): their initial state
 * and forcing are taken as physical, and their steps solve and project the
 * j = w (mod 2) blocks only; cyl_heat_grad_create and cyl_batch_create reject
 * such handles with CYL_E_UNSUPPORTED. */
int cyl_plan_set_physical(cyl_plan_t plan, int enable);

/* Lift from boundary traces (non-homogeneous Dirichlet data given on the
 * boundary only): lift = the transfinite (Coons) interpolant in (r, z) of
 * the four faces of the doubled grid's box on every theta line,
 *   L = (1-a) R_-(z) + a R_+(z) + (1-b) Z_-(r) + b Z_+(r) - (bilinear corner terms),
 * a = (1 + r)/2, b = (1 + z)/2, corners from the z-faces.  rface: device
 * [2][n_theta][n_z] (the values at r = -1, then at r = +1: the side wall at
 * theta + pi and at theta); zface: device [2][n_theta][n_r] (z = -1, then
 * z = +1); lift: device [n_theta][n_z][n_r], written (value space).  For
 * data that agree on the box's edges the lift takes the given values on all
 * faces; pass it as bc_lift to cyl_poisson_solve or cyl_heat_create (the
 * r^2-weighted equations of Section 3 admit any lift with those boundary
 * values, and the discrete solution depends on the boundary values only).
 * Enqueued on the plan's stream; allocates nothing. */
int cyl_trace_lift(cyl_plan_t plan, const double* rface, const double* zface, double* lift);

/* Horizontal (disk) Poisson solve of Section 4 (eq. ptpoisson, the building
 * block of the poloidal-toroidal decomposition): Delta_h u = f with
 * Delta_h = nabla^2 - d_zz, u = 0 on the side wall r = 1 (no condition in z,
 * where Delta_h has no derivative).  Diagonalised in theta (DFT) and z (every
 * Chebyshev z coefficient is its own problem): per wavenumber and z
 * coefficient one banded tau system in r, [A_w Q]_tau x = [R^2 C02 f]_tau,
 * u = Q x, solved directly (no ADI, no tolerance).  space: CYL_SPACE_VALUE or
 * CYL_SPACE_COEFF for f and u alike; in coefficient space u must not alias f.
 * The records are built with the plan; the call allocates nothing.  Timed
 * as the ADI phase when profiling. */
int cyl_disk_poisson_solve(cyl_plan_t plan, int space, const double* f, double* u);

/* Poloidal-toroidal decomposition of Section 4 (eqs. pt and ptpoisson):
 * for V = curl(lambda z) + curl curl(gamma z), z . V = -Delta_h gamma and
 * z . curl V = -Delta_h lambda.  Given the cylindrical components of V on the
 * doubled grid (v_r, v_theta, v_z: at (r, theta) with r < 0 the components
 * along (cos theta, sin theta) and (-sin theta, cos theta) at the point
 * r (cos theta, sin theta), i.e. with the signed radius), computes
 *   gamma:  Delta_h gamma  = -v_z,
 *   lambda: Delta_h lambda = -(z . curl V),
 * both with the potential zero on the side wall r = 1, by two disk solves
 * (as cyl_disk_poisson_solve).  The curl enters with r^2 weighting, as the
 * tau right side [-R (C02 + R C12 D1) V_theta + i w R C02 V_r]_tau, so no
 * division by r occurs; for even n_theta the theta derivative of the Nyquist
 * slot w = n_theta/2 is taken as zero.  The field need not be solenoidal.
 * space: CYL_SPACE_VALUE (all five arrays [n_theta][n_z][n_r] doubles; the
 * outputs may alias the inputs: all inputs are read first) or
 * CYL_SPACE_COEFF (all five coefficient planes; neither output may alias an
 * input).  lambda and gamma must differ.  Enqueued on the
 * plan's stream; uses the plan's three coefficient-plane buffers and
 * allocates nothing.  Timed as the ADI phase when profiling. */
int cyl_pt_decompose(cyl_plan_t plan, int space, const double* v_r, const double* v_theta, const double* v_z,
                     double* lambda, double* gamma);

/* Heat equation (d_t - alpha nabla^2) T = g (Section 3), advanced by BDF of
 * order bdf_order in {1, 4} with step dt (kappa^(1) = dt,
 * kappa^(4) = 12 dt / 25); g and the boundary data are time independent.
 * history: host array of bdf_order device pointers to the fields T(t),
 * T(t-dt), ... (newest first) in the given space.  The handle copies what it
 * needs; the caller's arrays may be freed after the call.  The handle owns its
 * device state until cyl_heat_destroy. */
int cyl_heat_create(cyl_heat_t* h, cyl_plan_t plan, double alpha, double dt, int bdf_order,
                    double adi_tol, int space, const double* const* history,
                    const double* g, const double* bc_lift);
/* Advance n_steps >= 0 steps (enqueue only; allocates nothing).  The plan
 * must stay alive while the handle is used; cyl_heat_destroy does not touch
 * the plan, so the two may be destroyed in either order. */
int cyl_heat_step(cyl_heat_t h, int n_steps);
/* Write the newest temperature field to T_out in the given space. */
int cyl_heat_read(cyl_heat_t h, int space, double* T_out);
int cyl_heat_destroy(cyl_heat_t h);

/* Reverse-mode differentiation of a BDF1 heat run (the chain rule through the
 * discrete method of Section 3; the paper gives no adjoint).  For a handle
 * created with bdf_order = 1, no lift, initial field T_0 = history[0] and
 * forcing g, a run of n_steps steps gives T_N; for a scalar loss L(T_N) with
 * gradient T_bar = dL/dT_N the backward call returns dL/dT_0, dL/dg and
 * dL/dalpha.  Each step's transposed Sylvester solve runs ADI with the forward
 * step's shifts (the transposed pencil has the same spectra).
 *
 * cyl_heat_grad_create: n_steps >= 1; checkpoint_every >= 1 (the forward run
 *   keeps the state every checkpoint_every steps; the backward run recomputes
 *   each segment from its checkpoint, i.e. about n_steps - checkpoint_every
 *   extra forward steps).  Allocates ceil(n_steps / checkpoint_every) states in
 *   E-layout plus checkpoint_every solution fields (8 (n_r-2)(n_z-2) n_theta
 *   bytes each) and the transposed ADI tables.  CYL_E_UNSUPPORTED for BDF4 or
 *   a lifted handle.  Every call but cyl_heat_grad_destroy needs the heat
 *   handle and its plan alive; the handles may be destroyed in any order.
 * cyl_heat_grad_forward: restart the heat handle from its T_0 and advance it
 *   n_steps (afterwards cyl_heat_read gives T_N).  Enqueue only.
 * cyl_heat_grad_backward: T_bar in `space`; T0_bar and g_bar receive the
 *   gradients in the same space (value space: arrays [n_theta][n_z][n_r];
 *   coefficient space: the gradient with respect to the stored doubles of the
 *   coefficient array); alpha_bar: DEVICE pointer to one double.  Requires a
 *   preceding forward call; may be repeated for other T_bar.  Enqueue only. */
int cyl_heat_grad_create(cyl_heat_grad_t* a, cyl_heat_t h, int n_steps, int checkpoint_every);
int cyl_heat_grad_forward(cyl_heat_grad_t a);
int cyl_heat_grad_backward(cyl_heat_grad_t a, int space, const double* T_bar, double* T0_bar,
                           double* g_bar, double* alpha_bar);
int cyl_heat_grad_destroy(cyl_heat_grad_t a);

/* Batched heat stepping over independent problems of uneven sizes (the
 * per-mode solves of Section 3 are independent within a problem and across
 * problems).  A batch step runs, for every member, the heat right side, the
 * ADI passes (and residual correction) and the history projection of
 * cyl_heat_step, but as a few launches over all members: one heat-right-side
 * launch, per ADI pass a few launches that take the parity blocks of all
 * members sorted by cost J(w) m_e n_e, one residual and one projection launch.
 * Results are identical to stepping every member with cyl_heat_step.
 *
 * cyl_batch_create: count >= 1 distinct heat handles whose plans share one
 *   stream.  The batch owns a right-side and a residual workspace per member
 *   (2 E-layout fields each), its own HIP stream and, unless
 *   CYL_BATCH_NO_GRAPH, a HIP graph of one step cycle (lcm of the members'
 *   BDF orders) that cyl_batch_step replays.  Unless CYL_BATCH_NO_TUNE, it
 *   times candidate launch configurations once and keeps the fastest: the
 *   grouping of the blocks into launches, persistent work-queue launches of
 *   the split kernels, 8- or 16-row groups.  The choice is cached per batch
 *   signature for the process and, when the environment variable
 *   CYLSPEC_TUNE_CACHE names a file, in that file (read once per process,
 *   rewritten whole when an entry is added; an unwritable path only loses
 *   the cache).
 * cyl_batch_step: advance every member n_steps (enqueue only; ordered after
 *   earlier work on the members' stream and before later work on it).
 *   Members must not be stepped by other calls while in the batch
 *   (CYL_E_INVALID_ARG).  Results are read with cyl_heat_read.
 * cyl_batch_describe: launches per ADI pass, whether a graph is replayed, and
 *   the chosen launch configuration (a string owned by the batch). */
enum { CYL_BATCH_NO_GRAPH = 1, CYL_BATCH_NO_TUNE = 2 };
int cyl_batch_create(cyl_batch_t* b, int count, const cyl_heat_t* heats, int flags);
int cyl_batch_step(cyl_batch_t b, int n_steps);
int cyl_batch_describe(cyl_batch_t b, int* launches_per_pass, int* uses_graph, const char** grouping);
int cyl_batch_destroy(cyl_batch_t b);

/* Host-only (needs no GPU): the ADI parameters the plan would use for
 * wavenumber w of an n_r x n_z grid.  kappa_alpha = 0 selects the Poisson
 * pencil, kappa_alpha > 0 the heat pencil of eq. (HelmholtzMatEqn).
 * bounds4 receives the enclosing spectral intervals [a, b] and [c, d] of
 * Section 3 (a, b for C^-1 A; c, d for -D B^-1); J receives the iteration
 * count; u and v (capacity cap) receive the shifts u_j (first half-step, in
 * [c, d]) and v_j (second half-step, in [a, b]). */
int cyl_adi_parameters(int n_r, int n_z, int w, double kappa_alpha, double adi_tol,
                       double* bounds4, int* J, double* u, double* v, int cap);

/* Profiling: record HIP events around every phase on the plan's stream. */
int cyl_plan_set_profiling(cyl_plan_t plan, int enable);
/* Synchronise, return and reset the accumulated per-phase device times. */
int cyl_plan_get_profile(cyl_plan_t plan, cyl_profile* out);

/* Device peak check (measurement support, not a step of the method): the
 * rates roofline fractions are quoted against, measured on this device.  On
 * hip_stream (a hipStream_t, NULL = the default stream) it times one warm-up
 * and then `reps` launches (1..1000) of each check with HIP events and keeps
 * the fastest:
 *   fp64_tflops: independent FP64 FMA chains in every lane of 8 workgroups
 *     of 256 lanes per compute unit, 2 operations per FMA;
 *   copy_gbs: a streaming copy dst[i] = src[i] of n doubles (device buffers,
 *     16-byte aligned, not overlapping, n > 0), 16 n bytes moved per launch.
 * Either output may be NULL to skip that check (src, dst and n are then
 * unused by it).  Synchronises the stream; allocates nothing; dst is
 * overwritten by the copy. */
int cyl_device_peaks(void* hip_stream, const double* src, double* dst, int64_t n, int reps,
                     double* fp64_tflops, double* copy_gbs);

const char* cyl_status_string(int status);
const char* cyl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CYLSPEC_H */
