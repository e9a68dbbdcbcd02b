"""Python binding of libcylspec (the MI355X CCF cylinder solver).

Thin ctypes layer over the C ABI in include/cylspec.h: it checks tensor
shapes, dtypes and devices and passes raw device pointers.  Every step of the
computation runs in the library's HIP kernels; there is no fallback.  PyTorch
provides device memory and the current HIP stream.

Layouts (see the header): value space is a float64 tensor [n_theta, n_z, n_r];
coefficient space is a complex128 tensor [n_theta // 2 + 1, n_z, n_r].
"""

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# CYLSPEC_LIBRARY: another build of the same library (the host sanitizer build)
LIB_PATH = os.environ.get("CYLSPEC_LIBRARY") or os.path.join(_PKG, "libcylspec.so")

CYL_OK = 0
CYL_SPACE_VALUE = 0
CYL_SPACE_COEFF = 1
STATUS = {0: "CYL_OK", 1: "CYL_E_INVALID_ARG", 2: "CYL_E_UNSUPPORTED", 3: "CYL_E_OUT_OF_MEMORY",
          4: "CYL_E_HIP", 5: "CYL_E_NOT_CONVERGED", 6: "CYL_E_INTERNAL"}

# Every entry point declared in include/cylspec.h.
EXPORTS = ["cyl_plan_create", "cyl_plan_destroy", "cyl_transform_fwd", "cyl_transform_inv",
           "cyl_poisson_solve", "cyl_heat_create", "cyl_heat_step", "cyl_heat_read",
           "cyl_heat_destroy", "cyl_adi_parameters", "cyl_plan_set_profiling",
           "cyl_plan_get_profile", "cyl_status_string", "cyl_last_error",
           "cyl_transform_fwd_adjoint", "cyl_transform_inv_adjoint", "cyl_heat_grad_create",
           "cyl_heat_grad_forward", "cyl_heat_grad_backward", "cyl_heat_grad_destroy",
           "cyl_batch_create", "cyl_batch_step", "cyl_batch_describe", "cyl_batch_destroy",
           "cyl_plan_set_physical", "cyl_trace_lift", "cyl_disk_poisson_solve", "cyl_pt_decompose", "cyl_device_peaks",
           "cyl_plan_prepare", "cyl_poisson_solve_noalloc"]

CYL_BATCH_NO_GRAPH = 1
CYL_BATCH_NO_TUNE = 2


class CylError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class SolveInfo(ctypes.Structure):
    _fields_ = [("J_max", ctypes.c_int), ("J_min", ctypes.c_int), ("passes", ctypes.c_int),
                ("fused_residual", ctypes.c_int), ("resid_ratio", ctypes.c_double),
                ("adi_iterations_mean", ctypes.c_double), ("ms_transform", ctypes.c_double),
                ("ms_rhs", ctypes.c_double), ("ms_adi", ctypes.c_double), ("ms_inverse", ctypes.c_double)]


_PHASES = ["transform_fwd", "rhs", "adi", "residual", "recombine", "transform_inv", "heat_rhs",
           "project", "adjoint"]


class Profile(ctypes.Structure):
    _fields_ = [("ms_" + p, ctypes.c_double) for p in _PHASES] + \
               [("n_" + p, ctypes.c_int) for p in _PHASES]


_lib = None


def load():
    """Load libcylspec.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcylspec.so is not built; run __graft_entry__.build() "
                          "or python paper_2206_04827_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    sig = {
        "cyl_plan_create": [ctypes.POINTER(P), I, I, I, P],
        "cyl_plan_destroy": [P],
        "cyl_transform_fwd": [P, P, P],
        "cyl_transform_inv": [P, P, P],
        "cyl_poisson_solve": [P, I, P, P, P, D, ctypes.POINTER(SolveInfo)],
        "cyl_plan_prepare": [P, D],
        "cyl_poisson_solve_noalloc": [P, I, P, P, P, D, ctypes.POINTER(SolveInfo)],
        "cyl_heat_create": [ctypes.POINTER(P), P, D, D, I, D, I, ctypes.POINTER(P), P, P],
        "cyl_heat_step": [P, I],
        "cyl_heat_read": [P, I, P],
        "cyl_heat_destroy": [P],
        "cyl_adi_parameters": [I, I, I, D, D, ctypes.POINTER(D), ctypes.POINTER(I),
                               ctypes.POINTER(D), ctypes.POINTER(D), I],
        "cyl_plan_set_profiling": [P, I],
        "cyl_plan_get_profile": [P, ctypes.POINTER(Profile)],
        "cyl_transform_fwd_adjoint": [P, P, P],
        "cyl_transform_inv_adjoint": [P, P, P],
        "cyl_heat_grad_create": [ctypes.POINTER(P), P, I, I],
        "cyl_heat_grad_forward": [P],
        "cyl_heat_grad_backward": [P, I, P, P, P, P],
        "cyl_heat_grad_destroy": [P],
        "cyl_batch_create": [ctypes.POINTER(P), I, ctypes.POINTER(P), I],
        "cyl_batch_step": [P, I],
        "cyl_batch_describe": [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_char_p)],
        "cyl_batch_destroy": [P],
        "cyl_plan_set_physical": [P, I],
        "cyl_trace_lift": [P, P, P, P],
        "cyl_disk_poisson_solve": [P, I, P, P],
        "cyl_pt_decompose": [P, I, P, P, P, P, P],
        "cyl_device_peaks": [P, P, P, ctypes.c_int64, I, ctypes.POINTER(D), ctypes.POINTER(D)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I
    lib.cyl_status_string.argtypes = [I]
    lib.cyl_status_string.restype = ctypes.c_char_p
    lib.cyl_last_error.argtypes = []
    lib.cyl_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status):
    if status != CYL_OK:
        raise CylError(status, load().cyl_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def adi_parameters(n_r, n_z, w, kappa_alpha=0.0, adi_tol=1e-12, cap=512):
    """Host-only: enclosing bounds (a, b, c, d), J and shifts (u, v) for wavenumber w."""
    lib = load()
    b4 = (ctypes.c_double * 4)()
    J = ctypes.c_int()
    u = (ctypes.c_double * cap)()
    v = (ctypes.c_double * cap)()
    _check(lib.cyl_adi_parameters(n_r, n_z, w, kappa_alpha, adi_tol, b4, ctypes.byref(J), u, v, cap))
    return {"bounds": list(b4), "J": J.value, "u": list(u[:J.value]), "v": list(v[:J.value])}


def device_peaks(n=1 << 26, reps=5, stream=None):
    """Measured FP64 FMA rate (TFLOP/s) and streaming-copy bandwidth (GB/s) of
    the current device (the copy moves 2 x 8 n bytes per launch)."""
    lib = load()
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    tf, gb = ctypes.c_double(), ctypes.c_double()
    s = ctypes.c_void_p(stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    _check(lib.cyl_device_peaks(s, _ptr(src), _ptr(dst), n, reps, ctypes.byref(tf), ctypes.byref(gb)))
    return {"fp64_tflops": tf.value, "copy_gbs": gb.value, "copy_bytes": 16 * n}


class Plan:
    """An n_r x n_z x n_theta CCF plan bound to a HIP stream (default: torch's current)."""

    def __init__(self, n_r, n_z, n_theta, stream=None):
        self._lib = load()
        self.n_r, self.n_z, self.n_theta = int(n_r), int(n_z), int(n_theta)
        self.nw = self.n_theta // 2 + 1
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._h = ctypes.c_void_p()
        self._prepared = set()
        _check(self._lib.cyl_plan_create(ctypes.byref(self._h), self.n_r, self.n_z, self.n_theta,
                                         ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if self._h:
            _check(self._lib.cyl_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shapes ------------------------------------------------------------
    @property
    def value_shape(self):
        return (self.n_theta, self.n_z, self.n_r)

    @property
    def coeff_shape(self):
        return (self.nw, self.n_z, self.n_r)

    def _check_tensor(self, t, space, name):
        if t is None:
            return
        if not t.is_cuda:
            raise ValueError("%s must be a device tensor" % name)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if space == CYL_SPACE_VALUE:
            if t.dtype != torch.float64 or tuple(t.shape) != self.value_shape:
                raise ValueError("%s must be float64 %s" % (name, self.value_shape))
        else:
            if t.dtype != torch.complex128 or tuple(t.shape) != self.coeff_shape:
                raise ValueError("%s must be complex128 %s" % (name, self.coeff_shape))

    def _out(self, space, out):
        if out is not None:
            self._check_tensor(out, space, "out")
            return out
        dev = torch.device("cuda", torch.cuda.current_device())
        if space == CYL_SPACE_VALUE:
            return torch.empty(self.value_shape, dtype=torch.float64, device=dev)
        return torch.empty(self.coeff_shape, dtype=torch.complex128, device=dev)

    # -- operations --------------------------------------------------------
    def transform_fwd(self, values, out=None):
        self._check_tensor(values, CYL_SPACE_VALUE, "values")
        out = self._out(CYL_SPACE_COEFF, out)
        _check(self._lib.cyl_transform_fwd(self._h, _ptr(values), _ptr(out)))
        return out

    def transform_inv(self, coeffs, out=None):
        self._check_tensor(coeffs, CYL_SPACE_COEFF, "coeffs")
        out = self._out(CYL_SPACE_VALUE, out)
        _check(self._lib.cyl_transform_inv(self._h, _ptr(coeffs), _ptr(out)))
        return out

    def transform_fwd_adjoint(self, coeffs_bar, out=None):
        """values_bar = F^T coeffs_bar (transpose of ``transform_fwd``)."""
        self._check_tensor(coeffs_bar, CYL_SPACE_COEFF, "coeffs_bar")
        out = self._out(CYL_SPACE_VALUE, out)
        _check(self._lib.cyl_transform_fwd_adjoint(self._h, _ptr(coeffs_bar), _ptr(out)))
        return out

    def transform_inv_adjoint(self, values_bar, out=None):
        """coeffs_bar = (F^-1)^T values_bar (transpose of ``transform_inv``)."""
        self._check_tensor(values_bar, CYL_SPACE_VALUE, "values_bar")
        out = self._out(CYL_SPACE_COEFF, out)
        _check(self._lib.cyl_transform_inv_adjoint(self._h, _ptr(values_bar), _ptr(out)))
        return out

    def set_physical(self, enable=True):
        """Physical-parity fast path for ``poisson_solve`` (j = w mod 2 blocks
        only; even n_theta)."""
        _check(self._lib.cyl_plan_set_physical(self._h, 1 if enable else 0))

    def trace_lift(self, rface, zface, out=None):
        """Coons lift of the boundary faces: rface [2, n_theta, n_z] (r = -1,
        r = +1), zface [2, n_theta, n_r] (z = -1, z = +1), device float64."""
        for t, shp, name in ((rface, (2, self.n_theta, self.n_z), "rface"),
                             (zface, (2, self.n_theta, self.n_r), "zface")):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and tuple(t.shape) == shp):
                raise ValueError("%s must be a contiguous float64 device tensor %s" % (name, shp))
        out = self._out(CYL_SPACE_VALUE, out)
        _check(self._lib.cyl_trace_lift(self._h, _ptr(rface), _ptr(zface), _ptr(out)))
        return out

    def prepare(self, adi_tol):
        """Build the ADI tables of a tolerance (host work, device allocation)."""
        adi_tol = float(adi_tol)
        if adi_tol not in self._prepared:
            _check(self._lib.cyl_plan_prepare(self._h, adi_tol))
            self._prepared.add(adi_tol)

    def poisson_solve(self, f, bc_lift=None, adi_tol=1e-12, space=None, out=None, info=False,
                      bc_traces=None, noalloc=False):
        """Solve nabla^2 u = f (u = lift on the boundary). Returns u (and info if asked).

        A tolerance not yet prepared is prepared first (outside graph capture:
        that allocates).  bc_traces: (rface, zface) boundary faces instead of a
        lift (value space); the lift is built with ``trace_lift``.  noalloc:
        use ``cyl_poisson_solve_noalloc`` (workspace in the library's static
        device scratch)."""
        self.prepare(adi_tol)
        if space is None:
            space = CYL_SPACE_COEFF if f.dtype == torch.complex128 else CYL_SPACE_VALUE
        if bc_traces is not None:
            if bc_lift is not None or space != CYL_SPACE_VALUE:
                raise ValueError("bc_traces needs value space and no bc_lift")
            bc_lift = self.trace_lift(*bc_traces)
        self._check_tensor(f, space, "f")
        self._check_tensor(bc_lift, space, "bc_lift")
        out = self._out(space, out)
        inf = SolveInfo() if info else None
        fn = self._lib.cyl_poisson_solve_noalloc if noalloc else self._lib.cyl_poisson_solve
        _check(fn(self._h, space, _ptr(f), _ptr(bc_lift), _ptr(out), float(adi_tol),
                  ctypes.byref(inf) if info else None))
        if info:
            return out, {k: getattr(inf, k) for k, _ in SolveInfo._fields_}
        return out

    def disk_poisson_solve(self, f, space=None, out=None):
        """Horizontal (disk) Poisson Delta_h u = f, u = 0 at r = 1 (no z condition)."""
        if space is None:
            space = CYL_SPACE_COEFF if f.dtype == torch.complex128 else CYL_SPACE_VALUE
        self._check_tensor(f, space, "f")
        out = self._out(space, out)
        _check(self._lib.cyl_disk_poisson_solve(self._h, space, _ptr(f), _ptr(out)))
        return out

    def pt_decompose(self, v_r, v_theta, v_z, space=None, out=None):
        """Poloidal-toroidal decomposition (lambda, gamma) of (v_r, v_theta, v_z):
        Delta_h gamma = -v_z, Delta_h lambda = -(z . curl V), both zero at r = 1."""
        if space is None:
            space = CYL_SPACE_COEFF if v_z.dtype == torch.complex128 else CYL_SPACE_VALUE
        for t, name in ((v_r, "v_r"), (v_theta, "v_theta"), (v_z, "v_z")):
            self._check_tensor(t, space, name)
        lam, gam = out if out is not None else (None, None)
        lam = self._out(space, lam)
        gam = self._out(space, gam)
        _check(self._lib.cyl_pt_decompose(self._h, space, _ptr(v_r), _ptr(v_theta), _ptr(v_z),
                                          _ptr(lam), _ptr(gam)))
        return lam, gam

    def set_profiling(self, enable=True):
        _check(self._lib.cyl_plan_set_profiling(self._h, 1 if enable else 0))

    def profile(self):
        p = Profile()
        _check(self._lib.cyl_plan_get_profile(self._h, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in Profile._fields_}


class Heat:
    """BDF heat stepping (d_t - alpha nabla^2) T = g on a plan."""

    def __init__(self, plan, history, g, alpha, dt, bdf_order=1, adi_tol=1e-12, bc_lift=None,
                 space=None):
        self.plan = plan
        self._lib = plan._lib
        if space is None:
            space = CYL_SPACE_COEFF if g.dtype == torch.complex128 else CYL_SPACE_VALUE
        if len(history) != bdf_order:
            raise ValueError("history must hold bdf_order fields, newest first")
        for i, t in enumerate(history):
            plan._check_tensor(t, space, "history[%d]" % i)
        plan._check_tensor(g, space, "g")
        plan._check_tensor(bc_lift, space, "bc_lift")
        arr = (ctypes.c_void_p * bdf_order)(*[t.data_ptr() for t in history])
        self._h = ctypes.c_void_p()
        _check(self._lib.cyl_heat_create(ctypes.byref(self._h), plan._h, float(alpha), float(dt),
                                         int(bdf_order), float(adi_tol), space, arr, _ptr(g),
                                         _ptr(bc_lift)))

    def step(self, n_steps=1):
        _check(self._lib.cyl_heat_step(self._h, int(n_steps)))

    def read(self, space=CYL_SPACE_VALUE, out=None):
        out = self.plan._out(space, out)
        _check(self._lib.cyl_heat_read(self._h, space, _ptr(out)))
        return out

    def close(self):
        if self._h:
            _check(self._lib.cyl_heat_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HeatGrad:
    """Reverse-mode differentiation of a BDF1 ``Heat`` run of n_steps steps.

    ``forward()`` restarts the heat handle from its initial field and runs it,
    keeping a checkpoint every ``checkpoint_every`` steps; ``backward(T_bar)``
    returns (dL/dT0, dL/dg, dL/dalpha) for T_bar = dL/dT_N.
    """

    def __init__(self, heat, n_steps, checkpoint_every=20):
        self.heat = heat
        self.plan = heat.plan
        self._lib = heat._lib
        self.n_steps = int(n_steps)
        self._h = ctypes.c_void_p()
        _check(self._lib.cyl_heat_grad_create(ctypes.byref(self._h), heat._h, self.n_steps,
                                              int(checkpoint_every)))

    def forward(self):
        _check(self._lib.cyl_heat_grad_forward(self._h))

    def backward(self, T_bar, space=None):
        if space is None:
            space = CYL_SPACE_COEFF if T_bar.dtype == torch.complex128 else CYL_SPACE_VALUE
        self.plan._check_tensor(T_bar, space, "T_bar")
        T0_bar = self.plan._out(space, None)
        g_bar = self.plan._out(space, None)
        alpha_bar = torch.empty((), dtype=torch.float64, device=T_bar.device)
        _check(self._lib.cyl_heat_grad_backward(self._h, space, _ptr(T_bar), _ptr(T0_bar),
                                                _ptr(g_bar), _ptr(alpha_bar)))
        return T0_bar, g_bar, alpha_bar

    def close(self):
        if self._h:
            _check(self._lib.cyl_heat_grad_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched stepping of several ``Heat`` handles (uneven sizes) in few launches.

    ``graph``: replay a captured HIP graph of one step cycle; ``tune``: time
    candidate launch configurations once and keep the fastest (cached per
    batch signature, on disk when CYLSPEC_TUNE_CACHE names a file).
    """

    def __init__(self, heats, graph=True, tune=True):
        self.heats = list(heats)
        self._lib = self.heats[0]._lib
        arr = (ctypes.c_void_p * len(self.heats))(*[h._h.value for h in self.heats])
        flags = (0 if graph else CYL_BATCH_NO_GRAPH) | (0 if tune else CYL_BATCH_NO_TUNE)
        self._h = ctypes.c_void_p()
        _check(self._lib.cyl_batch_create(ctypes.byref(self._h), len(self.heats), arr, flags))

    def step(self, n_steps=1):
        _check(self._lib.cyl_batch_step(self._h, int(n_steps)))

    def describe(self):
        n = ctypes.c_int()
        g = ctypes.c_int()
        s = ctypes.c_char_p()
        _check(self._lib.cyl_batch_describe(self._h, ctypes.byref(n), ctypes.byref(g), ctypes.byref(s)))
        return {"launches_per_pass": n.value, "graph": bool(g.value), "grouping": s.value.decode()}

    def close(self):
        if self._h:
            _check(self._lib.cyl_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
