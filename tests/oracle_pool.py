"""Per-wavenumber oracle solves spread over worker processes.

Test infrastructure: the oracle's per-mode solves are independent (the theta
decoupling of eq. (HelmholtzMatEqn)), so whole-field references at the
benchmark sizes are computed by single-threaded workers, one wavenumber per
task.  Workers are started with "spawn" and import only the oracle (never
torch or the HIP library).
"""

import multiprocessing as mp
import os

import numpy as np


def _limit_threads():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _poisson_task(args):
    _limit_threads()
    from oracle import problems as pb
    m, n, w, F = args
    return pb.poisson_mode(m, n, w, F)


def _heat_task(args):
    _limit_threads()
    from oracle import problems as pb
    p, l, hist_l, cg_l, alpha, h, steps, order = args
    n, m = cg_l.shape

    def full(x):
        z = np.zeros((p, n, m), dtype=np.complex128)
        z[l] = x
        return z

    # heat_coeffs on the one storage index l (the other slots are never solved)
    out = pb.heat_coeffs([full(x) for x in hist_l], full(cg_l), alpha, h, steps, order=order, modes=[l])
    return out[0][l]


def workers():
    return max(1, min(15, (os.cpu_count() or 2) - 1))


def poisson_modes(cf, ls):
    """Oracle T-coefficients (n x m, as stored in cf[l]) for storage indices ls."""
    from oracle import transforms as tr
    p, n, m = cf.shape
    wn = tr.wavenumbers(p)
    tasks = [(m, n, int(wn[l]), np.ascontiguousarray(cf[l].T)) for l in ls]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers()) as pool:
        out = pool.map(_poisson_task, tasks, chunksize=1)
    return {l: U.T for l, U in zip(ls, out)}


def heat_modes(c0_full, cg_full, alpha, h, steps, ls, order=1):
    """Oracle BDF heat coefficients after `steps` steps for storage indices ls
    (c0_full: list of `order` full-coefficient history fields, newest first)."""
    p = cg_full.shape[0]
    tasks = [(p, l, [np.ascontiguousarray(c[l]) for c in c0_full], np.ascontiguousarray(cg_full[l]),
              alpha, h, steps, order) for l in ls]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers()) as pool:
        out = pool.map(_heat_task, tasks, chunksize=1)
    return dict(zip(ls, out))
