"""Benchmark: value-space Poisson solve on the 256^3 CCF grid in FP64.

One step = one whole solve through the hot path: forward transform (theta DFT,
z and r DCT-I), tau right-hand side, ADI over every parity block of every
Fourier mode, recombination and inverse transform.  Input: seeded random
smooth forcing with a decaying CCF spectrum, resident in HBM before timing.
ADI tolerance 1e-10 (the 512^3 configuration's); the solution's relative
error against the oracle on the sampled wavenumbers is reported under
'accuracy' (bar: 1e-10).

Prints one JSON line.  Besides the headline value it carries:
  roofline      the ADI kernel's algorithmic FP64 rate (66 flop per interior
                unknown per iteration) against the vector FP64 peak, from HIP
                events recorded around every ADI launch on the plan's stream
                inside the timed region, and its HBM traffic by counters;
  roofline_model
                the whole solve against the streaming model (each ADI
                half-step one HBM round trip);
  cpu_baseline  the CPU oracle timed on the same solve (all wavenumbers):
                per-mode solves spread over worker processes, and on one core;
  heat_128      forward BDF1 heat steps per second on the 128^3 grid;
  heat_fwd_adjoint_192
                forward + adjoint BDF1 heat steps per second at 192^3: 200
                steps, alpha = 1, dt = 1e-3, checkpoint every 20 steps, loss
                |T_N - T_target|^2, gradients for T0, g and alpha;
  batched_64    64 independent BDF1 heat problems of uneven sizes (n_r = n_z
                in 48..384, n_theta in 32..256, alpha in [0.1, 2]), 50 steps:
                batched launches with a replayed step graph against stepping
                each problem on its own;
  physical_256  the same 256^3 solve for a physical forcing (a smooth
                function of x, y, z): the physical-parity fast path (the
                j = w mod 2 blocks only) against the general solve of the
                same input;
  disk_poisson_256
                the horizontal (disk) Poisson solve Delta_h u = f of
                Section 4 on the same grid and forcing (transforms plus one
                banded r-solve per wavenumber and z coefficient), with the
                solve kernel's algorithmic bandwidth;
  pt_decompose_256
                the poloidal-toroidal decomposition of Section 4 of a seeded
                three-component field on the same grid (three forward
                transforms, two disk solves, two inverse transforms).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Poisson unknowns/sec at 256³ FP64 (rel err≤1e-10); "
          "heat fwd+adjoint steps/sec")
FP64_PEAK_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# Algorithmic FP64 operations per interior unknown per ADI iteration (the
# streamlined passes of Algorithm 1): r-pass C W (6 diagonals), - E, the
# (u C - A) LU solve (2 + 3 diagonals and a reciprocal), (v C - A) Y (6), + E
# and the C solve (2 + 3): about 50; z-pass (v B + D)^-1 (lower 2, upper 1)
# and (u' B + D) (4 diagonals): about 16.
ADI_FLOPS_PER_UNKNOWN_ITER = 66.0
# The kernel's own formulation needs fewer (reported beside): r-pass 24 (one
# banded product and one LU solve after eliminating the half-step), z-pass 14.
ADI_KERNEL_FLOPS_PER_UNKNOWN_ITER = 38.0
# Algorithmic FP64 operations per unknown of the residual
# R = E - (A X B + C X D) with the parity-split bands A (1,2), C (2,3),
# B (2,1), D (1,0): A X then (.) B, C X then (.) D (16 FMA), two subtractions.
RESIDUAL_FLOPS_PER_UNKNOWN = 34.0
# Streaming model of the solve (each ADI half-step one trip through HBM):
# bytes per unknown per ADI iteration, and per solve for the transforms, the
# right side and the recombination (8 passes of 16 B).
STREAM_BYTES_PER_UNKNOWN_ITER = 40.0
STREAM_PASS_BYTES = 8 * 16.0
# HBM bytes per ADI launch at 256^3 (mean of the two passes, the first also
# forming the residual) from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by
# copy kernels reading and writing 512 MiB: fetch x2.0, write x1.0),
# valid for the ADI source whose SHA-256 starts with ADI_TRAFFIC_SHA, at ADI
# tolerance ADI_TRAFFIC_TOL (the traffic scales with the iteration count);
# reported as null otherwise.
ADI_TRAFFIC_BYTES_256 = 2.353e9
ADI_TRAFFIC_SHA = "9ba3d375f39dbe70"
ADI_TRAFFIC_TOL = 1e-10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-10,
                    help="ADI tolerance of the headline solve (the 512^3 configuration's; the "
                         "measured error against the oracle is reported under 'accuracy')")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-heat", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-reps", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-physical", action="store_true")
    ap.add_argument("--no-disk", action="store_true")
    ap.add_argument("--no-pt", action="store_true", help="skip the poloidal-toroidal decomposition leg")
    ap.add_argument("--no-small", action="store_true", help="skip the 32^3 latency leg")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="worker processes of the all-core CPU oracle leg (capped by the CPU count)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain elementwise kernel reading 512 MiB and writing "
                         "512 MiB (a known-size kernel for scaling FETCH_SIZE / WRITE_SIZE "
                         "counters)")
    return ap.parse_args()


def _oracle_mode(args):
    """One wavenumber of the oracle's Poisson solve, BLAS/LAPACK on one thread
    (runs in a worker process of the CPU baseline)."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    from threadpoolctl import threadpool_limits
    from oracle import problems as pb
    m, n, w, F = args
    with threadpool_limits(limits=1):
        return pb.poisson_mode(m, n, w, F)


def _warm(_):
    """Import the oracle in a worker before the timed map."""
    from threadpoolctl import threadpool_limits  # noqa: F401
    from oracle import problems  # noqa: F401
    return os.getpid()


def cpu_baseline(m, n, p, seed, workers, u_gpu=None):
    """Time the oracle (numpy/scipy, as it stands) on the whole solve.

    The forward and inverse transforms run in this process; the per-mode
    solves of all p wavenumbers run (a) in `workers` single-threaded worker
    processes (the value) and (b) here on one thread (single_thread).  With
    u_gpu (the GPU solution of the timed loop, host array) also returns its
    relative error against the oracle over all wavenumbers."""
    import multiprocessing as mp
    import numpy as np
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import problems as pb
    from oracle import transforms as tr
    workers = max(1, min(workers, os.cpu_count() or 1))
    h = synth.smooth_coeffs(m, n, p, seed)
    f = tr.inverse(tr.from_half(h, p))
    t0 = time.perf_counter()
    c = tr.forward(f)
    t_fwd = time.perf_counter() - t0
    wn = tr.wavenumbers(p)
    tasks = [(m, n, int(wn[l]), np.ascontiguousarray(c[l].T)) for l in range(p)]
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_warm, range(4 * workers), chunksize=1)     # workers started, oracle imported
        t0 = time.perf_counter()
        res = pool.map(_oracle_mode, tasks, chunksize=1)
        t_pool = time.perf_counter() - t0
    U = np.stack([x.T for x in res])
    t0 = time.perf_counter()
    tr.inverse(U)
    t_inv = time.perf_counter() - t0
    t_all = t_fwd + t_pool + t_inv
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        U1 = pb.poisson_coeffs(c)
        t_one = time.perf_counter() - t0
    t1 = t_fwd + t_one + t_inv
    assert np.array_equal(U1, U)
    acc = None
    if u_gpu is not None:
        got = tr.forward(u_gpu)
        num = float(np.linalg.norm((got - U).ravel()))
        den = float(np.linalg.norm(U.ravel()))
        mx = float(np.max(np.abs(got - U)) / np.max(np.abs(U)))
        acc = {"rel_l2": num / den, "rel_max": mx, "bar": 1e-10, "wavenumbers": "all %d" % p,
               "reference": "oracle per-mode Bartels-Stewart solves of the cpu_baseline run"}
    single = {"value": m * n * p / t1, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
              "sample": ("the whole %d^3 solve on one core: transforms plus the per-mode solves of "
                         "all %d wavenumbers with BLAS/LAPACK on one thread; %.2f s") % (m, p, t1)}
    return acc, {"value": m * n * p / t_all, "unit": "unknowns/s", "cores": int(workers), "kind": "oracle",
                 "sample": ("the whole %d^3 Poisson solve (no extrapolation): forward and inverse "
                            "transforms in one process (%.2f s), per-mode Bartels-Stewart + 2 "
                            "extended-precision refinements of all %d wavenumbers in %d single-threaded "
                            "worker processes (%.2f s)") % (m, t_fwd + t_inv, p, workers, t_pool),
                 "single_thread": single}


def heat_fwd_adjoint(cyl, torch, synth, reps, size=192, steps=200, every=20):
    """Forward + adjoint of a BDF1 heat run (gradients w.r.t. T0, g, alpha)."""
    m = n = p = size
    S = synth.SEED_BASE
    pl = cyl.Plan(m, n, p)
    T0 = torch.from_numpy(synth.eigenmode_values(synth.eigenmode_params(S + 5), m, n, p)).cuda()
    g = pl.transform_inv(torch.from_numpy(synth.smooth_coeffs(m, n, p, S + 6)).cuda())
    Tt = pl.transform_inv(torch.from_numpy(synth.smooth_coeffs(m, n, p, S + 7)).cuda())
    H = cyl.Heat(pl, [T0], g, 1.0, 1e-3, 1, 1e-12)
    G = cyl.HeatGrad(H, steps, every)

    def one():
        G.forward()
        TN = H.read()
        return G.backward(2.0 * (TN - Tt))

    one()                                  # warm-up (first launches)
    torch.cuda.synchronize()
    pl.set_profiling(True)
    pl.profile()
    t_fwd = t_all = 0.0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        TN = H.read()
        T0b, gb, ab = G.backward(2.0 * (TN - Tt))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_fwd += t1 - t0
        t_all += t2 - t0
    prof = pl.profile()
    pl.set_profiling(False)
    # plain forward run of the same problem (no checkpoints) for comparison
    H2 = cyl.Heat(pl, [T0], g, 1.0, 1e-3, 1, 1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H2.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    nseg = (steps + every - 1) // every
    res = {"steps_per_s": steps * reps / t_all, "ms_per_fwd_adjoint_run": 1e3 * t_all / reps,
           "ms_forward_part": 1e3 * t_fwd / reps, "ms_backward_part": 1e3 * (t_all - t_fwd) / reps,
           "plain_forward_steps_per_s": steps / t_plain,
           "heat_solves_per_run": {"forward": steps, "recompute": steps - min(every, steps),
                                   "transposed": steps},
           "config": {"workload": "heat_bdf1_%d^3_fwd_adjoint" % size, "steps": steps,
                      "checkpoint_every": every, "checkpoints": nseg, "alpha": 1.0, "dt": 1e-3,
                      "adi_tol": 1e-12, "loss": "sum (T_N - T_target)^2",
                      "gradients": ["T0", "g", "alpha"]},
           "alpha_grad": float(ab),
           "phase_ms_per_run": {k[3:]: round(prof[k] / reps, 3) for k in prof if k.startswith("ms_")}}
    G.close()
    H.close()
    H2.close()
    pl.close()
    return res


def batched_heat(cyl, torch, synth, count, steps):
    """64 uneven BDF1 heat problems: per-problem stepping vs one batch."""
    S = synth.SEED_BASE
    specs = synth.batch_specs(S + 10, count=count)
    t0 = time.perf_counter()
    plans, heats = [], []
    for i, (m, n, p, alpha) in enumerate(specs):
        pl = cyl.Plan(m, n, p)
        T0 = torch.from_numpy(synth.eigenmode_values(synth.eigenmode_params(S + 10 + i), m, n, p)).cuda()
        g = pl.transform_inv(torch.from_numpy(synth.smooth_coeffs(m, n, p, S + 100 + i)).cuda())
        heats.append(cyl.Heat(pl, [T0], g, alpha, 1e-3, 1, 1e-12))
        plans.append(pl)
        del T0, g
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    for h in heats:
        h.step(1)                              # warm-up: first launches of every size
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h in heats:
        h.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = cyl.Batch(heats)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    batch.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    info = batch.describe()
    unknowns = sum(m * n * p for m, n, p, _ in specs)
    res = {"problem_steps_per_s": count * steps / t_batch, "ms_per_batched_step": 1e3 * t_batch / steps,
           "plain_problem_steps_per_s": count * steps / t_plain, "plain_ms_per_step_all": 1e3 * t_plain / steps,
           "speedup_vs_plain": t_plain / t_batch, "unknowns_per_step": unknowns,
           "unknowns_per_s": unknowns * steps / t_batch,
           "launches_per_adi_pass": info["launches_per_pass"], "graph": info["graph"],
           "grouping": info["grouping"], "setup_s": t_setup, "batch_create_s": t_create,
           "config": {"workload": "batched_heat_%d_uneven" % count, "problems": count, "steps": steps,
                      "n_r=n_z": [min(s[0] for s in specs), max(s[0] for s in specs)],
                      "n_theta": [min(s[2] for s in specs), max(s[2] for s in specs)],
                      "alpha": [0.1, 2.0], "dt": 1e-3, "bdf": 1, "adi_tol": 1e-12}}
    batch.close()
    for h in heats:
        h.close()
    for pl in plans:
        pl.close()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single device (sharding the "
              "Fourier modes across GPUs is not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2206_04827_amd as cyl
    import synth

    torch.cuda.set_device(0)
    m = n = p = args.size
    plan = cyl.Plan(m, n, p)
    coeff = torch.from_numpy(synth.smooth_coeffs(m, n, p, synth.SEED_BASE + 3)).cuda()
    f = plan.transform_inv(coeff)          # forcing values on the grid, resident in HBM
    u = torch.empty_like(f)
    # one untimed solve with the residual check (builds the shift tables)
    _, info = plan.poisson_solve(f, adi_tol=args.tol, out=u, info=True)
    for _ in range(args.warmup):
        plan.poisson_solve(f, adi_tol=args.tol, out=u)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    plan.profile()                         # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.poisson_solve(f, adi_tol=args.tol, out=u)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile()
    plan.set_profiling(False)
    u_head = u.clone()                     # the timed loop's solution (for the accuracy check)
    ms_step = 1e3 * elapsed / args.steps
    value = m * n * p * args.steps / elapsed

    n_adi = max(1, prof["n_adi"])
    adi_ms = prof["ms_adi"] / n_adi
    passes = info["passes"]
    fused = bool(info["fused_residual"])
    interior = (m - 2) * (n - 2) * p
    flops_per_launch = interior * (ADI_FLOPS_PER_UNKNOWN_ITER * info["adi_iterations_mean"] +
                                   (RESIDUAL_FLOPS_PER_UNKNOWN / passes if fused else 0.0))
    kernel_flops = interior * ADI_KERNEL_FLOPS_PER_UNKNOWN_ITER * info["adi_iterations_mean"]
    achieved = flops_per_launch / (adi_ms * 1e-3) / 1e12
    import hashlib
    src = os.path.join(ROOT, "paper_2206_04827_amd", "csrc", "adi.hip")
    with open(src, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    traffic = (ADI_TRAFFIC_BYTES_256 if (sha == ADI_TRAFFIC_SHA and m == 256 and passes == 2
                                         and args.tol == ADI_TRAFFIC_TOL) else None)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_adi_split (one ADI pass over all parity blocks%s)" %
                          (", the first also forming the residual" if fused else ""),
                "avg_launch_ms": round(adi_ms, 4), "launches": n_adi,
                "flop_per_unknown_iter": ADI_FLOPS_PER_UNKNOWN_ITER,
                "kernel_formulation_tflops": round(kernel_flops / (adi_ms * 1e-3) / 1e12, 3),
                "hbm_gbs_from_counters": (round(traffic / (adi_ms * 1e-3) / 1e9, 1) if traffic else None),
                "hbm_frac_from_counters": (round(traffic / (adi_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                           if traffic else None)}
    phases = {k[3:]: round(prof[k] / args.steps, 4) for k in prof if k.startswith("ms_")}

    # the device's own peaks (FP64 FMA chains, streaming copy), measured next
    # to the vendor figures the fractions are quoted against
    peaks = cyl.device_peaks()
    roofline["measured_peak"] = round(peaks["fp64_tflops"], 2)
    roofline["frac_of_measured_peak"] = round(achieved / peaks["fp64_tflops"], 4)
    # the whole solve against the streaming model of the same iterations: each
    # ADI half-step one HBM round trip (40 B per unknown per iteration: r-pass
    # reads W and E and writes Z, z-pass reads Z and writes W) plus eight
    # transform / right-side / recombination passes of 16 B per unknown; the
    # FP64 term at 66 flop per unknown per iteration
    n_unk = float(m * n * p)
    j_total = passes * info["adi_iterations_mean"]
    b_stream = (STREAM_BYTES_PER_UNKNOWN_ITER * j_total + STREAM_PASS_BYTES) * n_unk
    f_adi = ADI_FLOPS_PER_UNKNOWN_ITER * j_total * n_unk
    t_model = max(b_stream / (HBM_PEAK_GBS * 1e9), f_adi / (FP64_PEAK_TFLOPS * 1e12))
    model = {"model": "streaming ADI (40 B per unknown per iteration) + 8 passes x 16 B per unknown",
             "iterations": round(j_total, 2), "bytes": b_stream, "t_model_ms": round(1e3 * t_model, 4),
             "t_measured_ms": round(ms_step, 4), "speed_vs_streaming_model": round(1e3 * t_model / ms_step, 4),
             "frac_vs_measured_copy": round(1e3 * b_stream / (peaks["copy_gbs"] * 1e9) / ms_step, 4),
             "fp64_frac_of_solve": round(f_adi / (ms_step * 1e-3 * FP64_PEAK_TFLOPS * 1e12), 4)}

    out = {"metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "poisson_%d^3_value_space" % m, "n_r": m, "n_z": n, "n_theta": p,
                      "adi_tol": args.tol, "adi_passes": passes,
                      "adi_iterations_mean_per_pass": info["adi_iterations_mean"],
                      "forcing": "seeded decaying random CCF spectrum",
                      "parallelism": "single GPU"},
           "resid_ratio": info["resid_ratio"], "phase_ms_per_step": phases,
           "roofline": roofline, "roofline_model": model,
           "device_peaks": {"fp64_tflops": round(peaks["fp64_tflops"], 2), "copy_gbs": round(peaks["copy_gbs"], 1),
                            "copy_bytes_per_launch": peaks["copy_bytes"],
                            "vendor_fp64_tflops": FP64_PEAK_TFLOPS, "vendor_hbm_gbs": HBM_PEAK_GBS}}

    if not args.no_physical:
        fp = torch.from_numpy(synth.physical_values(m, n, p, synth.SEED_BASE + 4)).cuda()
        legs = {}
        for phys in (False, True):
            plan.set_physical(phys)
            _, pinfo = plan.poisson_solve(fp, adi_tol=args.tol, out=u, info=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                plan.poisson_solve(fp, adi_tol=args.tol, out=u)
            torch.cuda.synchronize()
            legs[phys] = (1e3 * (time.perf_counter() - t0) / args.steps, pinfo["resid_ratio"])
        plan.set_physical(False)
        out["physical_256"] = {"ms_per_solve": legs[True][0], "unknowns_per_s": m * n * p / (legs[True][0] * 1e-3),
                               "general_ms_per_solve": legs[False][0],
                               "speedup_vs_general": legs[False][0] / legs[True][0],
                               "resid_ratio": legs[True][1],
                               "config": {"workload": "poisson_%d^3_physical_forcing" % m,
                                          "forcing": "seeded smooth function of x, y, z",
                                          "adi_tol": args.tol}}
        del fp

    if not args.no_disk:
        plan.disk_poisson_solve(f, out=u)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        plan.profile()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.disk_poisson_solve(f, out=u)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        dp = plan.profile()
        plan.set_profiling(False)
        kms = dp["ms_adi"] / max(1, dp["n_adi"])
        # read f, write and re-read the forward sweep, write u: 4 x 16 B per complex coefficient
        dbytes = 64.0 * (p // 2 + 1) * n * m
        out["disk_poisson_256"] = {"ms_per_solve": ms, "unknowns_per_s": m * n * p / (ms * 1e-3),
                                   "kernel": "k_disk", "kernel_ms": kms,
                                   "kernel_bytes": dbytes, "kernel_gbs": dbytes / (kms * 1e-3) / 1e9,
                                   "kernel_hbm_frac": dbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                   "transforms_ms": (dp["ms_transform_fwd"] + dp["ms_transform_inv"]) / args.steps,
                                   "config": {"workload": "disk_poisson_%d^3_value_space" % m,
                                              "forcing": "seeded decaying random CCF spectrum"}}

    if not args.no_pt:
        # poloidal-toroidal decomposition of a seeded field (three components)
        vr, vt = plan.transform_inv(coeff), f
        vz = plan.transform_inv(torch.from_numpy(synth.smooth_coeffs(m, n, p, synth.SEED_BASE + 6)).cuda())
        lam, gam = torch.empty_like(f), torch.empty_like(f)
        plan.pt_decompose(vr, vt, vz, out=(lam, gam))
        torch.cuda.synchronize()
        plan.set_profiling(True)
        plan.profile()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.pt_decompose(vr, vt, vz, out=(lam, gam))
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        pp_ = plan.profile()
        plan.set_profiling(False)
        out["pt_decompose_%d" % m] = {
            "ms_per_call": ms, "unknowns_per_s": m * n * p / (ms * 1e-3),
            "disk_solves_ms": pp_["ms_adi"] / args.steps,
            "transforms_ms": (pp_["ms_transform_fwd"] + pp_["ms_transform_inv"]) / args.steps,
            "config": {"workload": "pt_decomposition_%d^3_value_space" % m,
                       "field": "three seeded decaying random CCF spectra"}}
        del vr, vz, lam, gam

    if not args.no_small:
        # the smallest configuration (32^3, ADI tolerance 1e-12): bound by the
        # latency of the ADI's sequential iterations; eager solves and the
        # same solve captured once into a HIP graph and replayed
        ms_ = ns_ = ps_ = 32
        s32 = torch.cuda.Stream()
        with torch.cuda.stream(s32):
            plan32 = cyl.Plan(ms_, ns_, ps_, stream=s32)
            f32 = plan32.transform_inv(torch.from_numpy(synth.smooth_coeffs(ms_, ns_, ps_, synth.SEED_BASE)).cuda())
            u32 = torch.empty_like(f32)
            _, info32 = plan32.poisson_solve(f32, adi_tol=1e-12, out=u32, info=True)
            s32.synchronize()
            reps = 200
            t0 = time.perf_counter()
            for _ in range(reps):
                plan32.poisson_solve(f32, adi_tol=1e-12, out=u32)
            s32.synchronize()
            eager_us = 1e6 * (time.perf_counter() - t0) / reps
            # phase breakdown (HIP events around every phase; a separate,
            # untimed loop since the events add host work)
            plan32.set_profiling(True)
            plan32.profile()
            for _ in range(20):
                plan32.poisson_solve(f32, adi_tol=1e-12, out=u32)
            pr32 = plan32.profile()
            plan32.set_profiling(False)
            phases32 = {k[3:]: round(1e3 * pr32[k] / 20, 2) for k in pr32 if k.startswith("ms_") and pr32[k] > 0}
        g32 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g32, stream=s32):
            plan32.poisson_solve(f32, adi_tol=1e-12, out=u32)
        g32.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g32.replay()
        torch.cuda.synchronize()
        graph_us = 1e6 * (time.perf_counter() - t0) / reps
        out["poisson_32"] = {"us_per_solve": eager_us, "solves_per_s": 1e6 / eager_us,
                             "unknowns_per_s": ms_ * ns_ * ps_ * 1e6 / eager_us,
                             "graph_us_per_solve": graph_us, "phase_us_per_solve": phases32,
                             "adi_iterations_max": info32["J_max"],
                             "resid_ratio": info32["resid_ratio"],
                             "config": {"workload": "poisson_32^3_value_space", "adi_tol": 1e-12}}
        del plan32, g32

    if not args.no_heat:
        hp = cyl.Plan(128, 128, 128)
        prm = synth.eigenmode_params(synth.SEED_BASE + 1)
        T0 = torch.from_numpy(synth.eigenmode_values(prm, 128, 128, 128)).cuda()
        gc = torch.from_numpy(synth.smooth_coeffs(128, 128, 128, synth.SEED_BASE + 2)).cuda()
        g = hp.transform_inv(gc)
        H = cyl.Heat(hp, [T0], g, 1.0, 1e-3, 1, 1e-12)
        H.step(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.step(100)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        out["heat_128"] = {"steps_per_s": 100 / th, "ms_per_step": 1e3 * th / 100,
                           "note": "forward BDF1 steps only"}
        H.close()
        if not args.no_physical:
            # physical initial state (the eigenmodes are) and physical forcing
            gp = torch.from_numpy(synth.physical_values(128, 128, 128, synth.SEED_BASE + 5)).cuda()
            rates = {}
            for phys in (False, True):
                hp.set_physical(phys)
                Hp = cyl.Heat(hp, [T0], gp, 1.0, 1e-3, 1, 1e-12)
                Hp.step(5)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Hp.step(100)
                torch.cuda.synchronize()
                rates[phys] = 100 / (time.perf_counter() - t0)
                Hp.close()
            hp.set_physical(False)
            out["heat_128_physical"] = {"steps_per_s": rates[True], "general_steps_per_s": rates[False],
                                        "speedup_vs_general": rates[True] / rates[False],
                                        "config": {"workload": "heat_bdf1_128^3_physical",
                                                   "initial": "seeded Bessel x sine eigenmodes",
                                                   "forcing": "seeded smooth function of x, y, z"}}
        hp.close()

    if not args.no_adjoint:
        out["heat_fwd_adjoint_192"] = heat_fwd_adjoint(cyl, torch, synth, args.adjoint_reps)

    if not args.no_batch:
        print("bench: batched heat leg", file=sys.stderr, flush=True)
        out["batched_64"] = batched_heat(cyl, torch, synth, args.batch_count, args.batch_steps)

    if args.calibrate_copy:
        a = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.add(a, 1.0, out=b)           # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = a.numel() * 8

    if not args.no_cpu_baseline:
        print("bench: CPU oracle leg", file=sys.stderr, flush=True)
        acc, out["cpu_baseline"] = cpu_baseline(m, n, p, synth.SEED_BASE + 3, args.cpu_workers,
                                                u_gpu=u_head.cpu().numpy())
        out["accuracy"] = acc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
