"""Shared helpers of the GPU parity tests: seeded inputs and error measures."""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import transforms as tr

S = synth.SEED_BASE
TOL = 1e-10          # relative parity tolerance for the solvers (both norms)


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def banner(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def smooth_values(m, n, p, seed):
    """Random smooth forcing (decaying CCF spectrum) as grid values, via the oracle."""
    h = synth.smooth_coeffs(m, n, p, seed)
    return tr.inverse(tr.from_half(h, p))


def rel_errors(got, ref):
    d = np.asarray(got) - np.asarray(ref)
    l2 = np.linalg.norm(d.ravel()) / max(np.linalg.norm(np.asarray(ref).ravel()), 1e-300)
    mx = np.max(np.abs(d)) / max(np.max(np.abs(ref)), 1e-300)
    return float(l2), float(mx)


def assert_close(got, ref, tol=TOL, what=""):
    l2, mx = rel_errors(got, ref)
    print("  %s rel l2 %.3e  rel max %.3e" % (what, l2, mx), flush=True)
    assert l2 <= tol and mx <= tol, (what, l2, mx)
