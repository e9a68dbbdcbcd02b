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


def half_slots(p):
    """(slot, storage index) pairs of the Hermitian half: slot w >= 0 holds
    wavenumber w, except that for even p the slot p/2 holds w = -p/2."""
    out = []
    for w in range(p // 2 + 1):
        wn = -w if (p % 2 == 0 and w == p // 2) else w
        out.append((w, wn + p // 2))
    return out


def assert_slots_close(got_half, ref_by_l, p, tol=TOL, what=""):
    """Compare every Hermitian-half slot of got_half (nw x n x m complex) with
    the oracle's full-coefficient modes ref_by_l[storage index] (n x m), in both
    norms over all slots, and print the worst slot."""
    num = den = 0.0
    dmax = rmax = 0.0
    worst = (0.0, None)
    for w, l in half_slots(p):
        d = got_half[w] - ref_by_l[l]
        num += float(np.sum(np.abs(d) ** 2))
        den += float(np.sum(np.abs(ref_by_l[l]) ** 2))
        dmax = max(dmax, float(np.max(np.abs(d))))
        rmax = max(rmax, float(np.max(np.abs(ref_by_l[l]))))
        e = float(np.linalg.norm(d)) / max(float(np.linalg.norm(ref_by_l[l])), 1e-300)
        if e >= worst[0]:
            worst = (e, w)
    l2 = (num / den) ** 0.5
    mx = dmax / rmax
    print("  %s all %d slots rel l2 %.3e rel max %.3e (worst slot w=%s: %.3e)"
          % (what, p // 2 + 1, l2, mx, worst[1], worst[0]), flush=True)
    assert l2 <= tol and mx <= tol, (what, l2, mx)
