"""Batched heat stepping over problems of uneven sizes.

A batch step performs, for every member, the arithmetic of cyl_heat_step in the
same order (same kernels on the same blocks, only gathered into fewer
launches), so batched members must equal twins stepped one by one bit for bit;
one member is also checked against the oracle.  The captured step graph is
replayed several times with eager work and synchronisation in between, and
every replay is checked.
"""

import numpy as np
import pytest

import paper_2206_04827_amd as cyl
from oracle import problems as pb
from tests.gpu_common import S, TOL, assert_close, banner, dev, host, need_gpu, smooth_values

pytestmark = pytest.mark.gpu

# (n_r, n_z, n_theta, bdf order, alpha): split-sweep, one-thread-per-line and
# HBM-state ADI kernels, one- and two-pass tolerances, a BDF4 member.
SPECS = [(20, 20, 8, 1, 0.7), (21, 17, 7, 1, 1.3), (48, 48, 16, 1, 0.2), (26, 40, 6, 4, 0.9),
         (66, 66, 10, 1, 1.0), (200, 200, 4, 1, 0.5), (262, 262, 4, 1, 1.7)]


def _make(specs, seed, dt=1e-3):
    out = []
    for q, (m, n, p, order, alpha) in enumerate(specs):
        plan = cyl.Plan(m, n, p)
        hist = [smooth_values(m, n, p, seed + 10 * q + i) for i in range(order)]
        g = smooth_values(m, n, p, seed + 10 * q + 9)
        out.append((plan, hist, g, order, alpha))
    return out


def _heats(probs, dt=1e-3):
    return [cyl.Heat(plan, [dev(x) for x in hist], dev(g), alpha, dt, order, 1e-12)
            for plan, hist, g, order, alpha in probs]


@pytest.mark.parametrize("graph,tune", [(True, True), (False, False)])
def test_batch_equals_individual_stepping(graph, tune):
    need_gpu()
    banner("batch vs individual graph=%s tune=%s" % (graph, tune))
    probs = _make(SPECS, S + 200)
    A = _heats(probs)
    B = _heats(probs)
    batch = cyl.Batch(A, graph=graph, tune=tune)
    info = batch.describe()
    print("  batch:", info, flush=True)
    assert info["graph"] == graph and info["launches_per_pass"] >= 1
    for rep, n in enumerate([4, 4, 5, 3]):     # whole cycles (graph replays) and eager remainders
        batch.step(n)
        for h in B:
            h.step(n)
        for q, (ha, hb) in enumerate(zip(A, B)):
            a, b = host(ha.read()), host(hb.read())
            assert np.array_equal(a, b), (rep, q, float(np.max(np.abs(a - b))))
    batch.close()


def test_batch_member_matches_oracle():
    """Small members (split, one-thread-per-line and BDF4) and a member on the
    split sweeps with the block state in global memory (n = 262) against the
    oracle after 6 batched steps."""
    need_gpu()
    banner("batch member vs oracle")
    probs = _make([SPECS[0], SPECS[3], SPECS[4], SPECS[6]], S + 300)
    A = _heats(probs)
    batch = cyl.Batch(A)
    batch.step(6)
    for (plan, hist, g, order, alpha), h in zip(probs, A):
        ref = pb.heat(hist, g, alpha, 1e-3, 6, order=order)
        assert_close(host(h.read()), ref, TOL, "batched %dx%dx%d" % plan.value_shape[::-1])


def test_member_stepped_outside_the_batch_is_rejected():
    need_gpu()
    probs = _make(SPECS[:2], S + 400)
    A = _heats(probs)
    batch = cyl.Batch(A, tune=False)
    batch.step(1)
    A[1].step(1)
    with pytest.raises(cyl.CylError) as e:
        batch.step(1)
    assert e.value.status == 1


def test_batch_rejects_bad_arguments():
    need_gpu()
    probs = _make(SPECS[:1], S + 500)
    A = _heats(probs)
    with pytest.raises(cyl.CylError):
        cyl.Batch([A[0], A[0]])


def test_b64_sizes_batch_equals_individual():
    """The largest problems of the 64-problem configuration (HBM-state and
    split ADI kernels at their real sizes) plus small ones: batched stepping
    equals stepping each problem on its own, bit for bit."""
    need_gpu()
    import synth
    specs = synth.batch_specs(S + 10)
    order = sorted(range(len(specs)), key=lambda i: -specs[i][0] * specs[i][1] * specs[i][2])
    pick = order[:3] + order[-2:]
    banner("B64 subset %s" % [specs[i] for i in pick])
    probs = []
    for i in pick:
        m, n, p, alpha = specs[i]
        T0 = synth.eigenmode_values(synth.eigenmode_params(S + 10 + i), m, n, p)
        g = smooth_values(m, n, p, S + 100 + i)
        probs.append((cyl.Plan(m, n, p), [T0], g, 1, alpha))
    A = _heats(probs)
    B = _heats(probs)
    batch = cyl.Batch(A)
    batch.step(2)
    for h in B:
        h.step(2)
    for q, (ha, hb) in enumerate(zip(A, B)):
        a, b = host(ha.read()), host(hb.read())
        assert np.array_equal(a, b), (q, float(np.max(np.abs(a - b))))


@pytest.mark.parametrize("grouping", [0, 2])
def test_work_queue_launches_equal_individual_stepping(grouping, monkeypatch):
    """Persistent work-queue launches of the split kernels (LDS and global
    state) take the same blocks through the same code: bit for bit equal to
    stepping each member alone, over graph replays."""
    need_gpu()
    banner("batch work-queue launches grouping=%d" % grouping)
    monkeypatch.setenv("CYLSPEC_BATCH_QUEUE", "1")
    monkeypatch.setenv("CYLSPEC_BATCH_GROUPING", str(grouping))
    probs = _make([SPECS[0], SPECS[2], SPECS[4], SPECS[5], SPECS[6]], S + 600)
    A = _heats(probs)
    B = _heats(probs)
    batch = cyl.Batch(A, tune=False)
    info = batch.describe()
    print("  batch:", info, flush=True)
    assert "work-queue" in info["grouping"]
    for n in (3, 2):
        batch.step(n)
        for h in B:
            h.step(n)
        for q, (ha, hb) in enumerate(zip(A, B)):
            a, b = host(ha.read()), host(hb.read())
            assert np.array_equal(a, b), (n, q, float(np.max(np.abs(a - b))))
    batch.close()


TUNE_SPECS = [(24, 24, 6, 1, 0.4), (56, 40, 8, 1, 1.1)]


def _tune_probe():
    """Create the batch of TUNE_SPECS (tuned) and print its description."""
    import json
    probs = _make(TUNE_SPECS, S + 700)
    batch = cyl.Batch(_heats(probs))
    print("PROBE " + json.dumps(batch.describe()), flush=True)


def test_tune_cache_file_is_written_and_read(tmp_path):
    """CYLSPEC_TUNE_CACHE: the first process tunes and writes its choice
    (one "signature<TAB>configuration" line, beside the entries already in
    the file; malformed lines are dropped); a second process finds it and
    does not tune again (no "batch tuned" line), with the same configuration."""
    need_gpu()
    import os
    import re
    import subprocess
    import sys
    path = tmp_path / "tune.txt"
    # a foreign entry survives, malformed lines are dropped
    path.write_text("gfx-other/1|0:8:8:4:1;\tg2q0s8\nnot a line\nkey\tg9q9s9\n")
    env = dict(os.environ, CYLSPEC_TUNE_CACHE=str(path), CYLSPEC_LOG="1")
    env.pop("CYLSPEC_BATCH_QUEUE", None)
    env.pop("CYLSPEC_BATCH_GROUPING", None)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cmd = [sys.executable, "-c", "import tests.test_gpu_batch as t; t._tune_probe()"]
    runs = [subprocess.run(cmd, cwd=root, env=env, capture_output=True, text=True, timeout=300) for _ in range(2)]
    for r in runs:
        assert r.returncode == 0, r.stderr[-2000:]
    lines = path.read_text().splitlines()
    assert "gfx-other/1|0:8:8:4:1;\tg2q0s8" in lines, lines
    ours = [l for l in lines if not l.startswith("gfx-other/")]
    assert len(lines) == 2 and len(ours) == 1, lines
    assert re.fullmatch(r"gfx\S*/\d+\|\S+\tg[012]q[01]s(8|16)", ours[0]), lines
    assert "batch tuned" in runs[0].stderr and "batch tuned" not in runs[1].stderr
    desc = [re.search(r"^PROBE (.*)$", r.stdout, re.M).group(1) for r in runs]
    assert desc[0] == desc[1]
