"""Batch plans as two instance halves on two streams, against the oracle
(GPU, through the C ABI).

With kpm_set_streams(2) at plan creation (or automatically, from
sum R N >= 2^19 site-probes) a batch plan splits its instances into two
halves of nearly equal R N, each with its own kernel tables and tuning; their
recursions run side by side on the caller's stream and on a second stream,
with interleaved step launches, or as one graph per half.  What each instance
computes is unchanged (App. B: eq. alpha for the moments, eq. F_KPM for
Omega, eq. dFdH with the beta recursion for rho).  The cases: three uneven
lattices (halves of two instances and one; the one-instance half takes the
single-lattice tile arithmetic and, when asked, the balanced adjoint split),
direct launches and graph replays, FP64 and FP32, fixed probe blocks with
several schedules and the automatic block (each half tuned as its own shape);
the split plan reproduces the one-stream plan bit for bit at a fixed block;
graph replays repeat bit for bit; and the automatic rule.  Instance groups
(kpm_batch_groups: groups of lattices run one after another, each sized to
the Infinity Cache) likewise.  The 48-lattice batch against the oracle
(tests/test_gpu_fullsize_oracle.py) runs as 3 groups, each split.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as wl
from tests import helpers as H
from tests.gpu_helpers import host, problem, theta_dev

pytestmark = pytest.mark.gpu

M, K = 40, 5


def _cfg(Lx, Ly, nv, probes):
    return wl.Config("bs", Lx, Ly, nv, 0.13, M, tuple(probes), "fp64", vortex=nv > 0, complex_noise=0.02,
                     ckpt_k=K)


CFGS = [
    _cfg(16, 16, 4, (wl.ProbeSpec("colored_z4", 1, 71, 4, 4, 1, 0, 1.0),)),
    _cfg(9, 7, 2, (wl.ProbeSpec("colored_z4", 1, 77, 4, 3, 1, 0, 1.0),
                   wl.ProbeSpec("dense_z4", 3, 99, weight=1 / 3))),
    _cfg(12, 10, 2, (wl.ProbeSpec("dense_z4", 24, 5, weight=1 / 24),)),
]


@pytest.fixture(autouse=True)
def _reset():
    from paper_2212_05685_amd import kpm
    yield
    kpm.kpm_set_streams(0)
    kpm.kpm_set_batch_groups(0)
    kpm.kpm_set_probe_block(0)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, kpm.KPM_SCHED_DEFAULT)


@functools.lru_cache(maxsize=None)
def _oracle(q):
    cfg = CFGS[q]
    st, a, b, C = H.oracle_inputs(cfg)
    return H.plain(cfg, st, a, b, C)


@functools.lru_cache(maxsize=None)
def _inputs(prec):
    probs, hs, abs_, Cs = [], [], [], []
    for cfg in CFGS:
        p = problem(cfg, precision=prec)
        h = p.build_H(*theta_dev(cfg))
        ab = p.bounds(h)
        probs.append(p)
        hs.append(h)
        abs_.append(ab)
        Cs.append(p.coefficients(ab))
    return probs, hs, abs_, Cs


def _plan(prec, streams, groups=0):
    from paper_2212_05685_amd import kpm
    probs = _inputs(prec)[0]
    kpm.kpm_set_streams(streams)
    kpm.kpm_set_batch_groups(groups)
    plan = kpm.kpm_batch_create([q.lat for q in probs], [q.probes for q in probs], M,
                                kpm.KPM_FP64 if prec == "fp64" else kpm.KPM_FP32, K)
    kpm.kpm_set_streams(0)
    kpm.kpm_set_batch_groups(0)
    return plan


def _call(plan, prec, use_graph):
    from paper_2212_05685_amd import kpm
    _, hs, abs_, Cs = _inputs(prec)
    omega = torch.zeros(len(CFGS), dtype=torch.float64, device="cuda")
    rhos = [torch.zeros_like(h) for h in hs]
    kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=use_graph)
    return host(omega), [host(r) for r in rhos]


def _check_oracle(om, rhos, prec):
    tol = 1e-10 if prec == "fp64" else 1e-5
    for q in range(len(CFGS)):
        ref = _oracle(q)
        assert abs(om[q] - ref["omega"]) < tol * abs(ref["omega"])
        assert H.rel_err(rhos[q], ref["rho"]) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("P,sa", [(4, -1), (2, 2), (1, 4), (0, -1)], ids=["P4", "P2strips", "P1bal", "auto"])
def test_halves_against_oracle(prec, P, sa):
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(P)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, sa)
    plan = _plan(prec, 2)
    try:
        assert kpm.kpm_batch_streams(plan) == 2
        for use_graph in (False, True, True):
            om, rhos = _call(plan, prec, use_graph)
            _check_oracle(om, rhos, prec)
        tune = kpm.kpm_batch_tuning(plan)
        assert tune["source"] == ("fixed" if P else "timed") or (P == 0 and tune["source"] != "fixed")
    finally:
        kpm.kpm_batch_destroy(plan)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_halves_match_one_stream_bitwise(prec):
    """At a fixed probe block and schedule an instance's kernels and sums do
    not depend on the other instances, so the split plan's results equal the
    one-stream plan's bit for bit, and graph replays repeat them."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(2)
    one, two = _plan(prec, 1), _plan(prec, 2)
    try:
        assert kpm.kpm_batch_streams(one) == 1 and kpm.kpm_batch_streams(two) == 2
        om1, r1 = _call(one, prec, False)
        runs = [_call(two, prec, g) for g in (False, True, True, True)]
    finally:
        kpm.kpm_batch_destroy(one)
        kpm.kpm_batch_destroy(two)
    for om2, r2 in runs:
        assert np.array_equal(om1, om2)
        assert all(np.array_equal(a, b) for a, b in zip(r1, r2))


def test_automatic_rule():
    from paper_2212_05685_amd import kpm
    for streams, want in ((0, 1), (1, 1), (2, 2)):
        plan = _plan("fp32", streams)
        try:
            assert kpm.kpm_batch_streams(plan) == want
        finally:
            kpm.kpm_batch_destroy(plan)
    # the 48 uneven lattices (7.2e6 site-probes) and their first 4 (7.1e5)
    # split automatically, their first 3 (5.1e5 < 2^19) do not; a plan of
    # one lattice never does
    cfgs = wl.C4_instances(48)
    probs = [problem(c, precision="fp32") for c in cfgs]
    rn = lambda n: sum(q.R * c.N for q, c in zip(probs[:n], cfgs[:n]))
    assert rn(3) < 2 ** 19 <= rn(4)
    for n, streams, want in ((48, 0, 2), (48, 1, 1), (4, 0, 2), (3, 0, 1), (1, 2, 1)):
        kpm.kpm_set_streams(streams)
        plan = kpm.kpm_batch_create([q.lat for q in probs[:n]], [q.probes for q in probs[:n]], cfgs[0].M,
                                    kpm.KPM_FP32, cfgs[0].ckpt_k)
        kpm.kpm_set_streams(0)
        try:
            assert kpm.kpm_batch_streams(plan) == want
        finally:
            kpm.kpm_batch_destroy(plan)
    torch.cuda.empty_cache()


def _key(probs, fp32):
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    inst = ",".join(f"{q.lat.Lx * q.lat.Ly}x{q.R}" for q in probs)
    return f"{arch}:{props.multi_processor_count}:{'f' if fp32 else 'd'}:{inst}/2"


def test_pair_tuning_cache(tmp_path, monkeypatch):
    """Automatic block: the halves are tuned as a pair (each candidate timed on
    both halves at once), one line "<key of all instances>/2" goes to the cache
    file, both halves take its pick, and a second plan of the shape reuses it
    from the process cache.  The lattices in reverse order: a shape no other
    test of this process has tuned."""
    from paper_2212_05685_amd import kpm
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KPM_TUNE_CACHE", str(path))
    kpm.kpm_set_probe_block(0)
    probs, hs, abs_, Cs = (x[::-1] for x in _inputs("fp64"))
    key = _key(probs, False)
    picks = []
    for source in ("timed", "process cache"):
        kpm.kpm_set_streams(2)
        plan = kpm.kpm_batch_create([q.lat for q in probs], [q.probes for q in probs], M, kpm.KPM_FP64, K)
        kpm.kpm_set_streams(0)
        try:
            assert kpm.kpm_batch_streams(plan) == 2
            omega = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
            rhos = [torch.zeros_like(h) for h in hs]
            kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=True)
            om, rh = host(omega)[::-1], [host(r) for r in rhos][::-1]
            tune = kpm.kpm_batch_tuning(plan)
        finally:
            kpm.kpm_batch_destroy(plan)
        assert tune["source"] == source
        _check_oracle(om, rh, "fp64")
        picks.append([tune["fwd_probe_block"], tune["fwd_schedule"], tune["adj_probe_block"],
                      tune["adj_schedule"]])
        lines = [ln.split() for ln in path.read_text().splitlines()]
        assert [ln[0] for ln in lines] == [key]
        assert [int(v) for v in lines[0][1:]] == picks[0]
    assert picks[0] == picks[1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("groups,streams", [(2, 1), (2, 2), (3, 2)])
def test_groups(prec, groups, streams):
    """Instance groups run one after another (forced here: the 16 x 16 lattice
    alone and the other two together, or one group per lattice), with and
    without instance halves inside a group: every instance matches the oracle,
    and at a fixed probe block the results equal the one-group one-stream
    plan's bit for bit, in direct launches and graph replays."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(2)
    one = _plan(prec, 1, 1)
    plan = _plan(prec, streams, groups)
    try:
        assert kpm.kpm_batch_groups(one) == 1 and kpm.kpm_batch_groups(plan) == groups
        # a group of two lattices splits into halves when asked; single-lattice groups cannot
        assert kpm.kpm_batch_streams(plan) == (2 if streams == 2 and groups == 2 else 1)
        om1, r1 = _call(one, prec, False)
        runs = [_call(plan, prec, g) for g in (False, True, True)]
    finally:
        kpm.kpm_batch_destroy(one)
        kpm.kpm_batch_destroy(plan)
    _check_oracle(*runs[0], prec)
    for om2, r2 in runs:
        assert np.array_equal(om1, om2)
        assert all(np.array_equal(a, b) for a, b in zip(r1, r2))


def test_group_rule():
    """Automatic groups: as many as keep each group's adjoint working set
    (6 x 16 B (FP32) or 32 B (FP64) x sum R N) within 240 MB: the 48 uneven
    lattices (7.2e6 site-probes) in 3 groups in FP32 and 6 in FP64; their
    first 3 lattices in one."""
    from paper_2212_05685_amd import kpm
    cfgs = wl.C4_instances(48)
    probs = [problem(c, precision="fp32") for c in cfgs]
    rn = sum(q.R * c.N for q, c in zip(probs, cfgs))
    want = {kpm.KPM_FP32: -(-6 * 16 * rn // 240_000_000), kpm.KPM_FP64: -(-6 * 32 * rn // 240_000_000)}
    assert want == {kpm.KPM_FP32: 3, kpm.KPM_FP64: 6}
    for n, prec in ((48, kpm.KPM_FP32), (48, kpm.KPM_FP64), (3, kpm.KPM_FP32)):
        plan = kpm.kpm_batch_create([q.lat for q in probs[:n]], [q.probes for q in probs[:n]], cfgs[0].M,
                                    prec, cfgs[0].ckpt_k)
        try:
            assert kpm.kpm_batch_groups(plan) == (want[prec] if n == 48 else 1)
        finally:
            kpm.kpm_batch_destroy(plan)
    torch.cuda.empty_cache()
