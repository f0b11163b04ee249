"""Kernel configuration choices against the oracle, through the C ABI.

Every block schedule of the recursion kernels (tile-major, probe ranges per
XCD, strips per XCD, strips tile by tile, and the balanced adjoint split) must
give the same energy, moments and density matrix: the schedule only permutes
(tile, probe) work over blocks, and so reorders FP64 sums at most (App. B,
eqs. alpha and dFdH).  The batch
autotuner times (probe block, schedule) pairs, remembers its picks per shape
in the process and in a text file, and a plan configured from that file
computes the same results as single lattices.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as wl
from tests import helpers as H
from tests.gpu_helpers import host, problem, theta_dev

pytestmark = pytest.mark.gpu

TOL = 1e-10
TOL32 = 1e-5


def _cfg(Lx=17, Ly=19, nv=2, M=40, k=6, probes=None):
    probes = probes or (wl.ProbeSpec("colored_z4", 1, 77, 4, 3, 1, 0, 1.0),
                        wl.ProbeSpec("dense_z4", 3, 99, weight=1 / 3))
    return wl.Config("t", Lx, Ly, nv, 0.13, M, tuple(probes), "fp64", vortex=nv > 0,
                     complex_noise=0.02, ckpt_k=k)


@functools.lru_cache(maxsize=None)
def _oracle(Lx, Ly, nv, M, k):
    cfg = _cfg(Lx, Ly, nv, M, k)
    st, a, b, C = H.oracle_inputs(cfg)
    return H.plain(cfg, st, a, b, C)


@pytest.fixture(autouse=True)
def _reset():
    from paper_2212_05685_amd import kpm
    yield
    kpm.kpm_set_probe_block(0)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, kpm.KPM_SCHED_DEFAULT)


def _single(cfg, prec, P, sf, sa):
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(P)
    kpm.kpm_set_schedule(sf, sa)
    p = problem(cfg, precision=prec)
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    C = p.coefficients(ab)
    omega, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    assert p.status() == 0
    return host(omega)[0], host(mu), rho


SCHEDS = [(sf, sa) for sf in (0, 1, 2, 3) for sa in (0, 1, 2, 3, 4)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sf,sa", SCHEDS, ids=[f"f{a}a{b}" for a, b in SCHEDS])
def test_schedules_against_oracle(prec, sf, sa):
    """17x19 (ragged tiles), 27 probes, probe block 2: 4 probe ranges, so the
    per-XCD range schedule runs as requested."""
    cfg = _cfg()
    om, mu, rho = _single(cfg, prec, 2, sf, sa)
    ref = _oracle(17, 19, 2, 40, 6)
    tol = TOL if prec == "fp64" else TOL32
    assert abs(om - ref["omega"]) < tol * abs(ref["omega"])
    assert np.max(np.abs(mu - ref["mu"])) < tol * np.max(np.abs(ref["mu"]))
    assert H.rel_err(rho, ref["rho"]) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_range_schedule_falls_back_when_ranges_do_not_divide_8(prec):
    """Probe block 1: 7 probe ranges, which the range schedule cannot spread
    over 8 XCDs; the launch falls back to tile-major."""
    cfg = _cfg()
    om, mu, rho = _single(cfg, prec, 1, 1, 1)
    ref = _oracle(17, 19, 2, 40, 6)
    tol = TOL if prec == "fp64" else TOL32
    assert abs(om - ref["omega"]) < tol * abs(ref["omega"])
    assert H.rel_err(rho, ref["rho"]) < tol


def test_set_schedule_rejects_bad_values():
    from paper_2212_05685_amd import kpm
    for bad in ((5, 0), (0, -2), (7, 7)):
        with pytest.raises(RuntimeError):
            kpm.kpm_set_schedule(*bad)


def _key(cfgs, M, k, fp32):
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    inst = ",".join(f"{c.Lx * c.Ly}x{problem(c).R}" for c in cfgs)
    return f"{arch}:{props.multi_processor_count}:{'f' if fp32 else 'd'}:{inst}"


def _batch(cfgs, M, k, prec):
    from paper_2212_05685_amd import kpm
    probs = [problem(c, precision=prec) for c in cfgs]
    hs, abs_, Cs = [], [], []
    for q, c in zip(probs, cfgs):
        h = q.build_H(*theta_dev(c))
        hs.append(h)
        abs_.append(q.bounds(h))
        Cs.append(q.coefficients(abs_[-1]))
    plan = kpm.kpm_batch_create([q.lat for q in probs], [q.probes for q in probs], M,
                                kpm.KPM_FP64 if prec == "fp64" else kpm.KPM_FP32, k)
    try:
        omega = torch.zeros(len(cfgs), dtype=torch.float64, device="cuda")
        rhos = [torch.zeros_like(h) for h in hs]
        kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=True)
        tune = kpm.kpm_batch_tuning(plan)
        return host(omega), [host(r) for r in rhos], tune
    finally:
        kpm.kpm_batch_destroy(plan)


def _check_against_oracle(cfgs, M, k, om, rhos, tol):
    for c, o, r in zip(cfgs, om, rhos):
        st, a, b, C = H.oracle_inputs(c)
        ref = H.plain(c, st, a, b, C)
        assert abs(o - ref["omega"]) < tol * abs(ref["omega"])
        assert H.rel_err(r, ref["rho"]) < tol


def test_batch_tuner_disk_cache(tmp_path, monkeypatch):
    """First plan of a shape: timed, picks written to the cache file.  Second
    plan of that shape: this process's cache.  A shape whose line was written
    into the file beforehand: the file's picks, including a schedule the tuner
    would not pick by itself, with results still matching the oracle."""
    from paper_2212_05685_amd import kpm
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KPM_TUNE_CACHE", str(path))
    M, k = 33, 4
    cfgs = [_cfg(9, 7, 2, M, k), _cfg(13, 11, 4, M, k)]
    om, rhos, tune = _batch(cfgs, M, k, "fp64")
    assert tune["source"] == "timed"
    key = _key(cfgs, M, k, False)
    lines = [ln.split() for ln in path.read_text().splitlines()]
    mine = [ln for ln in lines if ln[0] == key]
    assert len(mine) == 1
    assert [int(v) for v in mine[0][1:]] == [tune["fwd_probe_block"], tune["fwd_schedule"],
                                            tune["adj_probe_block"], tune["adj_schedule"]]
    _check_against_oracle(cfgs, M, k, om, rhos, TOL)
    om2, rhos2, tune2 = _batch(cfgs, M, k, "fp64")
    assert tune2["source"] == "process cache"
    assert {k2: tune2[k2] for k2 in tune2 if k2 != "source"} == {k2: tune[k2] for k2 in tune if k2 != "source"}
    np.testing.assert_allclose(om2, om, rtol=1e-13)

    # a shape this process has not seen, configured by a hand-written line
    # (after one that does not parse and one with a value out of range)
    cfgs3 = [_cfg(10, 9, 2, M, k), _cfg(17, 6, 2, M, k)]
    key3 = _key(cfgs3, M, k, True)
    with open(path, "a") as f:
        f.write("garbage line\n")
        f.write(f"{key3} 3 0 2 2\n")
        f.write(f"{key3} 4 0 2 2\n")
    om3, rhos3, tune3 = _batch(cfgs3, M, k, "fp32")
    assert tune3["source"] == "disk cache"
    assert (tune3["fwd_probe_block"], tune3["fwd_schedule"], tune3["adj_probe_block"],
            tune3["adj_schedule"]) == (4, 0, 2, 2)
    _check_against_oracle(cfgs3, M, k, om3, rhos3, TOL32)


def test_batch_tuning_fixed_block():
    """With the probe block fixed the plan is not tuned and reports it."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(4)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_TILE_MAJOR, kpm.KPM_SCHED_STRIPS)
    M, k = 21, 4
    cfgs = [_cfg(8, 8, 2, M, k), _cfg(11, 5, 2, M, k)]
    om, rhos, tune = _batch(cfgs, M, k, "fp64")
    assert tune == {"fwd_probe_block": 4, "fwd_schedule": 0, "adj_probe_block": 4, "adj_schedule": 2,
                    "source": "fixed"}
    _check_against_oracle(cfgs, M, k, om, rhos, TOL)


def test_single_lattice_tuned_on_first_forward(tmp_path, monkeypatch):
    """Automatic probe block: the first energy evaluation of a shape tunes it
    (one line in the cache file, for that one-instance shape), later calls
    reuse the pick, and the energy, moments and gradient match the oracle."""
    from paper_2212_05685_amd import kpm
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KPM_TUNE_CACHE", str(path))
    kpm.kpm_set_probe_block(0)
    cfg = _cfg(15, 13, 2, 37, 5)
    key = _key([cfg], 37, 5, False)
    ref = None
    for rep in range(2):
        p = problem(cfg, precision="fp64")
        h = p.build_H(*theta_dev(cfg))
        ab = p.bounds(h)
        C = p.coefficients(ab)
        omega, mu = p.grand_potential(h, ab, C, want_mu=True)
        rho = host(p.grand_potential_grad(h, ab, C))
        if ref is None:
            ref = _oracle(15, 13, 2, 37, 5)
        assert abs(host(omega)[0] - ref["omega"]) < TOL * abs(ref["omega"])
        assert np.max(np.abs(host(mu) - ref["mu"])) < TOL * np.max(np.abs(ref["mu"]))
        assert H.rel_err(rho, ref["rho"]) < TOL
        lines = [ln.split() for ln in path.read_text().splitlines()]
        assert [ln[0] for ln in lines].count(key) == 1
