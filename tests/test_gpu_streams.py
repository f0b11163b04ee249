"""Probe halves on two streams against the oracle (GPU, through the C ABI).

With kpm_set_streams(2) a single-lattice call runs its probes as two halves,
each an instance over its share of the probe-indexed buffers (vectors, code
table, weights, checkpoints, moment partials, partial-sum slices), their
recursions on two streams; Omega, the moments and rho are reduced over both
halves.  What is computed is unchanged (App. B: the moments, eq. alpha; rho =
dOmega/dh, eq. dFdH with the beta recursion), up to the order of sums.  The
cases cover an odd probe count (halves of 14 and 13 probes, so the second
half starts inside a colored group and inside the dense group), probe blocks
that give one or several probe ranges per half, the balanced adjoint split
inside a half, the moments entry point, a repeated gradient after one
forward (the checkpoints of both halves rebuild their last alpha pair), and
the 100 x 100 workload, where the automatic setting splits.
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


@pytest.fixture(autouse=True)
def _reset():
    from paper_2212_05685_amd import kpm
    yield
    kpm.kpm_set_streams(0)
    kpm.kpm_set_probe_block(0)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, kpm.KPM_SCHED_DEFAULT)


def _cfg():
    probes = (wl.ProbeSpec("colored_z4", 1, 77, 4, 3, 1, 0, 1.0),
              wl.ProbeSpec("dense_z4", 3, 99, weight=1 / 3))
    return wl.Config("s", 17, 19, 2, 0.13, 40, probes, "fp64", vortex=True, complex_noise=0.02, ckpt_k=6)


@functools.lru_cache(maxsize=None)
def _oracle():
    cfg = _cfg()
    st, a, b, C = H.oracle_inputs(cfg)
    return H.plain(cfg, st, a, b, C)


def _run(cfg, prec, grads=1):
    p = problem(cfg, precision=prec)
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    C = p.coefficients(ab)
    omega, mu = p.grand_potential(h, ab, C, want_mu=True)
    rhos = [host(p.grand_potential_grad(h, ab, C)) for _ in range(grads)]
    assert p.status() == 0
    return host(omega)[0], host(mu), rhos


def _check(om, mu, rho, ref, tol):
    assert abs(om - ref["omega"]) < tol * abs(ref["omega"])
    assert np.max(np.abs(mu - ref["mu"])) < tol * np.max(np.abs(ref["mu"]))
    assert H.rel_err(rho, ref["rho"]) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("P,sa", [(1, -1), (2, -1), (4, 4), (32, -1)])
def test_halves_against_oracle(prec, P, sa):
    from paper_2212_05685_amd import kpm
    cfg = _cfg()
    assert problem(cfg).R == 27
    kpm.kpm_set_streams(2)
    kpm.kpm_set_probe_block(P)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, sa)
    om, mu, (rho,) = _run(cfg, prec)
    _check(om, mu, rho, _oracle(), TOL if prec == "fp64" else TOL32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_halves_match_one_stream(prec):
    from paper_2212_05685_amd import kpm
    cfg = _cfg()
    kpm.kpm_set_probe_block(2)
    kpm.kpm_set_streams(1)
    om1, mu1, (rho1,) = _run(cfg, prec)
    kpm.kpm_set_streams(2)
    om2, mu2, (rho2,) = _run(cfg, prec)
    # the moments are computed probe by probe in the same order either way
    assert np.array_equal(mu1, mu2)
    # the halves group the probes into other ranges (0-7, 8-13 | 14-21, 22-26
    # against 0-7, 8-15, 16-23, 24-26), so the FP64 partial sums of rho are
    # added in another order: evidence that the call did split
    assert not np.array_equal(rho1, rho2)
    tol = 1e-14 if prec == "fp64" else 1e-7
    assert abs(om1 - om2) <= tol * abs(om1)
    assert H.rel_err(rho2, rho1) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_halves_repeated_gradient(prec):
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_streams(2)
    kpm.kpm_set_probe_block(2)
    _, _, rhos = _run(_cfg(), prec, grads=3)
    assert np.array_equal(rhos[0], rhos[1]) and np.array_equal(rhos[0], rhos[2])


def test_halves_moments_entry_point():
    from paper_2212_05685_amd import kpm
    cfg = _cfg()
    kpm.kpm_set_streams(2)
    p = problem(cfg, precision="fp64")
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    mu = host(p.moments(h, ab))
    ref = _oracle()
    assert np.max(np.abs(mu - ref["mu"])) < TOL * np.max(np.abs(ref["mu"]))


def test_halves_tuned_as_pair(tmp_path, monkeypatch):
    """Automatic block: the first energy evaluation tunes the halves as a pair
    (each candidate timed on both halves at once); the cache file gets one
    line, keyed by the whole lattice's shape followed by "/2"; a second
    evaluation reuses the pick; results match the oracle."""
    from paper_2212_05685_amd import kpm
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KPM_TUNE_CACHE", str(path))
    kpm.kpm_set_streams(2)
    kpm.kpm_set_probe_block(0)
    cfg = _cfg()
    props = torch.cuda.get_device_properties(0)
    key = f"{props.gcnArchName.split(':')[0]}:{props.multi_processor_count}:d:{cfg.Lx * cfg.Ly}x27/2"
    for _ in range(2):
        om, mu, (rho,) = _run(cfg, "fp64")
        _check(om, mu, rho, _oracle(), TOL)
        lines = [ln.split() for ln in path.read_text().splitlines()]
        assert [ln[0] for ln in lines] == [key]


def test_set_streams_returns_previous_and_ignores_bad_values():
    from paper_2212_05685_amd import kpm
    assert kpm.kpm_set_streams(2) == 0
    assert kpm.kpm_set_streams(7) == 2
    assert kpm.kpm_set_streams(-1) == 2
    assert kpm.kpm_set_streams(1) == 2
    assert kpm.kpm_set_streams(0) == 1


C5_DENSE = (wl.ProbeSpec("dense_z4", 8, 20221299, weight=1 / 8),)


@pytest.fixture(scope="module")
def c5_oracle():
    cfg = wl.scaled(wl.C5("fp64"), probes=C5_DENSE)
    st, a, b, C = H.oracle_inputs(cfg)
    print(f"oracle: 100x100, M={cfg.M}, {cfg.R} dense Z4 probes ...", flush=True)
    return cfg, H.plain_parallel(cfg, st, a, b, C)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_halves_c5_against_oracle(c5_oracle, prec):
    """The 100 x 100 workload (M = 4096, checkpoints every 64) with 8 dense
    probes as two halves of 4, one probe per wave."""
    from paper_2212_05685_amd import kpm
    cfg, ref = c5_oracle
    kpm.kpm_set_streams(2)
    kpm.kpm_set_probe_block(1)
    om, mu, (rho,) = _run(cfg, prec)
    e = H.rel_err(rho, ref["rho"])
    print(f"100x100 {prec} halves: max|drho|/max|rho| = {e:.2e}")
    _check(om, mu, rho, ref, TOL if prec == "fp64" else TOL32)
    torch.cuda.empty_cache()
