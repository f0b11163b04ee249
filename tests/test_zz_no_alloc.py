"""kpm_moments_noalloc (static scratch, no allocation) against kpm_moments on
the same inputs, through the C ABI: two calls in a row, the second on a
smaller lattice with fewer probes, in both precisions; the smaller case also
against the oracle's plain recursion (FP64 1e-10, FP32 1e-5 relative to the
largest moment).  A problem beyond the scratch is rejected with nothing
enqueued."""
import numpy as np
import pytest
import torch

import workloads as wl
from tests import helpers as H
from tests.gpu_helpers import host, problem, theta_dev

pytestmark = pytest.mark.gpu


def _cfg(Lx, Ly, nv, M, probes):
    return wl.Config("na", Lx, Ly, nv, 0.13, M, probes, "fp64", vortex=nv > 0, complex_noise=0.02)


BIG = _cfg(40, 36, 2, 300, (wl.ProbeSpec("colored_z4", 1, 41, 8, 8, 1, 0, 1.0),
                            wl.ProbeSpec("dense_z4", 5, 43, weight=0.2)))
SMALL = _cfg(9, 7, 2, 64, (wl.ProbeSpec("colored_z4", 1, 47, 3, 3, 0, 0, 1.0),))


def _both(cfg, prec):
    from paper_2212_05685_amd import kpm
    p = problem(cfg, precision=prec)
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    mu = torch.full((p.R, cfg.M), np.nan, dtype=torch.float64, device="cuda")
    kpm.kpm_moments_noalloc(p.lat, h, ab, p.probes, cfg.M, p.precision, mu)
    got = host(mu).copy()
    ref = host(p.moments(h, ab))
    assert p.status() == 0
    return got, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_workspace_call_twice(prec):
    tol = 1e-10 if prec == "fp64" else 1e-5
    for cfg in (BIG, SMALL):
        got, ref = _both(cfg, prec)
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    st, a, b, C = H.oracle_inputs(SMALL)
    orc = H.plain(SMALL, st, a, b, C, want_grad=False)["mu"]
    assert np.max(np.abs(got - orc)) < tol * np.max(np.abs(orc))


def test_noalloc_rejects_too_large():
    from paper_2212_05685_amd import kpm
    cfg = wl.C5("fp32")
    p = problem(cfg, precision="fp32")
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    mu = torch.full((p.R, cfg.M), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_noalloc(p.lat, h, ab, p.probes, cfg.M, p.precision, mu)
    assert e.value.status == kpm.KPM_ETOOBIG
    assert bool((mu == 7.0).all().item())
