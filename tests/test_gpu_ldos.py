"""GPU parity of the KPM local density of states (kpm_ldos) against the
oracle (oracle/ldos.py: plain recursion moments of the unit probes, then the
damped series), through the C ABI.

* 17 x 19 with two vortices: 10 Nambu indices starting mid-lattice, M from 2
  to 257, 300 energies (two blocks, ragged) including some outside the band
  (where the density is 0 by definition); FP64 to 1e-10 of max |A|, FP32
  recursion to 1e-5;
* 100 x 100 (M = 4096): the two sites next to a vortex centre, FP64 and FP32.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import builder, ldos
from tests import helpers as H
from tests.gpu_helpers import dev, host, problem

pytestmark = pytest.mark.gpu


def _run(cfg, prec, first, count, E):
    st = H.stencil(cfg)
    a, b = H.bounds(cfg, st)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    ref, _ = ldos.ldos(Hs, a, b, first, count, cfg.M, E(a, b), cfg.Lx, cfg.Ly)
    ref = np.where(np.isfinite(ref), ref, 0.0)
    pb = problem(cfg, precision=prec)
    out = pb.ldos(dev(st), dev(np.array([a, b])), first, count, dev(E(a, b)))
    return host(out), ref


@pytest.mark.parametrize("M", [2, 64, 257])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_ldos_against_oracle(M, prec, tol):
    cfg = wl.Config("l", 17, 19, 2, 0.16, M, (wl.ProbeSpec("unit", 1),), vortex=True, complex_noise=0.02)
    a, b = H.bounds(cfg, H.stencil(cfg))

    def E(a, b):
        return np.linspace(b - 1.02 * a, b + 1.02 * a, 300)    # a few points outside the band

    got, ref = _run(cfg, prec, 2 * 150 + 1, 10, E)
    outside = np.abs((E(a, b) - b) / a) >= 1.0
    assert outside.any() and np.all(got[:, outside] == 0.0)
    inside = ~outside
    assert np.max(np.abs(got[:, inside] - ref[:, inside])) < tol * np.max(np.abs(ref[:, inside]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_ldos_fullsize_vortex_core(prec, tol):
    cfg = wl.C5(prec)
    X, Y = wl.vortex_centres(cfg.Lx, cfg.Ly, cfg.n_v)[0]
    i0 = int(Y) * cfg.Lx + int(X)

    def E(a, b):
        return np.linspace(b - 0.5 * a, b + 0.5 * a, 500)

    got, ref = _run(cfg, prec, 2 * i0, 4, E)
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref))
