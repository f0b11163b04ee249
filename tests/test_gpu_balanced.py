"""The balanced adjoint schedule against the oracle (GPU, through the C ABI).

The balanced schedule cuts the adjoint step's (tile, probe) work into one
equal contiguous share per resident block.  A share can end inside one tile's
probes and go on with the next tile, and several blocks then add into the same
tile's partial sums through separate FP64 slices.  None of this changes what is
computed: rho = dOmega/dh is App. B's eq. dFdH with the beta recursion, up to
the order of the FP64 sums.  The cases below make shares cross tile and probe-
group boundaries in every way the split allows:
* 17 x 19 (ragged tiles), 27 probes: odd R, one probe group, shares of 8-9
  units against segments of 27, so up to 5 blocks share a tile;
* 24 x 20, 40 probes: two probe groups of 20;
* 64 x 64, 64 probes: the grid is the chip's resident block count (shares of
  10-11 units in FP32, 32 in FP64);
* the 100 x 100 workload (M = 4096, checkpoints every 64) with 16 dense Z4
  probes: shares of about 8 units in FP32 and 20 in FP64.
Each case also checks that the split applies at all (the library falls back
to the range schedule when its slices would not fit the partial-sum buffer),
from the same arithmetic as the library's, for every resident block count
from 1 to 3 per compute unit.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from tests import helpers as H
from tests.gpu_helpers import host, problem, theta_dev

pytestmark = pytest.mark.gpu


def _split(ntiles, R, G):
    """(blocks, groups, slices per group) of the balanced split, or None."""
    W = ntiles * R
    G = min(G, W // 8)
    G -= G % 8
    if G < 8:
        return None
    ng = 2 if R % 2 == 0 else 1
    Lg = R // ng
    S = max(((seg + 1) * Lg * G - 1) // W - ((seg * Lg + 1) * G - 1) // W + 1
            for seg in range(ng * ntiles))
    if ng * S > (R + 3) // 4:
        return None
    return G, ng, S


def _applies(cfg, R):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ntiles = ((cfg.Lx + 7) // 8) * ((cfg.Ly + 3) // 4)
    return all(_split(ntiles, R, bpc * cus) is not None for bpc in (1, 2, 3))


@pytest.fixture(autouse=True)
def _reset():
    from paper_2212_05685_amd import kpm
    yield
    kpm.kpm_set_probe_block(0)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, kpm.KPM_SCHED_DEFAULT)


def _run(cfg, prec):
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(4)
    kpm.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, kpm.KPM_SCHED_BALANCED)
    p = problem(cfg, precision=prec)
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    C = p.coefficients(ab)
    omega, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    assert p.status() == 0
    out = host(omega)[0], host(mu), rho, p.R
    del p
    torch.cuda.empty_cache()
    return out


def _check(cfg, prec, ref):
    om, mu, rho, R = _run(cfg, prec)
    assert _applies(cfg, R)
    tol = 1e-10 if prec == "fp64" else 1e-5
    e_om = abs(om - ref["omega"]) / abs(ref["omega"])
    e_mu = float(np.max(np.abs(mu - ref["mu"])) / np.max(np.abs(ref["mu"])))
    e_rho = H.rel_err(rho, ref["rho"])
    print(f"{cfg.Lx}x{cfg.Ly} R={R} {prec}: Omega {e_om:.1e}, moments {e_mu:.1e}, rho {e_rho:.1e}")
    assert e_om < tol and e_mu < tol and e_rho < tol


SMALL = {
    "17x19_R27": wl.Config("b1", 17, 19, 2, 0.13, 40,
                           (wl.ProbeSpec("colored_z4", 1, 77, 4, 3, 1, 0, 1.0),
                            wl.ProbeSpec("dense_z4", 3, 99, weight=1 / 3)),
                           vortex=True, complex_noise=0.02, ckpt_k=6),
    "24x20_R40": wl.Config("b2", 24, 20, 2, 0.13, 33,
                           (wl.ProbeSpec("dense_z4", 40, 5, weight=1 / 40),),
                           vortex=True, complex_noise=0.02, ckpt_k=5),
    "64x64_R64": wl.Config("b3", 64, 64, 2, 0.15, 24,
                           (wl.ProbeSpec("colored_z4", 1, 31, 8, 8, 0, 0, 1.0),),
                           vortex=True, ckpt_k=8),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", sorted(SMALL))
def test_balanced_against_oracle(name, prec):
    cfg = SMALL[name]
    st, a, b, C = H.oracle_inputs(cfg)
    _check(cfg, prec, H.plain(cfg, st, a, b, C))


C5_DENSE16 = (wl.ProbeSpec("dense_z4", 16, 20221307, weight=1 / 16),)


@pytest.fixture(scope="module")
def c5_oracle16():
    cfg = wl.scaled(wl.C5("fp64"), probes=C5_DENSE16)
    st, a, b, C = H.oracle_inputs(cfg)
    print(f"oracle: 100x100, M={cfg.M}, {cfg.R} dense Z4 probes ...", flush=True)
    return cfg, H.plain_parallel(cfg, st, a, b, C)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_balanced_c5_against_oracle(c5_oracle16, prec):
    cfg, ref = c5_oracle16
    _check(cfg, prec, ref)
