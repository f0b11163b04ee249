"""Density-matrix parity against the oracle's plain KPM (O2) at full size,
element by element (GPU, through the C ABI).

App. B (eq. dFdH with the beta recursion) defines rho = dOmega/dh; the oracle
stores every alpha_m and beta_m and contracts them on the stencil pairs, the
library runs the fused adjoint kernel with reversible recomputation of alpha
from checkpoints.  Both sides take their own stencil, bounds and coefficients.

* The 100 x 100 workload (two vortices, period-8 pair/charge-density seed,
  M = 4096, checkpoints every 64) with 8 dense Z4 probes of weight 1/8: the
  oracle costs seconds per probe there, so the probe count is cut, not the
  lattice or M.  One probe per wave gives two probe ranges of four probes,
  which takes the lattice-strip schedule over the 8 XCDs and the sparse-row
  adjoint loop, as the benchmark's launches do; two probes per wave give one
  range.  FP64 to 1e-10, FP32 vectors to 1e-5 (relative to max |rho|).
* The 64 x 64 workload (two vortices, doping 0.15, M = 2048) on all its 192
  probes (64 colored + 128 dense Z4, each set of weight 1/2), in the tuned
  launch configuration: FP64 to 1e-10, FP32 vectors to 1e-5.
* The 48-lattice batch (M = 1024, 64 colored probes each), FP32, replayed as
  the benchmark does (3 groups of lattices one after another, each as two
  instance halves on two streams, one graph each):
  the smallest and the largest lattice and one with four vortices, against
  O2 on all their probes, to 1e-5; and the FP64 batch (6 groups) to 1e-10.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as wl
from tests import helpers as H
from tests.gpu_helpers import host, problem, theta_dev

pytestmark = pytest.mark.gpu

C5_DENSE = (wl.ProbeSpec("dense_z4", 8, 20221299, weight=1 / 8),)


@pytest.fixture(autouse=True)
def _reset_block():
    from paper_2212_05685_amd import kpm
    yield
    kpm.kpm_set_probe_block(0)


@pytest.fixture(scope="module")
def c5_oracle():
    cfg = wl.scaled(wl.C5("fp64"), probes=C5_DENSE)
    st, a, b, C = H.oracle_inputs(cfg)
    print(f"oracle: 100x100, M={cfg.M}, {cfg.R} dense Z4 probes ...", flush=True)
    return cfg, H.plain_parallel(cfg, st, a, b, C)


@pytest.mark.parametrize("prec,P", [("fp64", 1), ("fp32", 1), ("fp32", 2)])
def test_c5_rho_against_oracle(c5_oracle, prec, P):
    from paper_2212_05685_amd import kpm
    cfg, ref = c5_oracle
    kpm.kpm_set_probe_block(P)
    p = problem(cfg, precision=prec)
    n, chi, dlt = theta_dev(cfg)
    h = p.build_H(n, chi, dlt)
    ab = p.bounds(h)
    C = p.coefficients(ab)
    om, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    assert p.status() == 0
    om, mu = host(om)[0], host(mu)
    e_om = abs(om - ref["omega"]) / abs(ref["omega"])
    e_mu = float(np.max(np.abs(mu - ref["mu"])) / np.max(np.abs(ref["mu"])))
    e_rho = H.rel_err(rho, ref["rho"])
    print(f"100x100 {prec} P={P}: |dOmega|/|Omega| = {e_om:.2e}, moments {e_mu:.2e}, "
          f"max|drho|/max|rho| = {e_rho:.2e}")
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert e_om < tol and e_mu < tol and e_rho < tol
    del p
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def c3_oracle():
    cfg = wl.C3()
    st, a, b, C = H.oracle_inputs(cfg)
    print(f"oracle: 64x64, M={cfg.M}, {cfg.R} probes ...", flush=True)
    return cfg, H.plain_parallel(cfg, st, a, b, C)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_rho_against_oracle(c3_oracle, prec):
    cfg, ref = c3_oracle
    p = problem(cfg, precision=prec)
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    C = p.coefficients(ab)
    om, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    assert p.status() == 0
    om, mu = host(om)[0], host(mu)
    e_om = abs(om - ref["omega"]) / abs(ref["omega"])
    e_mu = float(np.max(np.abs(mu - ref["mu"])) / np.max(np.abs(ref["mu"])))
    e_rho = H.rel_err(rho, ref["rho"])
    print(f"64x64 {prec}: |dOmega|/|Omega| = {e_om:.2e}, moments {e_mu:.2e}, "
          f"max|drho|/max|rho| = {e_rho:.2e}")
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert e_om < tol and e_mu < tol and e_rho < tol
    del p
    torch.cuda.empty_cache()


def _c4_pick(cfgs):
    """Indices of the smallest lattice, the largest and the first with four vortices."""
    small = min(range(len(cfgs)), key=lambda q: (cfgs[q].N, q))
    large = max(range(len(cfgs)), key=lambda q: (cfgs[q].N, -q))
    four = next(q for q in range(len(cfgs)) if cfgs[q].n_v == 4 and q not in (small, large))
    return [small, large, four]


@functools.lru_cache(maxsize=None)
def _c4_oracle(q):
    cfg = wl.C4_instances(48)[q]
    st, a, b, C = H.oracle_inputs(cfg)
    return H.plain_parallel(cfg, st, a, b, C)


@pytest.mark.parametrize("prec,groups,tol", [("fp32", 3, 1e-5), ("fp64", 6, 1e-10)])
def test_c4_batched_rho_against_oracle(prec, groups, tol):
    """FP32: 3 instance groups; FP64 (twice the bytes per record): 6."""
    from paper_2212_05685_amd import kpm
    cfgs = wl.C4_instances(48)
    probs, hs, abs_, Cs = [], [], [], []
    for cfg in cfgs:
        q = problem(cfg, precision=prec)
        h = q.build_H(*theta_dev(cfg))
        ab = q.bounds(h)
        probs.append(q)
        hs.append(h)
        abs_.append(ab)
        Cs.append(q.coefficients(ab))
    M, k = cfgs[0].M, cfgs[0].ckpt_k
    plan = kpm.kpm_batch_create([q.lat for q in probs], [q.probes for q in probs], M,
                                kpm.KPM_FP32 if prec == "fp32" else kpm.KPM_FP64, k)
    try:
        omega = torch.zeros(len(cfgs), dtype=torch.float64, device="cuda")
        rhos = [torch.zeros_like(h) for h in hs]
        assert kpm.kpm_batch_streams(plan) == 2 and kpm.kpm_batch_groups(plan) == groups
        for _ in range(2):          # tune + capture, then a replay of the graphs
            kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=True)
        om = host(omega)
        got = {q: host(rhos[q]) for q in range(len(cfgs))}
    finally:
        kpm.kpm_batch_destroy(plan)
    del probs, hs, abs_, Cs, rhos
    torch.cuda.empty_cache()
    for q in _c4_pick(cfgs):
        cfg = cfgs[q]
        ref = _c4_oracle(q)
        e_om = abs(om[q] - ref["omega"]) / abs(ref["omega"])
        e_rho = H.rel_err(got[q], ref["rho"])
        print(f"batch instance {q} ({cfg.Lx}x{cfg.Ly}, n_v={cfg.n_v}, doping {cfg.doping:.3f}, {prec}): "
              f"|dOmega|/|Omega| = {e_om:.2e}, max|drho|/max|rho| = {e_rho:.2e}")
        assert e_om < tol and e_rho < tol
