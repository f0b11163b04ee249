"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Tolerances: FP64 form |dOmega|/|Omega| <= 1e-10 and max|d rho|/max|rho| <=
1e-10 (the same bar for moments relative to mu_0); the FP32 recursion 1e-5
against the same FP64 oracle; element-wise kernels
(builder, VJP, bounds, coefficients) to 1e-12 relative or better.  Sizes span
several 256-site chunks with a ragged tail, several probe blocks with a
ragged last block, checkpoint intervals from 2 to 64 and M down to 2.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import builder, chebyshev, mapping
from tests import helpers as H
from tests.gpu_helpers import dev, host, problem, theta_dev

pytestmark = pytest.mark.gpu

TOL = 1e-10
TOL32 = 1e-5     # FP32 recursion against the FP64 oracle


def _cfg(Lx=17, Ly=19, nv=2, M=48, probes=None, **kw):
    probes = probes or (wl.ProbeSpec("colored_z4", 1, 77, 4, 3, 1, 0, 1.0),
                        wl.ProbeSpec("dense_z4", 3, 99, weight=1 / 3))
    base = dict(vortex=nv > 0, complex_noise=0.02, ckpt_k=5)
    base.update(kw)
    return wl.Config("p", Lx, Ly, nv, 0.13, M, tuple(probes), "fp64", **base)


@pytest.fixture(autouse=True)
def _reset_block():
    from paper_2212_05685_amd import kpm
    yield
    kpm.kpm_set_probe_block(0)


@pytest.mark.parametrize("cfg", [wl.C1(), _cfg(), _cfg(12, 10, 4, pdw=0.02)], ids=["C1", "17x19", "12x10nv4"])
def test_build_h_and_bounds(cfg):
    p = problem(cfg)
    n, chi, dlt = theta_dev(cfg)
    h = p.build_H(n, chi, dlt)
    ref = H.stencil(cfg)
    got = host(h)
    assert np.max(np.abs(got - ref)) < 1e-13
    ab = host(p.bounds(h))
    a, b = H.bounds(cfg, ref)
    assert abs(ab[0] - a) < 1e-14 * a and abs(ab[1] - b) < 1e-14 * a


def test_build_vjp():
    cfg = _cfg(9, 7, 2)
    p = problem(cfg)
    n, chi, dlt = wl.make_theta(cfg)
    rng = np.random.default_rng(5)
    rho = rng.normal(size=(19, cfg.N)) + 1j * rng.normal(size=(19, cfg.N))
    rho[16:18] = rho[16:18].real
    gn, gc, gd = p.build_H_vjp(dev(n), dev(chi), dev(dlt), dev(rho))
    rn, rc, rd = builder.build_vjp(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt, rho)
    assert H.rel_err(host(gn), rn) < 1e-12
    assert H.rel_err(host(gc), rc) < 1e-12
    assert H.rel_err(host(gd), rd) < 1e-12


@pytest.mark.parametrize("M", [2, 3, 256, 4096])
def test_coefficients(M):
    cfg = wl.C1()
    p = problem(cfg, M=M)
    ab = dev(np.array([2.61, 0.013]))
    C = host(p.coefficients(ab))
    ref = chebyshev.kpm_coefficients(M, cfg.T, 2.61, 0.013)
    assert np.max(np.abs(C - ref)) < 1e-12 * np.max(np.abs(ref))


def _run_forward(cfg, prec="fp64", P=0, M=None, ckpt_k=None):
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(P)
    p = problem(cfg, precision=prec, M=M, ckpt_k=ckpt_k)
    n, chi, dlt = theta_dev(cfg)
    h = p.build_H(n, chi, dlt)
    ab = p.bounds(h)
    C = p.coefficients(ab)
    return p, h, ab, C


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16, 32])
def test_moments_fp64_probe_blocks(P):
    cfg = _cfg()
    p, h, ab, C = _run_forward(cfg, P=P)
    mu = host(p.moments(h, ab))
    st, a, b, Cref = H.oracle_inputs(cfg)
    ref = H.plain(cfg, st, a, b, Cref, want_grad=False)["mu"]
    assert mu.shape == ref.shape
    assert np.max(np.abs(mu - ref)) < TOL * np.max(np.abs(ref))


@pytest.mark.parametrize("M,k,P", [(2, 2, 4), (3, 2, 1), (4, 3, 2), (48, 5, 4), (64, 64, 8), (33, 2, 16),
                                   (257, 2, 8)])
def test_energy_grad_fp64(M, k, P):
    """Checkpoint intervals 2 (every adjoint step at an anchor) to 64."""
    cfg = _cfg(M=M, ckpt_k=k)
    p, h, ab, C = _run_forward(cfg, P=P)
    omega, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    st, a, b, Cref = H.oracle_inputs(cfg)
    ref = H.plain(cfg, st, a, b, Cref)
    om = host(omega)[0]
    assert abs(om - ref["omega"]) < TOL * abs(ref["omega"])
    assert np.max(np.abs(host(mu) - ref["mu"])) < TOL * np.max(np.abs(ref["mu"]))
    assert H.rel_err(rho, ref["rho"]) < TOL
    assert p.status() == 0


def _stencil_run(cfg, st, P=0, prec=None, tol=TOL):
    """Energy, moments and gradient of an arbitrary stencil on the GPU and in the
    oracle (each side computes its own bounds and coefficients)."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(P)
    p = problem(cfg, precision=prec)
    h = dev(st)
    ab = p.bounds(h)
    C = p.coefficients(ab)
    omega, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    a, b = H.bounds(cfg, st)
    ref = H.plain(cfg, st, a, b, H.coefficients(cfg, a, b))
    assert abs(host(omega)[0] - ref["omega"]) < tol * abs(ref["omega"])
    assert np.max(np.abs(host(mu) - ref["mu"])) < tol * np.max(np.abs(ref["mu"]))
    assert H.rel_err(rho, ref["rho"]) < tol
    assert p.status() == 0


def _random_stencil(cfg, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    st = scale * (rng.normal(size=(19, cfg.N)) + 1j * rng.normal(size=(19, cfg.N)))
    st[16:18] = st[16:18].real
    return st


@pytest.mark.parametrize("P", [2, 8])
def test_general_stencil_full_rows(P):
    """Every one of the 19 stencil entries nonzero: on-site and next-nearest-
    neighbour anomalous entries included (the full-row kernels)."""
    cfg = _cfg(M=40, ckpt_k=6)
    _stencil_run(cfg, _random_stencil(cfg, 11), P)


@pytest.mark.parametrize("P", [2, 8])
def test_general_stencil_full_rows_fp32(P):
    """The FP32 recursion (its own kernels: full rows here) against the FP64
    oracle at the FP32 form's tolerance, 1e-5 relative."""
    cfg = _cfg(M=40, ckpt_k=6)
    _stencil_run(cfg, _random_stencil(cfg, 11), P, prec="fp32", tol=TOL32)


@pytest.mark.parametrize("M,k,P", [(2, 2, 4), (3, 2, 1), (4, 3, 2), (5, 2, 8), (48, 5, 4), (33, 2, 16),
                                   (40, 6, 32), (257, 2, 32), (40, 3, 8)])
def test_energy_grad_fp32(M, k, P):
    """FP32 recursion, FP64 reductions: Omega, moments and rho against the FP64
    oracle to 1e-5 relative, over step counts of both parities, checkpoint
    intervals down to 2 (every launch next to an anchor or storing one), probe
    blocks from 1 to 32 (ragged last waves: 27 probes) and a ragged tile edge."""
    cfg = _cfg(M=M, ckpt_k=k)
    p, h, ab, C = _run_forward(cfg, prec="fp32", P=P)
    omega, mu = p.grand_potential(h, ab, C, want_mu=True)
    rho = host(p.grand_potential_grad(h, ab, C))
    st, a, b, Cref = H.oracle_inputs(cfg)
    ref = H.plain(cfg, st, a, b, Cref)
    assert abs(host(omega)[0] - ref["omega"]) < TOL32 * abs(ref["omega"])
    assert np.max(np.abs(host(mu) - ref["mu"])) < TOL32 * np.max(np.abs(ref["mu"]))
    assert H.rel_err(rho, ref["rho"]) < TOL32
    assert p.status() == 0


def test_mixed_sparse_and_full_rows_fp32():
    """As below, in the FP32 recursion, whose adjoint has separate sparse-row
    and full-row loops."""
    cfg = _cfg(M=40, ckpt_k=6)
    st = H.stencil(cfg).copy()
    rnd = _random_stencil(cfg, 12, 0.05)
    for i in (0, 37, 200, cfg.N - 1):
        for e in (9, 10, 13, 14, 18):
            st[e, i] = rnd[e, i]
    _stencil_run(cfg, st, prec="fp32", tol=TOL32)


def test_mixed_sparse_and_full_rows():
    """The model's stencil with anomalous next-nearest-neighbour and on-site
    entries added on a few sites only: some waves of a launch take the sparse
    rows, the others the full rows."""
    cfg = _cfg(M=40, ckpt_k=6)
    st = H.stencil(cfg).copy()
    rnd = _random_stencil(cfg, 12, 0.05)
    for i in (0, 37, 200, cfg.N - 1):
        for e in (9, 10, 13, 14, 18):           # nnn (i a, j b != a) and on-site (i0, i1)
            st[e, i] = rnd[e, i]
    _stencil_run(cfg, st)


def test_c1_exact_trace_against_dense():
    cfg = wl.C1()
    p, h, ab, C = _run_forward(cfg)
    out = p.density_matrix(h, ab, C)
    st, a, b, Cref = H.oracle_inputs(cfg)
    om, rho = H.dense_truncated(cfg, st, a, b, Cref)
    assert abs(host(out["omega"])[0] - om) < TOL * abs(om)
    r = host(out["rho"])
    assert H.rel_err(r, rho) < TOL
    # particle-hole pin at the truncation: rho_{i1,i1} + rho_{i2,i2} = g_1 (b = 0)
    assert host(ab)[1] == 0.0
    assert np.allclose(r[16].real + r[17].real, np.cos(np.pi / (cfg.M + 1)), atol=1e-12)
    op = mapping.order_parameters(r)
    for key in ("n_up", "n_dn", "chi_up", "chi_dn", "delta_up", "delta_dn"):
        assert np.max(np.abs(host(out[key]) - op[key])) < 1e-13, key


def test_fp32_form_against_fp64_form():
    cfg = _cfg(24, 20, 2, M=512, ckpt_k=64,
               probes=(wl.ProbeSpec("colored_z4", 2, 5, 8, 8, 1, 0, 0.5),))
    res = {}
    for prec in ("fp64", "fp32"):
        p, h, ab, C = _run_forward(cfg, prec=prec)
        om = host(p.grand_potential(h, ab, C))[0]
        rho = host(p.grand_potential_grad(h, ab, C))
        res[prec] = (om, rho)
    e_om = abs(res["fp32"][0] - res["fp64"][0]) / abs(res["fp64"][0])
    e_rho = H.rel_err(res["fp32"][1], res["fp64"][1])
    print(f"FP32 form vs FP64 form: |dOmega|/|Omega| = {e_om:.2e}, max|drho|/max|rho| = {e_rho:.2e}")
    assert e_om < 1e-5 and e_rho < 1e-5


def test_bounds_violation_is_reported():
    cfg = _cfg(M=64)
    p, h, ab, C = _run_forward(cfg)
    bad = ab.clone()
    bad[0] = ab[0] * 0.5             # spectrum no longer inside [-1, 1]
    p.grand_potential(h, bad, C)
    from paper_2212_05685_amd import kpm
    assert p.status() == kpm.KPM_EBOUNDS
    p.grand_potential(h, ab, C)
    assert p.status() == 0


def test_deterministic():
    cfg = _cfg(M=40)
    p, h, ab, C = _run_forward(cfg)
    o1 = host(p.grand_potential(h, ab, C)).copy()
    r1 = host(p.grand_potential_grad(h, ab, C)).copy()
    o2 = host(p.grand_potential(h, ab, C))
    r2 = host(p.grand_potential_grad(h, ab, C))
    assert np.array_equal(o1, o2) and np.array_equal(r1, r2)


def test_grad_requires_forward():
    from paper_2212_05685_amd import kpm
    cfg = _cfg(M=16)
    p, h, ab, C = _run_forward(cfg)
    with pytest.raises(kpm.KpmError) as e:
        p.grand_potential_grad(h, ab, C)
    assert e.value.status == kpm.KPM_EWORKSPACE


@pytest.mark.parametrize("prec,M,k", [("fp64", 40, 8), ("fp64", 2, 2), ("fp64", 3, 2),
                                      ("fp64", 65, 64), ("fp32", 257, 64), ("fp32", 47, 4)])
def test_grad_twice_after_one_forward(prec, M, k):
    """A second adjoint after one forward call (a second backward pass) must
    give the same rho: the first adjoint ran the alpha ping-pong down to
    alpha_0, alpha_1, and the repeated call rebuilds alpha_{M-2}, alpha_{M-1}
    from the last checkpoint pair.  Both equal the oracle's rho."""
    cfg = _cfg(M=M, ckpt_k=k)
    p, h, ab, C = _run_forward(cfg, prec=prec)
    om = host(p.grand_potential(h, ab, C))[0]
    r1 = host(p.grand_potential_grad(h, ab, C)).copy()
    r2 = host(p.grand_potential_grad(h, ab, C)).copy()
    r3 = host(p.grand_potential_grad(h, ab, C))
    assert p.status() == 0
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    st, a, b, Cref = H.oracle_inputs(cfg, M=M)
    ref = H.plain(cfg, st, a, b, Cref)
    tol = TOL if prec == "fp64" else 1e-5
    assert abs(om - ref["omega"]) < tol * abs(ref["omega"])
    assert H.rel_err(r2, ref["rho"]) < tol


def test_autograd_backward_twice():
    """torch.autograd.grad twice on one graph (retain_graph) and a backward
    after a second forward on the same problem give the first gradients."""
    from paper_2212_05685_amd.autograd import GrandPotential
    cfg = _cfg(8, 8, 2, M=70, ckpt_k=8, probes=(wl.ProbeSpec("colored_z4", 1, 3, 4, 4, 1, 0, 1.0),))
    p = problem(cfg)
    th = [x.requires_grad_(True) for x in theta_dev(cfg)]
    om = GrandPotential.apply(*th, p)
    g1 = [host(g).copy() for g in torch.autograd.grad(om, th, retain_graph=True)]
    g2 = [host(g).copy() for g in torch.autograd.grad(om, th, retain_graph=True)]
    # another forward on the same problem (its workspace now holds other checkpoints)
    th_b = [x.detach().clone().requires_grad_(True) for x in th]
    with torch.no_grad():
        th_b[0] += 1e-3
    om_b = GrandPotential.apply(*th_b, p)
    g3 = [host(g).copy() for g in torch.autograd.grad(om, th, retain_graph=True)]
    gb = [host(g) for g in torch.autograd.grad(om_b, th_b)]
    for a_, b_, c_ in zip(g1, g2, g3):
        assert np.array_equal(a_, b_) and np.array_equal(a_, c_)
    assert max(H.rel_err(x, y) for x, y in zip(gb, g1)) > 1e-8   # a different point


@pytest.mark.parametrize("k", [8, 2])
def test_batch_matches_single(k):
    """Batch plan (plain and graph-replayed) against single lattices, at
    checkpoint intervals 8 and 2."""
    from paper_2212_05685_amd import kpm
    cfgs = [_cfg(9, 7, 2, M=40, ckpt_k=k), _cfg(16, 16, 4, M=40, ckpt_k=k),
            _cfg(5, 6, 0, M=40, ckpt_k=k, probes=(wl.ProbeSpec("unit", 60),))]
    singles, hs, abs_, Cs, rhos = [], [], [], [], []
    for cfg in cfgs:
        p, h, ab, C = _run_forward(cfg)
        singles.append((host(p.grand_potential(h, ab, C))[0], host(p.grand_potential_grad(h, ab, C))))
        hs.append(h)
        abs_.append(ab)
        Cs.append(C)
        rhos.append(torch.zeros_like(h))
    probs = [problem(c) for c in cfgs]
    plan = kpm.kpm_batch_create([q.lat for q in probs], [q.probes for q in probs], 40, kpm.KPM_FP64, k)
    try:
        for use_graph in (False, True, True):
            omega = torch.zeros(len(cfgs), dtype=torch.float64, device="cuda")
            for r in rhos:
                r.zero_()
            kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=use_graph)
            om = host(omega)
            for q in range(len(cfgs)):
                assert abs(om[q] - singles[q][0]) < 1e-12 * abs(singles[q][0])
                assert H.rel_err(host(rhos[q]), singles[q][1]) < 1e-12
    finally:
        kpm.kpm_batch_destroy(plan)


def test_autograd_matches_finite_differences():
    from paper_2212_05685_amd.autograd import GrandPotential
    cfg = _cfg(8, 8, 2, M=64, ckpt_k=8,
               probes=(wl.ProbeSpec("colored_z4", 1, 3, 4, 4, 0, 0, 0.5),
                       wl.ProbeSpec("dense_z4", 4, 4, weight=0.125)))
    p = problem(cfg)
    n, chi, dlt = theta_dev(cfg)
    n.requires_grad_(True)
    chi.requires_grad_(True)
    dlt.requires_grad_(True)
    om = GrandPotential.apply(n, chi, dlt, p)
    om.backward()
    gn, gc, gd = host(n.grad), host(chi.grad), host(dlt.grad)
    # central differences with (a, b) and C frozen at the base point
    h0 = p.build_H(n.detach(), chi.detach(), dlt.detach())
    ab = p.bounds(h0)
    C = p.coefficients(ab)

    def omega(n_, c_, d_):
        return host(p.grand_potential(p.build_H(n_, c_, d_), ab, C))[0]

    e = 1e-6
    nd, cd, dd = n.detach(), chi.detach(), dlt.detach()
    for i in [0, 9, 27, 63]:
        dn = torch.zeros_like(nd)
        dn[i] = e
        fd = (omega(nd + dn, cd, dd) - omega(nd - dn, cd, dd)) / (2 * e)
        assert abs(fd - gn[i]) < 1e-5 * max(1.0, abs(gn[i]))
        for d in range(4):
            for unit in (1.0, 1j):
                dc = torch.zeros_like(cd)
                dc[d, i] = e * unit
                fd = (omega(nd, cd + dc, dd) - omega(nd, cd - dc, dd)) / (2 * e)
                want = gc[d, i].real if unit == 1.0 else gc[d, i].imag
                assert abs(fd - want) < 1e-5 * max(1.0, abs(want))
                fd = (omega(nd, cd, dd + dc) - omega(nd, cd, dd - dc)) / (2 * e)
                want = gd[d, i].real if unit == 1.0 else gd[d, i].imag
                assert abs(fd - want) < 1e-5 * max(1.0, abs(want))
