"""Pins for the oracle's KPM functions (chebyshev, kpm_plain O2, dense O1,
kspace O3, fock, probes, mapping) against closed forms, independent
derivations, published test vectors and brute force.

* Jackson damping: the closed form equals Weisse et al.'s construction as the
  autocorrelation of a_v ~ sin(pi (v+1)/(M+1)), normalised, and g_0 = 1;
* coefficients: the undamped series reproduces f(a x + b) pointwise, the odd
  part of f is e/2 so c_1 = a/4 and c_odd>1 = 0 at b = 0, and doubling the
  quadrature changes nothing;
* Gershgorin bounds: the discs of hand-built matrices worked out by hand
  (including a tight case whose rescaled spectrum is exactly -+0.995), and
  the stencil-built sparse form equals the dense rows and encloses eigh;
* moments: mu_0 = sum_l w_l |r_l|^2; exact-trace moments equal
  sum_n cos(m arccos x_n) from eigh; odd moments vanish for particle-hole
  symmetric h (b = 0);
* O2 (paper's recursion + adjoint) equals O1 (dense truncated function,
  Daleckii-Krein for probes); dense dE/dh is Hermitian;
* per site rho_{i1,i1} + rho_{i2,i2} = g_1 = cos(pi/(M+1)) for the
  exact-trace truncated result, = 1 for the Fermi result;
* finite differences of Omega_M (O2) w.r.t. a Hermitian bond pair equal
  2 Re rho and -2 Im rho;
* Omega_M -> Omega*, rho_M -> rho* as M grows, at the Jackson rate 1/M^2;
* Fock-space brute force equals Omega* = sum f(E_n) and rho* = n_F(h)^T;
* k-space rho of the uniform state equals dense rho*;
* SplitMix64 equals its published outputs; colored probes of one draw
  partition the identity.
"""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import builder, chebyshev, dense, fock, kpm_plain, kspace, mapping, probes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_jackson_closed_form_is_autocorrelation():
    for M in [2, 7, 64, 300]:
        v = np.arange(M)
        a = np.sin(np.pi * (v + 1) / (M + 1))
        a /= np.sqrt(np.sum(a * a))
        auto = np.array([np.dot(a[: M - n], a[n:]) for n in range(M)])
        assert np.allclose(chebyshev.jackson(M), auto, atol=1e-14)
        assert abs(chebyshev.jackson(M)[0] - 1.0) < 1e-14


def test_coefficients_reproduce_f_and_odd_part():
    T, a, b = 0.05, 2.7, 0.0
    M = 1500
    C = chebyshev.kpm_coefficients(M, T, a, b, damping=False)
    xs = np.linspace(-0.97, 0.97, 41)
    assert np.allclose(chebyshev.series(C, xs), chebyshev.fermi_energy_density(a * xs + b, T), atol=1e-12)
    # f(e) - f(-e) = e  =>  c_1 = a/4 (C_1 = 2 c_1), every other odd coefficient 0
    assert abs(C[1] - a / 2) < 1e-14
    # rounding of a K-term sum of |F| ~ a values: ~sqrt(K) eps a
    assert np.max(np.abs(C[3::2])) < 1e-13
    Cj = chebyshev.kpm_coefficients(M, T, a, b)
    assert abs(Cj[1] - np.cos(np.pi / (M + 1)) * a / 2) < 1e-14


def test_gershgorin_hand_built_discs():
    """Gershgorin discs of a hand-built 3 x 3 Hermitian matrix, worked out by
    hand: row 0 has centre 1 and radius |0.3i| + |0.2| = 0.5, row 1 centre -2
    and radius 0.3 + |0.1 + 0.1i| = 0.3 + 0.1 sqrt 2, row 2 centre 0.5 and
    radius 0.2 + 0.1 sqrt 2.  So Emin = -2.3 - 0.1 sqrt 2 (row 1) and
    Emax = 1.5 (row 0).  A radius that counted |h_II|, a sign slip on the
    centre or a column sum of the modulus-free entries each moves a bound."""
    s2 = np.sqrt(2.0)
    H = np.array([[1.0, 0.3j, 0.2],
                  [-0.3j, -2.0, 0.1 + 0.1j],
                  [0.2, 0.1 - 0.1j, 0.5]])
    Emin, Emax = chebyshev.gershgorin(H)
    assert abs(Emin - (-2.3 - 0.1 * s2)) < 1e-15
    assert abs(Emax - 1.5) < 1e-15
    import scipy.sparse as sp
    assert chebyshev.gershgorin_sparse(sp.csr_matrix(H)) == (Emin, Emax)
    # a diagonal matrix: the discs are points, the bounds the extreme entries
    assert chebyshev.gershgorin(np.diag([0.25, -3.0, 7.5])) == (-3.0, 7.5)
    # [[0, 1], [1, 0]] has eigenvalues -1, 1 and the discs are [-1, 1]: tight,
    # and the rescale maps them to -+0.995 (pad 0.01)
    P = np.array([[0.0, 1.0], [1.0, 0.0]])
    a, b = chebyshev.rescale(*chebyshev.gershgorin(P))
    assert abs(a - 2.0 / 1.99) < 1e-15 and b == 0.0
    assert np.allclose(np.linalg.eigvalsh((P - b * np.eye(2)) / a), [-0.995, 0.995], atol=1e-15)
    # a shifted spectrum: diag(3, 5) with coupling 1 -> discs [2, 4] and [4, 6]
    S = np.array([[3.0, 1.0], [1.0, 5.0]])
    assert chebyshev.gershgorin(S) == (2.0, 6.0)
    a, b = chebyshev.rescale(2.0, 6.0)
    assert abs(a - 4.0 / 1.99) < 1e-15 and b == 4.0


def test_gershgorin_of_stencil_matches_dense_rows():
    """The stencil-built sparse h gives the same bounds as its dense form,
    and those enclose the spectrum."""
    cfg = wl.C1()
    n, chi, dlt = wl.make_theta(cfg)
    st = builder.build_stencil(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    Hd = builder.dense_from_stencil(st, cfg.Lx, cfg.Ly)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    lo, hi = chebyshev.gershgorin(Hd)
    lo_s, hi_s = chebyshev.gershgorin_sparse(Hs)
    assert abs(lo - lo_s) < 1e-13 and abs(hi - hi_s) < 1e-13
    E = np.linalg.eigvalsh(Hd)
    assert lo <= E[0] and E[-1] <= hi


def test_quadrature_doubling_converged():
    M, T, a, b = 512, 0.005, 2.6, 0.013
    K = chebyshev.quad_nodes(M)
    C1 = chebyshev.kpm_coefficients(M, T, a, b, K=K)
    C2 = chebyshev.kpm_coefficients(M, T, a, b, K=2 * K)
    assert np.max(np.abs(C1 - C2)) < 1e-15 * np.max(np.abs(C1)) * 10


def test_splitmix64_published_outputs():
    for line in open(os.path.join(GOLDEN, "splitmix64.txt")):
        if line.startswith("#") or not line.strip():
            continue
        c, h = line.split()
        assert probes.splitmix64(0, int(c)) == int(h, 16)


def test_colored_probes_partition_identity():
    g = probes.ProbeGroup(probes.COLORED_Z4, 2, seed=11, px=3, py=2, split_nambu=1, weight=0.5)
    R, w = probes.probe_set([g], 7, 5)
    P = (R.T * w) @ R.conj()
    assert np.allclose(P.diagonal(), 1.0, atol=0)
    assert set(np.round(R[np.abs(R) > 0], 12).tolist()) <= {1, 1j, -1, -1j}


def _small(L=4, dop=0.125, M=64, nv=0, T=0.005, **kw):
    cfg = wl.Config("s", L, L, nv, dop, M, (wl.ProbeSpec("unit", 2 * L * L),), noise=0.01, T=T, **kw)
    n, chi, dlt = wl.make_theta(cfg)
    st = builder.build_stencil(L, L, nv, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    H = builder.dense_from_stencil(st, L, L)
    Emin, Emax = chebyshev.gershgorin(H)
    a, b = chebyshev.rescale(Emin, Emax)
    C = chebyshev.kpm_coefficients(M, T, a, b)
    return cfg, st, H, a, b, C


def test_exact_trace_moments_and_particle_hole():
    cfg, st, H, a, b, C = _small(L=4, M=48)
    assert b == 0.0          # symmetric Gershgorin interval for a singlet BdG matrix
    D = H.shape[0]
    R, w = probes.probe_set([probes.ProbeGroup(probes.UNIT, D)], 4, 4)
    out = kpm_plain.plain_kpm(builder.sparse_from_stencil(st, 4, 4), a, b, R, w, C, 4, 4, full=True)
    mu = out["mu"].sum(axis=0)
    assert abs(mu[0] - D) < 1e-12
    ref = dense.exact_trace_moments(H, len(C), a, b)
    assert np.allclose(mu, ref, atol=1e-10)
    assert np.max(np.abs(mu[1::2])) < 1e-10
    assert np.max(np.abs(out["mu_imag"])) < 1e-12
    # O2 adjoint == O1 dense truncated function
    om, rho = dense.truncated(H, C, a, b)
    assert abs(out["omega"] - om) < 1e-11 * abs(om)
    assert np.allclose(out["rho_full"], rho, atol=1e-12)
    assert np.allclose(out["rho_full"], out["rho_full"].conj().T, atol=1e-13)
    rs = out["rho"]
    assert np.allclose(rs, builder.stencil_from_dense(rho, 4, 4), atol=1e-12)
    g1 = np.cos(np.pi / (len(C) + 1))
    assert np.allclose(rs[16].real + rs[17].real, g1, atol=1e-12)


@pytest.mark.parametrize("kind", ["dense", "colored"])
def test_probe_adjoint_equals_daleckii_krein(kind):
    cfg, st, H, a, b, C = _small(L=4, M=40, nv=2, vortex=True, complex_noise=0.03)
    if kind == "dense":
        grp = [probes.ProbeGroup(probes.DENSE_Z4, 5, seed=3, weight=0.2)]
    else:
        grp = [probes.ProbeGroup(probes.COLORED_Z4, 1, seed=5, px=2, py=2, split_nambu=0, weight=1.0)]
    R, w = probes.probe_set(grp, 4, 4)
    out = kpm_plain.plain_kpm(builder.sparse_from_stencil(st, 4, 4), a, b, R, w, C, 4, 4, full=True)
    om, G = dense.probe_estimator(H, C, a, b, R, w)
    assert abs(out["omega"] - om) < 1e-11 * abs(om)
    assert np.allclose(out["rho_full"], G, atol=1e-11)
    assert np.allclose(G, G.conj().T, atol=1e-12)
    assert np.allclose(out["mu"][:, 0], (np.abs(R) ** 2).sum(axis=1), atol=1e-13)


def test_finite_difference_of_omega_M():
    cfg, st, H, a, b, C = _small(L=3, M=32, nv=2, vortex=True, complex_noise=0.03)
    grp = [probes.ProbeGroup(probes.DENSE_Z4, 3, seed=9, weight=1 / 3)]
    R, w = probes.probe_set(grp, 3, 3)
    out = kpm_plain.plain_kpm(builder.sparse_from_stencil(st, 3, 3), a, b, R, w, C, 3, 3)
    rho = out["rho"]
    e = 1e-6
    for ent, i in [(0, 0), (5, 4), (13, 8), (18, 2)]:
        for unit in (1.0, 1j):
            sp = st.copy()
            sp[ent, i] += e * unit
            sm = st.copy()
            sm[ent, i] -= e * unit
            op = kpm_plain.plain_kpm(builder.sparse_from_stencil(sp, 3, 3), a, b, R, w, C, 3, 3, want_grad=False)
            om = kpm_plain.plain_kpm(builder.sparse_from_stencil(sm, 3, 3), a, b, R, w, C, 3, 3, want_grad=False)
            fd = (op["omega"] - om["omega"]) / (2 * e)
            want = 2 * rho[ent, i].real if unit == 1.0 else -2 * rho[ent, i].imag
            assert abs(fd - want) < 1e-7


def test_truncated_converges_to_fermi():
    cfg, st, H, a, b, C = _small(L=4, M=16, T=0.08)
    om_star, rho_star = dense.exact(H, 0.08)
    errs = []
    for M in [64, 128, 256, 512]:
        Cm = chebyshev.kpm_coefficients(M, 0.08, a, b)
        om, rho = dense.truncated(H, Cm, a, b)
        errs.append((abs(om - om_star), np.max(np.abs(rho - rho_star))))
    # the Jackson kernel broadens by ~pi/M, so both errors fall as 1/M^2
    for k in range(1, 3):
        assert 3.6 < errs[k][0] / errs[k + 1][0] < 4.4
        assert 3.6 < errs[k][1] / errs[k + 1][1] < 4.4
    assert np.allclose(rho_star.diagonal()[0::2] + rho_star.diagonal()[1::2], 1.0, atol=1e-12)


def test_fock_brute_force():
    rng = np.random.default_rng(3)
    D = 6
    X = rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D))
    h = 0.5 * (X + X.conj().T)
    T = 0.4
    om_b, rho_b = fock.grand_potential_and_rho(h, T)
    om, rho = dense.exact(h, T)
    assert abs(om_b - om) < 1e-10
    assert np.allclose(rho_b, rho, atol=1e-10)


def test_kspace_rho_equals_dense():
    L, dop, T = 6, 0.15, 0.05
    cfg = wl.Config("u", L, L, 0, dop, 16, (wl.ProbeSpec("unit", 4),), T=T)
    n, chi, dlt = wl.make_theta(cfg)
    st = builder.build_stencil(L, L, 0, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    H = builder.dense_from_stencil(st, L, L)
    om, rho = dense.exact(H, T)
    on, bl = kspace.uniform_blocks(dop, chi[:, 0], dlt[:, 0], cfg.t, cfg.tp, cfg.J, cfg.mu)
    om_k, site = kspace.exact_omega_rho_site(on, bl, L, L, T)
    assert abs(om - om_k) < 1e-10 * abs(om)
    rs = builder.stencil_from_dense(rho, L, L)
    assert np.allclose(rs, site[:, None], atol=1e-12)
    # the chemical potential table gives the requested doping (n = 1 - delta)
    op = mapping.order_parameters(rs)
    n_site = op["n_up"] + op["n_dn"]
    Lbig = 64
    assert abs(kspace.density(on, bl, Lbig, Lbig, T) - (1 - dop)) < 2e-3
    assert np.allclose(n_site, n_site[0], atol=1e-12)
