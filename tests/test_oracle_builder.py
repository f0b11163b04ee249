"""Pins for oracle/gutzwiller.py and oracle/builder.py.

* the App. A Gutzwiller factors at m = 0 equal the textbook values
  g_t = 2 delta/(1+delta), g_s = 4/(1+delta)^2 used in the uniform configs;
* the autograd coefficients equal the printed eq. Tij at m = 0 and the printed
  pairing magnitude (3/4) J g^s |Delta| (eq. Dij);
* the onsite term eps_i = dW/dn_i equals a central finite difference of W;
* the Nambu matrix is Hermitian and particle-hole symmetric,
  (sigma_y) h^* (sigma_y) = -h for spin-singlet BdG;
* a uniform zero-field state has the spectrum of the closed-form Bloch
  matrices (k-space, eq. Tij written out by hand);
* with zero pairing and exchange and n_v = 2 Ly flux quanta the up-spin block
  reduces to Harper's equation (textbook Hofstadter problem) per k_y;
* the builder VJP equals central differences of the linearised energy, and
  the chain dOmega*/dtheta of the exact grand potential equals central
  differences of Omega*(h(theta)) computed by dense diagonalisation.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import builder, chebyshev, dense, kspace, lattice
from oracle.gutzwiller import energy_W, g_sxy_site, g_t_site


def test_gutzwiller_m0_textbook():
    d = np.linspace(0.02, 0.4, 17)
    gt = g_t_site(d, 0.0, +1) * g_t_site(d, 0.0, +1)
    assert np.allclose(gt, 2 * d / (1 + d), rtol=0, atol=1e-15)
    assert np.allclose(g_t_site(d, 0.0, -1), g_t_site(d, 0.0, +1), atol=0)
    gs = g_sxy_site(d, 0.0) ** 2
    assert np.allclose(gs, 4 / (1 + d) ** 2, rtol=0, atol=1e-15)
    # nonzero m splits the spin species (App. A: (1 + d + 2 s m)/(1 + d - 2 s m))
    assert g_t_site(0.1, 0.05, +1) > g_t_site(0.1, 0.05, -1)


def _cfg(**kw):
    base = wl.Config("t", 5, 4, 2, 0.14, 16, (wl.ProbeSpec("unit", 4),), complex_noise=0.02, vortex=True)
    return wl.replace(base, **kw)


def _coefs(cfg):
    n, chi, dlt = wl.make_theta(cfg)
    nt, ct, dt = builder._torch_inputs(n, chi, dlt)
    eps, T, P = builder.coefficients_torch(nt, ct, dt, cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu)
    return n, chi, dlt, eps.detach().numpy(), T.detach().numpy(), P.detach().numpy()


def test_coefficients_match_printed_formulas():
    cfg = _cfg()
    n, chi, dlt, eps, T, P = _coefs(cfg)
    delta = 1 - n
    g = np.sqrt(2 * delta / (1 + delta))
    gs = 2 / (1 + delta)
    hop = lattice.hopping(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp)
    for d in range(4):
        j = lattice.neighbour(cfg.Lx, cfg.Ly, d)
        want = -g * g[j] * hop[d]
        if d < 2:
            want = want - 0.75 * cfg.J * gs * gs[j] * np.conj(chi[d])
            assert np.allclose(np.abs(P[d]), 0.75 * cfg.J * gs * gs[j] * np.abs(dlt[d]), atol=1e-15)
        else:
            assert np.all(P[d] == 0)
        assert np.allclose(T[d], want, atol=1e-15)


def test_onsite_is_finite_difference_of_W():
    cfg = _cfg()
    n, chi, dlt, eps, _, _ = _coefs(cfg)
    hop = torch.tensor(lattice.hopping(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp))
    nbr = torch.tensor(np.stack([lattice.neighbour(cfg.Lx, cfg.Ly, d) for d in range(4)]))
    ct, dt = torch.tensor(chi), torch.tensor(dlt)
    h = 1e-6
    for i in [0, 7, 19]:
        e = np.zeros_like(n)
        e[i] = h
        Wp = energy_W(torch.tensor(n + e), ct, dt, hop, nbr, cfg.J, cfg.mu).item()
        Wm = energy_W(torch.tensor(n - e), ct, dt, hop, nbr, cfg.J, cfg.mu).item()
        assert abs((Wp - Wm) / (2 * h) - eps[i]) < 1e-7


def test_hermitian_and_particle_hole():
    cfg = _cfg()
    n, chi, dlt = wl.make_theta(cfg)
    st = builder.build_stencil(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    H = builder.dense_from_stencil(st, cfg.Lx, cfg.Ly)
    assert np.allclose(H, H.conj().T, atol=0)
    N = cfg.N
    Sy = np.kron(np.eye(N), np.array([[0, -1j], [1j, 0]]))
    assert np.allclose(Sy @ H.conj() @ Sy, -H, atol=1e-15)
    E = np.linalg.eigvalsh(H)
    assert np.allclose(np.sort(E), np.sort(-E), atol=1e-12)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    assert np.allclose(Hs.toarray(), H, atol=0)


@pytest.mark.parametrize("L,dop", [(6, 0.125), (8, 0.2)])
def test_uniform_state_matches_bloch_closed_form(L, dop):
    cfg = wl.Config("u", L, L, 0, dop, 16, (wl.ProbeSpec("unit", 4),))
    n, chi, dlt = wl.make_theta(cfg)
    chi[2] = 0.03     # give the next-nearest-neighbour bonds a bond order as well
    chi[3] = -0.02
    st = builder.build_stencil(L, L, 0, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    E = np.linalg.eigvalsh(builder.dense_from_stencil(st, L, L))
    on, bl = kspace.uniform_blocks(dop, chi[:, 0], dlt[:, 0], cfg.t, cfg.tp, cfg.J, cfg.mu)
    assert np.allclose(E, kspace.spectrum(on, bl, L, L), atol=1e-12)
    # the stencil itself equals the closed-form blocks at every site
    on2, bl2 = kspace.blocks_from_stencil_site(st[:, 3])
    assert np.allclose(on2, on, atol=1e-13) and np.allclose(bl2, bl, atol=1e-14)


def test_harper_reduction():
    Lx, Ly = 6, 4
    nv = 2 * Ly                     # twist exp(i pi nv y/Ly) = 1: k_y is conserved
    dop, t, tp = 0.1, 1.0, -0.3
    N = Lx * Ly
    n = np.full(N, 1 - dop)
    z = np.zeros((4, N), dtype=np.complex128)
    st = builder.build_stencil(Lx, Ly, nv, t, tp, 0.0, 0.0, n, z, z)
    H = builder.dense_from_stencil(st, Lx, Ly)
    E = np.linalg.eigvalsh(H)
    g = 2 * dop / (1 + dop)
    eps = st[16, 0].real
    harper = []
    for ky in 2 * np.pi * np.arange(Ly) / Ly:
        A = np.zeros((Lx, Lx), dtype=np.complex128)
        for x in range(Lx):
            A[x, x] = eps - 2 * g * t * np.cos(ky - 2 * np.pi * x / Lx)
            hop = -g * t - 2 * g * tp * np.cos(ky - 2 * np.pi * (x + 0.5) / Lx)
            A[x, (x + 1) % Lx] += hop
            A[(x + 1) % Lx, x] += np.conj(hop)
        harper.append(np.linalg.eigvalsh(A))
    harper = np.concatenate(harper)
    want = np.sort(np.concatenate([harper, -harper]))
    assert np.allclose(E, want, atol=1e-12)


def test_vjp_matches_finite_differences():
    cfg = _cfg(Lx=4, Ly=4)
    n, chi, dlt = wl.make_theta(cfg)
    rng = np.random.default_rng(7)
    rho = rng.normal(size=(19, cfg.N)) + 1j * rng.normal(size=(19, cfg.N))
    rho[16:18] = rho[16:18].real
    args = (cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu)
    gn, gc, gd = builder.build_vjp(*args, n, chi, dlt, rho)

    def lin(n_, c_, d_):
        h = builder.build_stencil(*args, n_, c_, d_)
        return (2 * (rho[:16] * h[:16]).real.sum() + (rho[16].real * h[16].real).sum()
                + (rho[17].real * h[17].real).sum() + 2 * (rho[18] * h[18]).real.sum())

    e = 1e-6
    for i in [0, 5, 11]:
        dn = np.zeros_like(n)
        dn[i] = e
        assert abs((lin(n + dn, chi, dlt) - lin(n - dn, chi, dlt)) / (2 * e) - gn[i]) < 1e-6
        for d in [0, 1, 2, 3]:
            for unit, arr in ((1.0, "re"), (1j, "im")):
                dc = np.zeros_like(chi)
                dc[d, i] = e * unit
                fd = (lin(n, chi + dc, dlt) - lin(n, chi - dc, dlt)) / (2 * e)
                want = gc[d, i].real if arr == "re" else gc[d, i].imag
                assert abs(fd - want) < 1e-6
                fd = (lin(n, chi, dlt + dc) - lin(n, chi, dlt - dc)) / (2 * e)
                want = gd[d, i].real if arr == "re" else gd[d, i].imag
                assert abs(fd - want) < 1e-6


def test_exact_grand_potential_chain_rule():
    """dOmega*/dtheta = VJP(rho*) against central differences of eigh-based Omega*."""
    cfg = _cfg(Lx=3, Ly=4)
    T = 0.05
    n, chi, dlt = wl.make_theta(cfg)
    args = (cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu)

    def omega(n_, c_, d_):
        st = builder.build_stencil(*args, n_, c_, d_)
        return dense.exact(builder.dense_from_stencil(st, cfg.Lx, cfg.Ly), T)

    _, rho = omega(n, chi, dlt)
    rs = builder.stencil_from_dense(rho, cfg.Lx, cfg.Ly)
    gn, gc, gd = builder.build_vjp(*args, n, chi, dlt, rs)
    e = 1e-5
    for i in [1, 6]:
        dn = np.zeros_like(n)
        dn[i] = e
        fd = (omega(n + dn, chi, dlt)[0] - omega(n - dn, chi, dlt)[0]) / (2 * e)
        assert abs(fd - gn[i]) < 1e-7
        for d in [0, 1, 3]:
            dc = np.zeros_like(chi)
            dc[d, i] = e
            fd = (omega(n, chi + dc, dlt)[0] - omega(n, chi - dc, dlt)[0]) / (2 * e)
            assert abs(fd - gc[d, i].real) < 1e-7
            fd = (omega(n, chi, dlt + 1j * dc)[0] - omega(n, chi, dlt - 1j * dc)[0]) / (2 * e)
            assert abs(fd - gd[d, i].imag) < 1e-7
