"""Pins of the spin-polarised builder (oracle/sdw.py):

* at m = 0 with equal spins it is the singlet builder (itself pinned to the
  printed coefficients), entry by entry;
* the Gutzwiller hopping factor equals App. A's printed g^t_{i sigma}
  (oracle.gutzwiller.g_t_site) at m != 0, and g^z = g^xy at m = 0;
* the bond entries have the printed structure of eqs. Tij and Dij at m != 0:
  explicit terms -g^t t - J (g^z/4 conj(chi_s) + g^xy/2 conj(chi_-s)) (and the
  same for Delta) plus the Gutzwiller-factor term dW/dg^z dg^z/dchi_s, the
  latter from the printed g^z alone;
* the onsite entries are the density derivatives of W (finite differences),
  with no spin splitting at m = 0;
* W is invariant under the global spin flip (up <-> down, m -> -m);
* the VJP (sum_IJ rho_IJ dh_IJ/dtheta) against central finite differences of
  the linearisation built from the first-order stencil, at m != 0, and at
  m = 0 with equal spins against the singlet builder's VJP (itself pinned by
  finite differences) through the chain rule of the spin embedding.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import builder, gutzwiller, lattice, sdw

T_, TP, J, MU = wl.T_HOP, wl.TP_HOP, wl.J_EX, 0.3


def _theta(Lx, Ly, seed, m_amp):
    rng = np.random.default_rng(seed)
    N = Lx * Ly
    n = rng.uniform(0.8, 0.9, N)
    m = m_amp * rng.uniform(-1, 1, N)
    cu = 0.2 + 0.03 * (rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)))
    cd = 0.2 + 0.03 * (rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)))
    du = 0.1 * np.array([1, -1, 0, 0])[:, None] + 0.02 * (rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)))
    dd = 0.1 * np.array([1, -1, 0, 0])[:, None] + 0.02 * (rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)))
    return n / 2 + m, n / 2 - m, cu, cd, du, dd


def test_reduces_to_singlet_builder():
    Lx, Ly, nv = 6, 5, 2
    cfg = wl.Config("s", Lx, Ly, nv, 0.15, 8, (wl.ProbeSpec("unit", 1),), vortex=True, complex_noise=0.03)
    n, chi, dlt = wl.make_theta(cfg)
    ref = builder.build_stencil(Lx, Ly, nv, T_, TP, J, MU, n, chi, dlt)
    got = sdw.build_stencil_sdw(Lx, Ly, nv, T_, TP, J, MU, n / 2, n / 2, chi, chi, dlt, dlt)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def test_factors_match_printed_forms():
    rng = np.random.default_rng(1)
    nu = torch.tensor(rng.uniform(0.38, 0.48, 20))
    nd = torch.tensor(rng.uniform(0.38, 0.48, 20))
    delta, m, gtu, gtd, gxy, A = sdw.factors(nu, nd)
    assert np.allclose(gtu.numpy(), gutzwiller.g_t_site(delta.numpy(), m.numpy(), +1), rtol=1e-14)
    assert np.allclose(gtd.numpy(), gutzwiller.g_t_site(delta.numpy(), m.numpy(), -1), rtol=1e-14)
    assert np.allclose(gxy.numpy(), gutzwiller.g_sxy_site(delta.numpy(), m.numpy()), rtol=1e-14)


def _gz(nu_i, nd_i, nu_j, nd_j, cu, cd, du, dd):
    """Printed g^z_ij (moduli reading) for one bond, torch scalars."""
    def site(nu, nd):
        d = 1 - nu - nd
        m = (nu - nd) / 2
        A = 1 - d ** 2 + 4 * m ** 2
        return d, m, A, 2 * (1 - d) / A
    di, mi, Ai, gi = site(nu_i, nd_i)
    dj, mj, Aj, gj = site(nu_j, nd_j)
    X = 1 + 12 * (1 - di) * (1 - dj) / torch.sqrt(Ai * Aj)
    cb, db = (cu + cd) / 2, (du + dd) / 2
    b = 2 * (db.abs() ** 2 - cb.abs() ** 2)
    return gi * gj * (b - 4 * mi * mj * X ** 2) / (b - 4 * mi * mj), gi * gj, mi * mj


@pytest.mark.parametrize("d", [0, 1])
def test_bond_entries_have_printed_structure(d):
    Lx, Ly, nv = 5, 4, 2
    nu, nd, cu, cd, du, dd = _theta(Lx, Ly, 3, 0.05)
    st = sdw.build_stencil_sdw(Lx, Ly, nv, T_, TP, J, MU, nu, nd, cu, cd, du, dd)
    hop = lattice.hopping(Lx, Ly, nv, T_, TP)
    nbr = lattice.neighbour(Lx, Ly, d)
    fac = sdw.factors(torch.tensor(nu), torch.tensor(nd))
    gtu, gtd = fac[2].numpy(), fac[3].numpy()
    for i in (0, 7, 13):
        j = nbr[i]
        z = [torch.tensor(v, requires_grad=True) for v in (cu[d, i], cd[d, i], du[d, i], dd[d, i])]
        gz, gxy, mm = _gz(torch.tensor(nu[i]), torch.tensor(nd[i]), torch.tensor(nu[j]), torch.tensor(nd[j]), *z)
        gg = torch.autograd.grad(gz, z)                     # 2 dg^z/dconj(z)
        gz, gxy, mm = gz.detach(), gxy.detach(), mm.detach()
        szsz = mm - 0.25 * sum(abs(v) ** 2 for v in (cu[d, i], cd[d, i], du[d, i], dd[d, i]))
        dW_dgz = J * float(szsz)
        # dW/dchi_up (Wirtinger): printed explicit terms + [dW/dchi]_g
        T_up = (-gtu[i] * gtu[j] * hop[d, i] - J * (float(gz) / 4 * np.conj(cu[d, i]) + float(gxy) / 2 * np.conj(cd[d, i]))
                + dW_dgz * np.conj(gg[0].numpy()) / 2)
        assert abs(st[4 * d + 0, i] - T_up) < 1e-12
        T_dn = (-gtd[i] * gtd[j] * hop[d, i] - J * (float(gz) / 4 * np.conj(cd[d, i]) + float(gxy) / 2 * np.conj(cu[d, i]))
                + dW_dgz * np.conj(gg[1].numpy()) / 2)
        assert abs(st[4 * d + 3, i] - (-np.conj(T_dn))) < 1e-12
        # dW/dDelta_up (Wirtinger): -J (g^z/4 conj(D_up) + g^xy/2 conj(D_dn)) + [..]_g
        D_up = -J * (float(gz) / 4 * np.conj(du[d, i]) + float(gxy) / 2 * np.conj(dd[d, i])) + dW_dgz * np.conj(gg[2].numpy()) / 2
        assert abs(st[4 * d + 1, i] - (-np.conj(D_up))) < 1e-12
        D_dn = -J * (float(gz) / 4 * np.conj(dd[d, i]) + float(gxy) / 2 * np.conj(du[d, i])) + dW_dgz * np.conj(gg[3].numpy()) / 2
        assert abs(st[4 * d + 2, i] - (-D_dn)) < 1e-12


def test_onsite_entries_are_density_derivatives():
    """h_{i0,i0} = dW/dn_{i up} and h_{i1,i1} = -dW/dn_{i dn} (central finite
    differences of W, which carries the printed (1/2) s sum_j g^z J m_j and
    the factor terms); no spin splitting at m = 0."""
    Lx, Ly, nv = 5, 4, 2
    nu, nd, cu, cd, du, dd = _theta(Lx, Ly, 5, 0.05)
    st = sdw.build_stencil_sdw(Lx, Ly, nv, T_, TP, J, MU, nu, nd, cu, cd, du, dd)
    hop = torch.tensor(lattice.hopping(Lx, Ly, nv, T_, TP))
    nbr = torch.tensor(np.stack([lattice.neighbour(Lx, Ly, d) for d in range(4)]))
    t = lambda x: torch.tensor(x)

    def W(a, b):
        return float(sdw.energy_W_sdw(t(a), t(b), t(cu), t(cd), t(du), t(dd), hop, nbr, J, MU))

    eps = 1e-6
    for i in (0, 9, 19):
        e = np.zeros_like(nu)
        e[i] = eps
        dup = (W(nu + e, nd) - W(nu - e, nd)) / (2 * eps)
        ddn = (W(nu, nd + e) - W(nu, nd - e)) / (2 * eps)
        assert abs(st[16, i].real - dup) < 1e-7 * max(1.0, abs(dup))
        assert abs(st[17, i].real + ddn) < 1e-7 * max(1.0, abs(ddn))
    nu0 = (nu + nd) / 2
    st0 = sdw.build_stencil_sdw(Lx, Ly, nv, T_, TP, J, MU, nu0, nu0, cu, cu, du, du)
    assert np.max(np.abs(st0[16].real + st0[17].real)) < 1e-13


def test_spin_flip_invariance():
    Lx, Ly, nv = 5, 4, 2
    nu, nd, cu, cd, du, dd = _theta(Lx, Ly, 7, 0.05)
    hop = torch.tensor(lattice.hopping(Lx, Ly, nv, T_, TP))
    nbr = torch.tensor(np.stack([lattice.neighbour(Lx, Ly, d) for d in range(4)]))
    t = lambda x: torch.tensor(x)
    W1 = sdw.energy_W_sdw(t(nu), t(nd), t(cu), t(cd), t(du), t(dd), hop, nbr, J, MU)
    W2 = sdw.energy_W_sdw(t(nd), t(nu), t(cd), t(cu), t(dd), t(du), hop, nbr, J, MU)
    assert abs(float(W1) - float(W2)) < 1e-12 * abs(float(W1))


def _lin(args, rho, th):
    st = sdw.build_stencil_sdw(*args, *th)
    return (2 * (rho[:16] * st[:16]).real.sum() + (rho[16].real * st[16].real).sum()
            + (rho[17].real * st[17].real).sum())


def test_vjp_matches_finite_differences():
    Lx, Ly, nv = 4, 4, 2
    th = list(_theta(Lx, Ly, 9, 0.05))
    rng = np.random.default_rng(4)
    rho = rng.normal(size=(19, Lx * Ly)) + 1j * rng.normal(size=(19, Lx * Ly))
    args = (Lx, Ly, nv, T_, TP, J, MU)
    g = sdw.vjp_sdw(*args, *th, rho)
    e = 1e-6
    rng2 = np.random.default_rng(8)
    for trial in range(6):
        dirs = []
        for a in th:
            dz = rng2.normal(size=a.shape) + (1j * rng2.normal(size=a.shape) if np.iscomplexobj(a) else 0)
            dirs.append(dz)
        plus = [a + e * dz for a, dz in zip(th, dirs)]
        minus = [a - e * dz for a, dz in zip(th, dirs)]
        fd = (_lin(args, rho, plus) - _lin(args, rho, minus)) / (2 * e)
        an = sum(float(np.sum((np.conj(gk) * dz).real)) for gk, dz in zip(g, dirs))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (trial, fd, an)


def test_vjp_reduces_to_singlet():
    Lx, Ly, nv = 5, 4, 2
    cfg = wl.Config("s", Lx, Ly, nv, 0.15, 8, (wl.ProbeSpec("unit", 1),), vortex=True, complex_noise=0.03)
    n, chi, dlt = wl.make_theta(cfg)
    rng = np.random.default_rng(6)
    rho = rng.normal(size=(19, cfg.N)) + 1j * rng.normal(size=(19, cfg.N))
    rho[18] = 0.0                               # h_18 = 0 in the spin-polarised form
    args = (Lx, Ly, nv, T_, TP, J, MU)
    gn, gc, gd = builder.build_vjp(*args, n, chi, dlt, rho)
    gu, gdn, gcu, gcd, gdu, gdd = sdw.vjp_sdw(*args, n / 2, n / 2, chi, chi, dlt, dlt, rho)
    scale = max(np.max(np.abs(gn)), np.max(np.abs(gc)))
    assert np.max(np.abs(0.5 * (gu + gdn) - gn)) < 1e-11 * scale
    assert np.max(np.abs(gcu + gcd - gc)) < 1e-11 * scale
    assert np.max(np.abs(gdu + gdd - gd)) < 1e-11 * scale
