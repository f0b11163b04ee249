"""Spin-polarised (collinear SDW) builder h(theta) = dW/drho (oracle; test
infrastructure only).

App. A at m_i != 0, magnetisation along z.  Per spin: n_{i sigma}, chi_{ij sigma}
= <c^dag_{i s} c_{j s}>, Delta_{ij sigma} = sigma <c_{i s} c_{j -s}>, with
delta_i = 1 - n_i, m_i = (n_{i up} - n_{i dn})/2 and the Gutzwiller factors of
App. A:

    g^t_{i s}  = sqrt( 2 delta (1 - delta) / (1 - delta^2 + 4 m^2)
                       * (1 + delta + 2 s m) / (1 + delta - 2 s m) ),
    g^xy_i     = 2 (1 - delta) / (1 - delta^2 + 4 m^2),
    X_ij       = 1 + 12 (1 - delta_i)(1 - delta_j)
                     / sqrt((1 - delta_i^2 + 4 m_i^2)(1 - delta_j^2 + 4 m_j^2)),
    g^z_ij     = g^xy_i g^xy_j [2(|Dbar|^2 - |chibar|^2) - 4 m_i m_j X_ij^2]
                               / [2(|Dbar|^2 - |chibar|^2) - 4 m_i m_j],

chibar = (chi_up + chi_dn)/2, Dbar = (Delta_up + Delta_dn)/2.

The paper prints only the derivatives of W (eqs. Tij, Dij, mu_i).  The energy
of H_renorm in the BdG Slater determinant, by Wick's theorem with only
opposite-spin pairing, is

    <S^z_i S^z_j>                  = m_i m_j - (1/4) sum_s (|chi_s|^2 + |Delta_s|^2),
    <(S^+_i S^-_j + S^-_i S^+_j)/2> = -Re(chi_up conj(chi_dn) + conj(Delta_up) Delta_dn),

so that

    W = - sum_bonds sum_s g^t_{i s} g^t_{j s} 2 Re(t_ij chi_{ij s})
        + J sum_nn [ g^z_ij <S^z S^z> + g^xy_ij <(S^+S^- + S^-S^+)/2> ]
        - mu sum_i (n_{i up} + n_{i dn}).

Its derivatives reproduce every explicitly printed term: dW/dchi_s gives
-g^t t - J (g^z/4 conj(chi_s) + g^xy/2 conj(chi_-s)) plus [dW/dchi]_g,
dW/dDelta* the same with Delta, and dW/dn_{i s} the term (1/2) s sum_j g^z J m_j
plus the Gutzwiller-factor terms.  At m = 0 with equal spins it is the
singlet W of ``gutzwiller.energy_W``.  The squares in g^z are read as moduli
(the factor must be real for complex bond variables).

h is the Wirtinger derivative of W as a function of rho_IJ = <d^dag_I d_J>,
d_i = (c_{i up}, c^dag_{i dn}):
    rho_{i0,j0} = chi_up,  rho_{i1,j1} = -conj(chi_dn),
    rho_{i0,j1} = -conj(Delta_up),  rho_{i1,j0} = -Delta_dn,
    rho_{i0,i0} = n_up,  rho_{i1,i1} = 1 - n_dn,
hence (torch's gradient of a real W w.r.t. a complex z is 2 dW/dconj z)
    h_{i0,j0} = conj(g_chi_up)/2,  h_{i1,j1} = -g_chi_dn/2,
    h_{i0,j1} = -g_Delta_up/2,     h_{i1,j0} = -conj(g_Delta_dn)/2,
    h_{i0,i0} = dW/dn_up,          h_{i1,i1} = -dW/dn_dn,   h_{i0,i1} = 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lattice


def factors(n_up, n_dn):
    """(delta, m, g^t_up, g^t_dn, g^xy, A) per site, A = 1 - delta^2 + 4 m^2."""
    n = n_up + n_dn
    delta = 1.0 - n
    m = 0.5 * (n_up - n_dn)
    A = 1.0 - delta ** 2 + 4.0 * m ** 2
    base = 2.0 * delta * (1.0 - delta) / A
    gt_up = torch.sqrt(base * (1.0 + delta + 2.0 * m) / (1.0 + delta - 2.0 * m))
    gt_dn = torch.sqrt(base * (1.0 + delta - 2.0 * m) / (1.0 + delta + 2.0 * m))
    gxy = 2.0 * (1.0 - delta) / A
    return delta, m, gt_up, gt_dn, gxy, A


def energy_W_sdw(n_up, n_dn, chi_up, chi_dn, dlt_up, dlt_dn, hop, nbr, J, mu):
    """W above (torch, fp64).  chi/dlt [4, N] complex per direction
    (+x, +y, +x+y, +x-y), hop [4, N] bare Peierls hoppings, nbr [4, N]."""
    delta, m, gtu, gtd, gxy, A = factors(n_up, n_dn)
    W = -mu * (n_up + n_dn).sum()
    for d in range(4):
        j = nbr[d]
        hopping = gtu * gtu[j] * 2.0 * (hop[d] * chi_up[d]).real + gtd * gtd[j] * 2.0 * (hop[d] * chi_dn[d]).real
        W = W - hopping.sum()
        if d < 2:
            cu, cd, du, dd = chi_up[d], chi_dn[d], dlt_up[d], dlt_dn[d]
            cbar, dbar = 0.5 * (cu + cd), 0.5 * (du + dd)
            sq = lambda z: z.real ** 2 + z.imag ** 2
            X = 1.0 + 12.0 * (1.0 - delta) * (1.0 - delta[j]) / torch.sqrt(A * A[j])
            mm = m * m[j]
            base = 2.0 * (sq(dbar) - sq(cbar))
            gz = gxy * gxy[j] * (base - 4.0 * mm * X ** 2) / (base - 4.0 * mm)
            szsz = mm - 0.25 * (sq(cu) + sq(cd) + sq(du) + sq(dd))
            sxy = -((cu * cd.conj()).real + (du.conj() * dd).real)
            W = W + J * (gz * szsz + gxy * gxy[j] * sxy).sum()
    return W


def build_stencil_sdw(Lx, Ly, n_v, t, tp, J, mu, n_up, n_dn, chi_up, chi_dn, dlt_up, dlt_dn):
    """h on the [19, N] stencil (numpy complex128) by autograd of W."""
    def leaf(x, dt):
        return torch.tensor(np.asarray(x, dtype=dt), requires_grad=True)

    nu, nd = leaf(n_up, np.float64), leaf(n_dn, np.float64)
    cu, cd = leaf(chi_up, np.complex128), leaf(chi_dn, np.complex128)
    du, dd = leaf(dlt_up, np.complex128), leaf(dlt_dn, np.complex128)
    hop = torch.tensor(lattice.hopping(Lx, Ly, n_v, t, tp))
    nbr = torch.tensor(np.stack([lattice.neighbour(Lx, Ly, d) for d in range(4)]))
    W = energy_W_sdw(nu, nd, cu, cd, du, dd, hop, nbr, J, mu)
    g = torch.autograd.grad(W, (nu, nd, cu, cd, du, dd))
    gnu, gnd, gcu, gcd, gdu, gdd = (x.detach().numpy() for x in g)
    N = Lx * Ly
    st = np.zeros((19, N), dtype=np.complex128)
    for d in range(4):
        st[4 * d + 0] = np.conj(gcu[d]) / 2.0
        st[4 * d + 1] = -gdu[d] / 2.0
        st[4 * d + 2] = -np.conj(gdd[d]) / 2.0
        st[4 * d + 3] = -gcd[d] / 2.0
    st[16] = gnu
    st[17] = -gnd
    return st


def vjp_sdw(Lx, Ly, n_v, t, tp, J, mu, n_up, n_dn, chi_up, chi_dn, dlt_up, dlt_dn, rho):
    """dOmega/dtheta = sum_IJ rho_IJ dh_IJ/dtheta over both halves of the h of
    ``build_stencil_sdw`` (kpm_build_H_sdw_vjp).  With h and rho Hermitian the
    sum is the linearisation
        S = sum_fwd 2 Re(rho_e h_e) + Re(rho_16) h_16 + Re(rho_17) h_17
    (h_18 = 0), differentiated by autograd through the first derivatives of W
    (second derivatives of W).  Complex gradients: dOmega/dRe z + i dOmega/dIm z.
    Returns (d n_up, d n_dn, d chi_up, d chi_dn, d delta_up, d delta_dn)."""
    def leaf(x, dt):
        return torch.tensor(np.asarray(x, dtype=dt), requires_grad=True)

    leaves = (leaf(n_up, np.float64), leaf(n_dn, np.float64), leaf(chi_up, np.complex128),
              leaf(chi_dn, np.complex128), leaf(dlt_up, np.complex128), leaf(dlt_dn, np.complex128))
    hop = torch.tensor(lattice.hopping(Lx, Ly, n_v, t, tp))
    nbr = torch.tensor(np.stack([lattice.neighbour(Lx, Ly, d) for d in range(4)]))
    W = energy_W_sdw(*leaves, hop, nbr, J, mu)
    gnu, gnd, gcu, gcd, gdu, gdd = torch.autograd.grad(W, leaves, create_graph=True)
    r = torch.tensor(np.asarray(rho, dtype=np.complex128))
    S = 0.0
    for d in range(4):
        ents = (gcu[d].conj() / 2.0, -gdu[d] / 2.0, -gdd[d].conj() / 2.0, -gcd[d] / 2.0)
        for q, h_e in enumerate(ents):
            S = S + 2.0 * (r[4 * d + q] * h_e).real.sum()
    S = S + (r[16].real * gnu).sum() + (r[17].real * (-gnd)).sum()
    g = torch.autograd.grad(S, leaves, allow_unused=True)
    return tuple((torch.zeros_like(x) if gi is None else gi).detach().numpy() for gi, x in zip(g, leaves))


def order_parameters_sdw(rho):
    """Per-spin theta from a [19, N] density-matrix stencil (the inverse of
    the rho entries listed above)."""
    return {"n_up": rho[16].real.copy(), "n_dn": 1.0 - rho[17].real,
            "chi_up": np.stack([rho[4 * d] for d in range(4)]),
            "chi_dn": np.stack([-np.conj(rho[4 * d + 3]) for d in range(4)]),
            "delta_up": np.stack([-np.conj(rho[4 * d + 1]) for d in range(4)]),
            "delta_dn": np.stack([-rho[4 * d + 2] for d in range(4)])}
