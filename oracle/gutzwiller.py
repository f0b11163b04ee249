"""Gutzwiller factors and the variational energy W (oracle; test infrastructure).

Paper App. A ("Renormalized mean-field theory"):

* on-site hopping factor g^t_{i sigma} = sqrt( 2 delta (1 - delta) / (1 - delta^2
  + 4 m^2) * (1 + delta + 2 sigma m) / (1 + delta - 2 sigma m) ), bond factor
  g^t_{ij sigma} = g^t_{i sigma} g^t_{j sigma};
* transverse exchange factor g^{s,xy}_i = 2 (1 - delta) / (1 - delta^2 + 4 m^2),
  g^{s,xy}_{ij} = g^{s,xy}_i g^{s,xy}_j; at m = 0 the longitudinal factor
  g^{s,z}_{ij} equals g^{s,xy}_{ij}.
* W = <H_renorm> - lambda(<Psi|Psi> - 1) - mu (sum_i n_i - N_e), whose
  derivatives define the effective TB-BdG coefficients (eqs. Tij, Dij, mu_i).

The paper prints only the derivatives of W.  At m_i = 0 and for spin-singlet
order parameters (chi_up = chi_dn = chi, Delta_up = Delta_dn = Delta) the
energy whose derivatives reproduce eqs. Tij / Dij / mu_i is

    W = - sum_{bonds b=(ij)} sum_sigma g^t_ij (t_ij chi_ij + c.c.)
        - (3/2) J sum_{nn bonds} g^s_ij (|chi_ij|^2 + |Delta_ij|^2)
        - mu sum_i n_i                                   (+ const),

with n_i = n_{i up} + n_{i dn} = 1 - delta_i and every undirected bond counted
once.  The spin sum of the hopping term gives a factor 2.
"""
from __future__ import annotations

import numpy as np
import torch


def g_t_site(delta, m, sigma):
    """g^t_{i sigma} (App. A) for arrays delta, m and sigma = +1 / -1."""
    delta = np.asarray(delta, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    num = 2.0 * delta * (1.0 - delta)
    den = 1.0 - delta ** 2 + 4.0 * m ** 2
    ratio = (1.0 + delta + 2.0 * sigma * m) / (1.0 + delta - 2.0 * sigma * m)
    return np.sqrt(num / den * ratio)


def g_sxy_site(delta, m):
    """g^{s,xy}_i (App. A)."""
    delta = np.asarray(delta, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    return 2.0 * (1.0 - delta) / (1.0 - delta ** 2 + 4.0 * m ** 2)


def energy_W(n, chi, dlt, hop, nbr, J, mu):
    """Reconstructed W at m = 0, singlet order parameters (torch, fp64).

    n   : [N] float64 total electron density n_i = 1 - delta_i
    chi : [4, N] complex128 bond order <c^dag_{i s} c_{j s}> per spin, j = i + d
    dlt : [4, N] complex128 singlet pairing <c_{i up} c_{j dn}> on bond (i, i+d)
    hop : [4, N] complex128 bare Peierls hoppings t_ij
    nbr : [4, N] int64 head-site index j for bond (i, d)
    Only d = 0, 1 (nearest neighbours) carry exchange J; the paper has no
    next-nearest-neighbour exchange or pairing, so dlt[2:] does not enter W.
    """
    delta = 1.0 - n
    g = torch.sqrt(2.0 * delta / (1.0 + delta))          # g^t_i at m = 0
    gs = 2.0 / (1.0 + delta)                             # g^{s,xy}_i at m = 0
    W = -mu * n.sum()
    for d in range(4):
        j = nbr[d]
        gt_ij = g * g[j]
        # sum over both spins of (t_ij chi_ij + c.c.) = 4 Re(t_ij chi_ij)
        W = W - (gt_ij * 4.0 * (hop[d] * chi[d]).real).sum()
        if d < 2:
            gs_ij = gs * gs[j]
            # |z|^2 written as re^2 + im^2: abs() has no usable derivative at z = 0
            sq = chi[d].real ** 2 + chi[d].imag ** 2 + dlt[d].real ** 2 + dlt[d].imag ** 2
            W = W - 1.5 * J * (gs_ij * sq).sum()
    return W
