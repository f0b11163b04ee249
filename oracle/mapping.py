"""rho -> order parameters (oracle; test infrastructure only).

Paper: Model and methods, order parameters delta_i, m_i (eqs. delta, mz),
chi_ij sigma = <c^dag_{i s} c_{j s}> (eq. chi), Delta_ij sigma =
sigma <c_{i s} c_{j -s}> (eq. pairing); App. B Nambu spinor d = (c_up, c^dag_dn)
and rho_IJ = <d^dag_I d_J>.  With rho Hermitian:

    n_{i up} = rho_{i1,i1}                 n_{i dn} = 1 - rho_{i2,i2}
    chi_ij up = rho_{i1,j1}                chi_ij dn = -conj(rho_{i2,j2})
    Delta_ij up = <c_{i up} c_{j dn}> = -conj(rho_{i1,j2})
    Delta_ij dn = -<c_{i dn} c_{j up}> = <c_{j up} c_{i dn}> = -rho_{i2,j1}

for the bond (i, j = i + d) stored at its tail site.
"""
from __future__ import annotations

import numpy as np


def order_parameters(rho: np.ndarray):
    """rho stencil [19, N] -> dict of n_up, n_dn [N] and chi/Delta per spin [4, N]."""
    n_up = rho[16].real.copy()
    n_dn = 1.0 - rho[17].real
    chi_up = np.stack([rho[4 * d + 0] for d in range(4)])
    chi_dn = np.stack([-np.conj(rho[4 * d + 3]) for d in range(4)])
    dlt_up = np.stack([-np.conj(rho[4 * d + 1]) for d in range(4)])
    dlt_dn = np.stack([-rho[4 * d + 2] for d in range(4)])
    return {"n_up": n_up, "n_dn": n_dn, "chi_up": chi_up, "chi_dn": chi_dn,
            "delta_up": dlt_up, "delta_dn": dlt_dn}
