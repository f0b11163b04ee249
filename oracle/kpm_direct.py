"""O4: direct probing estimate of the density matrix (oracle; test
infrastructure only).

App. B expands the grand-potential density in Chebyshev polynomials of the
rescaled matrix, F_M(x) = sum_m C_m T_m(x), and estimates traces with probe
vectors.  Besides the adjoint route (the derivative of the probe-estimated
Omega, O2), the density matrix can be estimated directly from the expansion
of f' = n_F applied to each probe:

    rho_IJ = dOmega/dh_IJ ~= (1/a) sum_l w_l conj(r_{l,I}) [F_M'(H~) r_l]_J,

i.e. (1/a) [F_M'(H~) P]_JI with P = sum_l w_l r_l r_l^dag.  F_M' is the exact
derivative of the truncated, damped series, so for the complete set of unit
vectors (P = 1) both routes give (1/a) F_M'(H~)^T, the truncated rho of O1.

Steps, in this order:
1. D = coefficients of F_M' in the same basis (numpy's Chebyshev derivative);
2. y_l = sum_m D_m alpha_m with the recursion of App. B (eq. alpha);
3. rho on the stencil pairs (I, J): (1/a) sum_l w_l conj(r_{l,I}) y_{l,J};
   the two diagonal entries (i0, i0), (i1, i1) keep their real part (the
   diagonal of the Hermitian rho is real; for a finite probe set the
   estimate's imaginary part there is probing noise, and the stencil layout
   stores those entries as real);
4. Omega from the moments of the same recursion (eq. F_KPM).
"""
from __future__ import annotations

import numpy as np

from .kpm_plain import rescaled, stencil_pairs


def derivative_coefficients(C: np.ndarray) -> np.ndarray:
    """D with sum_k D_k T_k(x) = d/dx sum_m C_m T_m(x); len(D) = len(C)
    (the top entry is zero)."""
    D = np.zeros(len(C))
    d = np.polynomial.chebyshev.chebder(np.asarray(C, dtype=np.float64))
    D[:len(d)] = d
    return D


def direct_rho(Hs, a, b, probes, weights, C, Lx, Ly):
    """Steps 1-4 on probes (R x 2N).  Returns dict with rho [19, N], omega and
    y [R, 2N]."""
    Ht = rescaled(Hs, a, b)
    M = len(C)
    D = derivative_coefficients(C)
    R, dim = probes.shape
    I, J = stencil_pairs(Lx, Ly)
    rho = np.zeros(I.shape, dtype=np.complex128)
    ys = np.zeros((R, dim), dtype=np.complex128)
    omega = 0.0
    for ell in range(R):
        r = probes[ell]
        w = weights[ell]
        prev, cur = None, r.copy()
        y = D[0] * cur
        mom = [np.vdot(r, cur).real]
        for m in range(1, M):
            nxt = (Ht @ cur) if m == 1 else 2.0 * (Ht @ cur) - prev
            prev, cur = cur, nxt
            y = y + D[m] * cur
            mom.append(np.vdot(r, cur).real)
        omega += w * float(np.dot(C, mom))
        ys[ell] = y
        rho += w * np.conj(r[I]) * y[J]
    rho[16] = rho[16].real
    rho[17] = rho[17].real
    return {"rho": rho / a, "omega": omega, "y": ys}
