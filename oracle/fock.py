"""Brute-force many-body check for a handful of fermion modes (oracle).

Paper App. B: for H = sum_IJ h_IJ d^dag_I d_J with canonical fermions d_I, the
grand potential is Omega = -T log Tr e^{-H/T} and rho_IJ = <d^dag_I d_J>.
Here both are computed literally in the 2^D-dimensional Fock space (Jordan-
Wigner matrices, dense matrix exponential), with no single-particle shortcut,
to pin the closed forms used by ``dense.exact``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def annihilators(D: int):
    """Jordan-Wigner matrices of d_0 .. d_{D-1} on 2^D states."""
    Z = np.diag([1.0, -1.0])
    I2 = np.eye(2)
    a = np.array([[0.0, 1.0], [0.0, 0.0]])   # |1> -> |0>
    ops = []
    for k in range(D):
        m = np.array([[1.0]])
        for q in range(D):
            m = np.kron(m, Z if q < k else (a if q == k else I2))
        ops.append(m)
    return ops


def grand_potential_and_rho(h: np.ndarray, T: float):
    D = h.shape[0]
    d = annihilators(D)
    H = np.zeros((2 ** D, 2 ** D), dtype=np.complex128)
    for I in range(D):
        for J in range(D):
            if h[I, J] != 0:
                H += h[I, J] * (d[I].T @ d[J])
    E0 = np.linalg.eigvalsh(H).min()
    rhoM = sla.expm(-(H - E0 * np.eye(2 ** D)) / T)
    Z = np.trace(rhoM).real
    omega = E0 - T * np.log(Z)
    rho = np.zeros((D, D), dtype=np.complex128)
    for I in range(D):
        for J in range(D):
            rho[I, J] = np.trace(rhoM @ (d[I].T @ d[J])) / Z
    return float(omega), rho
